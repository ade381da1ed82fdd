"""Pins of the phase-field transport, momentum predictor and Runge-Kutta
substep oracle (oracle/flow.c) against what the mathematics fixes: exact
conservation, closed forms of the discrete operators on Fourier modes,
exact stationary states, the continuum limit at second order (the ACDI
equilibrium profile, the Taylor-Green vortex, the regularization term of a
profile whose flux has a closed form), the curvature of spheres and
cylinders, the Laplace pressure jump of a static drop, and the third-order
accuracy of the Runge-Kutta coefficients.  No GPU."""
import math

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests import manufactured as MF


def grid(orc, nx, ny, nz, lx, ly, lz, bc=(0, 0, 0), zf=None):
    return orc.Grid(nx, ny, nz, lx, ly, W.zf_uniform(nz, lz) if zf is None else zf, *bc)


def centres(n, L):
    return (np.arange(n) + 0.5) * (L / n)


def vol(g):
    dzf = np.diff(g.zf)
    return (g.lx / g.nx) * (g.ly / g.ny) * dzf[:, None, None] * np.ones(g.shape)


def smooth_phi(rng, g):
    """A smooth field in (0.02, 0.98): a few random low modes."""
    x, y = centres(g.nx, g.lx), centres(g.ny, g.ly)
    z = 0.5 * (g.zf[:-1] + g.zf[1:])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    s = np.zeros(g.shape)
    for _ in range(4):
        kx, ky, kz = rng.integers(1, 3, 3)
        s += rng.normal() * np.cos(2 * math.pi * (kx * X / g.lx + ky * Y / g.ly) + kz * Z + rng.uniform(0, 6))
    return 0.5 + 0.48 * np.tanh(s)


BCS = [(0, 0, 0), (0, 0, 1), (1, 0, 1), (0, 1, 0), (1, 1, 1)]


# ------------------------------------------------------------------ ACDI

@pytest.mark.parametrize("bc", BCS)
def test_acdi_conserves_phase_volume(orc, bc):
    rng = np.random.default_rng(7)
    g = grid(orc, 12, 10, 8, 1.2, 1.0, 1.0, bc, zf=W.zf_tanh(8, 1.0, 1.5))
    phi = smooth_phi(rng, g)
    u, v, w = (rng.uniform(-1, 1, g.shape) for _ in range(3))
    fl = orc.flow_params(gamma=1.3, eps=0.08)
    r = orc.acdi_rhs(g, fl, phi, u, v, w)
    s = (r * vol(g)).sum()
    assert abs(s) <= 1e-13 * (np.abs(r) * vol(g)).sum()
    assert np.abs(r).max() > 1e-3


@pytest.mark.parametrize("bc", BCS)
def test_acdi_constant_phase_in_solenoidal_flow_is_steady(orc, bc):
    rng = np.random.default_rng(3)
    gs = W.GridSpec(12, 10, 8, 1.2, 1.0, W.zf_tanh(8, 1.0, 1.2), *bc)
    g = orc.Grid.from_workload(gs)
    u, v, w = MF.divfree_field(rng, gs)
    phi = np.full(g.shape, 0.37)
    r = orc.acdi_rhs(g, orc.flow_params(gamma=2.0, eps=0.1), phi, u, v, w)
    assert np.abs(r).max() <= 1e-13 * max(np.abs(u).max(), 1.0) * 12 / 1.2


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_acdi_advection_of_a_fourier_mode(orc, axis):
    """Gamma = 0, uniform velocity U along one axis, phi = 1/2 + b sin(k x):
    the centred flux difference is -U b k cos(k x) sin(k h)/(k h) exactly."""
    n, L, U, b, m = 16, 2.0, 0.7, 0.3, 3
    g = grid(orc, n, n, n, L, L, L)
    xc = centres(n, L)
    k = 2 * math.pi * m / L
    shape = [1, 1, 1]
    shape[2 - axis] = n
    phi = 0.5 + b * np.sin(k * xc).reshape(shape) * np.ones(g.shape)
    vel = [np.zeros(g.shape) for _ in range(3)]
    vel[axis][:] = U
    r = orc.acdi_rhs(g, orc.flow_params(gamma=0.0, eps=0.1), phi, *vel)
    h = L / n
    want = (-U * b * np.cos(k * xc) * math.sin(k * h) / h).reshape(shape) * np.ones(g.shape)
    assert np.abs(r - want).max() <= 1e-13


@pytest.mark.parametrize("axis", [0, 2])
def test_acdi_equilibrium_profile_second_order(orc, axis):
    """phi = (1 + tanh(s/(2 eps)))/2 makes the regularization flux vanish in
    the continuum (psi = s, n = 1, eps phi' = (1 - tanh^2)/4); the discrete
    right-hand side with u = 0 falls as h^2 at fixed eps (walls across s)."""
    eps, L = 0.05, 1.0
    errs = []
    for n in (32, 64, 128):
        bc = [0, 0, 0]
        bc[axis] = 1
        dims = [2, 2, 2]
        dims[axis] = n
        lens = [2.0 / 32, 2.0 / 32, 2.0 / 32]
        lens[axis] = L
        g = grid(orc, *dims, *lens, bc)
        s = centres(n, L) - 0.5
        shape = [1, 1, 1]
        shape[2 - axis] = n
        phi = (0.5 * (1 + np.tanh(s / (2 * eps)))).reshape(shape) * np.ones(g.shape)
        z = np.zeros(g.shape)
        errs.append(np.abs(orc.acdi_rhs(g, orc.flow_params(gamma=1.0, eps=eps), phi, z, z, z)).max())
    assert errs[0] / errs[1] > 3.6 and errs[1] / errs[2] > 3.8, errs


@pytest.mark.parametrize("thick,sign", [(2.0, 1.0), (0.6, -1.0)])
def test_acdi_sharpens_thick_and_widens_thin_profiles(orc, thick, sign):
    """Thicker than equilibrium: phi falls on the phase-2 side and rises on
    the phase-1 side of the interface; thinner: the reverse."""
    n, L, eps = 128, 1.0, 0.02
    g = grid(orc, n, 2, 2, L, 2 * L / n, 2 * L / n, (1, 0, 0))
    s = centres(n, L) - 0.5
    phi = (0.5 * (1 + np.tanh(s / (2 * eps * thick)))) * np.ones(g.shape)
    z = np.zeros(g.shape)
    r = orc.acdi_rhs(g, orc.flow_params(gamma=1.0, eps=eps), phi, z, z, z)[0, 0]
    near = (np.abs(s) > 0.2 * eps) & (np.abs(s) < 2.0 * eps)
    assert np.all(np.sign(r[near]) == sign * np.sign(s[near]))


def sphere_phi(n, L, R, eps, centre=(0.5, 0.5, 0.5), cyl=False):
    c = centres(n, L)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    d2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (0 if cyl else (Z - centre[2]) ** 2)
    d = np.sqrt(d2)
    return 0.5 * (1 + np.tanh((R - d) / (2 * eps))), d


def test_acdi_normals_point_into_phase_one(orc):
    n, L, R = 32, 1.0, 0.25
    eps = 0.51 * L / n
    g = grid(orc, n, n, n, L, L, L)
    phi, d = sphere_phi(n, L, R, eps)
    psi, nx, ny, nz = orc.acdi_normals(g, orc.flow_params(gamma=1.0, eps=eps), phi)
    mag = np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    assert np.abs(mag[d > 0.02] - 1.0).max() <= 1e-14
    c = centres(n, L)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    band = np.abs(d - R) < 2 * L / n
    cosang = -(nx * (X - 0.5) + ny * (Y - 0.5) + nz * (Z - 0.5))[band] / d[band]
    assert cosang.min() > 0.99
    # psi = eps ln(phi/(1-phi)) exactly for phi strictly inside (0, 1)
    m = (phi > 1e-6) & (phi < 1 - 1e-6)
    assert np.abs(psi[m] - eps * np.log(phi[m] / (1 - phi[m]))).max() <= 1e-12 * eps * 20


def test_acdi_normals_exact_for_a_tilted_plane_on_a_stretched_grid(orc):
    """psi linear in x and z: the central differences are exact on any
    spacing, so n = (a, 0, b)/sqrt(a^2 + b^2) at every cell whose
    neighbours are inside the walls."""
    g = grid(orc, 8, 2, 12, 1.0, 0.25, 1.0, (1, 0, 1), zf=W.zf_tanh(12, 1.0, 1.8))
    eps, a, b = 0.05, 0.3, 0.8
    x = centres(8, 1.0)
    z = 0.5 * (g.zf[:-1] + g.zf[1:])
    psi = a * (x[None, None, :] - 0.5) + b * (z[:, None, None] - 0.5) + np.zeros(g.shape)
    phi = 1.0 / (1.0 + np.exp(-psi / eps))
    _, nx, ny, nz = orc.acdi_normals(g, orc.flow_params(gamma=1.0, eps=eps, eps_s=0.0), phi)
    inner = (slice(1, -1), slice(None), slice(1, -1))
    r = math.hypot(a, b)
    assert np.abs(nx[inner] - a / r).max() <= 1e-12
    assert np.abs(nz[inner] - b / r).max() <= 1e-12
    assert np.abs(ny).max() == 0.0


@pytest.mark.parametrize("cyl", [False, True])
def test_curvature_of_spheres_and_cylinders(orc, cyl):
    errs = []
    for n in (32, 64):
        L, R = 1.0, 0.25
        eps = 0.51 * L / n
        g = grid(orc, n, n, n, L, L, L)
        phi, d = sphere_phi(n, L, R, eps, cyl=cyl)
        k = orc.curvature(g, orc.flow_params(gamma=1.0, eps=eps), phi)
        exact = (1.0 if cyl else 2.0) / R
        band = np.abs(phi - 0.5) < 0.2
        errs.append(np.abs(k[band] / exact - 1).max())
    assert errs[0] < 0.08 and errs[1] < 0.04, errs


def test_acdi_axis_permutation(orc):
    rng = np.random.default_rng(11)
    n = 10
    g = grid(orc, n, n, n, 1.0, 1.0, 1.0)
    phi = smooth_phi(rng, g)
    u, v, w = (rng.uniform(-1, 1, g.shape) for _ in range(3))
    fl = orc.flow_params(gamma=1.1, eps=0.07)
    r = orc.acdi_rhs(g, fl, phi, u, v, w)
    # x <-> z: arrays [k][j][i] transposed, u <-> w swapped
    t = lambda a: np.ascontiguousarray(a.transpose(2, 1, 0))
    r2 = orc.acdi_rhs(g, fl, t(phi), t(w), t(v), t(u))
    assert np.abs(t(r2) - r).max() <= 1e-12 * np.abs(r).max()


# -------------------------------------------------------------- momentum

def two_phase(orc, g, rng, sigma=0.0, gamma=1.0, g_acc=(0.0, 0.0, 0.0), mu=(0.02, 0.001), rho=(1000.0, 1.0)):
    return orc.flow_params(rho1=rho[0], rho2=rho[1], mu1=mu[0], mu2=mu[1], sigma=sigma, g=g_acc, gamma=gamma,
                           eps=0.08)


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 0, 1)])
def test_momentum_of_a_uniform_flow_is_the_body_force(orc, bc):
    rng = np.random.default_rng(5)
    g = grid(orc, 10, 8, 6, 1.0, 0.8, 0.6, bc, zf=W.zf_tanh(6, 0.6, 1.2))
    phi = smooth_phi(rng, g)
    fl = two_phase(orc, g, rng, g_acc=(0.3, -0.2, -9.81))
    U = [np.full(g.shape, 0.7), np.full(g.shape, -0.4), np.full(g.shape, 0.0 if bc[2] else 0.25)]
    if bc[2]:
        U[2][-1] = 0.0
    ru, rv, rw = orc.momentum_rhs(g, fl, phi, *U)
    # the no-slip walls shear the tangential velocity of the wall-adjacent faces
    inner = slice(1, -1) if bc[2] else slice(None)
    assert np.abs(ru[inner] - 0.3).max() <= 1e-12 and np.abs(rv[inner] + 0.2).max() <= 1e-12
    wz = rw[:-1] if bc[2] else rw
    assert np.abs(wz + 9.81).max() <= 1e-12
    if bc[2]:
        assert np.all(rw[-1] == 0.0)
        assert np.abs(ru[0] - 0.3).min() > 1e-6


@pytest.mark.parametrize("c,d", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_momentum_viscous_term_on_a_shear_mode(orc, c, d):
    """Component c = A sin(k x_d), constant mu and rho, no other motion: the
    right-hand side is -(mu/rho)(4/h^2) sin^2(k h/2) A sin(k x_d) exactly
    (advection vanishes: the field does not vary along c, the transverse
    transport is zero)."""
    n, L, A, m = 16, 2.0, 0.8, 2
    # phi = 1/4 everywhere: mu and rho are the linear maps at 1/4
    mu1, mu2, rho1, rho2 = 0.05, 0.01, 4.0, 1.0
    mu, rho = mu2 + 0.25 * (mu1 - mu2), rho2 + 0.25 * (rho1 - rho2)
    g = grid(orc, n, n, n, L, L, L)
    h, k = L / n, 2 * math.pi * m / L
    # component c sits at the cell centre along d (d != c)
    xd = centres(n, L)
    shape = [1, 1, 1]
    shape[2 - d] = n
    vel = [np.zeros(g.shape) for _ in range(3)]
    vel[c][:] = (A * np.sin(k * xd)).reshape(shape)
    fl = orc.flow_params(rho1=rho1, rho2=rho2, mu1=mu1, mu2=mu2, gamma=1.0, eps=0.1)
    out = orc.momentum_rhs(g, fl, np.full(g.shape, 0.25), *vel)
    want = -(mu / rho) * (4 / h ** 2) * math.sin(k * h / 2) ** 2 * vel[c]
    assert np.abs(out[c] - want).max() <= 1e-12 * np.abs(want).max()
    for e in range(3):
        if e != c:
            assert np.abs(out[e]).max() <= 1e-13


def test_momentum_rigid_rotation_has_no_viscous_stress(orc):
    """u = -W (y - yc), v = W (x - xc): grad u + grad u^T = 0 for the
    discrete differences too, so the viscous part (the difference between
    mu and mu = 0) vanishes at faces away from the walls, for any mu field."""
    rng = np.random.default_rng(2)
    n = 16
    g = grid(orc, n, n, 6, 1.0, 1.0, 0.4, (1, 1, 0))
    h = 1.0 / n
    xc, xf = centres(n, 1.0), (np.arange(n) + 1.0) * h
    u = np.broadcast_to(-1.3 * (xc - 0.5)[:, None], (6, n, n)).copy()
    v = np.broadcast_to(1.3 * (xc - 0.5)[None, :], (6, n, n)).copy()
    u[:, :, -1] = 0.0
    v[:, -1, :] = 0.0
    w = np.zeros(g.shape)
    phi = smooth_phi(rng, g)
    base = dict(rho1=3.0, rho2=1.0, sigma=0.0, gamma=0.0, eps=0.08)
    a = orc.momentum_rhs(g, orc.flow_params(mu1=0.05, mu2=0.002, **base), phi, u, v, w)
    b = orc.momentum_rhs(g, orc.flow_params(mu1=0.0, mu2=0.0, **base), phi, u, v, w)
    inner = (slice(None), slice(2, -3), slice(2, -3))
    for x, y in zip(a, b):
        assert np.abs((x - y)[inner]).max() <= 1e-12
    assert np.abs((a[0] - b[0])[:, 0, :]).max() > 1e-3  # the no-slip walls do shear it


@pytest.mark.parametrize("bc", [(0, 0, 0)])
def test_momentum_is_conserved_at_constant_density(orc, bc):
    rng = np.random.default_rng(8)
    g = grid(orc, 10, 8, 6, 1.0, 0.8, 0.6, bc, zf=W.zf_tanh(6, 0.6, 1.0))
    phi = smooth_phi(rng, g)
    u, v, w = (rng.uniform(-1, 1, g.shape) for _ in range(3))
    fl = orc.flow_params(rho1=1.0, rho2=1.0, mu1=0.05, mu2=0.001, sigma=0.0, gamma=1.0, eps=0.08)
    out = orc.momentum_rhs(g, fl, phi, u, v, w)
    dzf = np.diff(g.zf)
    dzc = np.empty(g.nz)
    dzc[:-1] = 0.5 * (dzf[:-1] + dzf[1:])
    dzc[-1] = 0.5 * (dzf[-1] + dzf[0])
    vx = (g.lx / g.nx) * (g.ly / g.ny) * dzf[:, None, None]
    vz = (g.lx / g.nx) * (g.ly / g.ny) * dzc[:, None, None]
    for o, vv in zip(out, (vx, vx, vz)):
        s = (o * vv).sum()
        assert abs(s) <= 1e-13 * (np.abs(o) * vv).sum()


def test_momentum_regularization_term_second_order(orc):
    """phi = (1 + tanh(x/(4 eps)))/2 (twice the equilibrium thickness) has
    the flux a = Gamma (1/8 - 1/4)(1 - tanh^2(x/(4 eps))) in the continuum;
    with u = A sin(2 pi x / L), mu = 0, sigma = 0 the Gamma-dependent part of
    the u right-hand side is (rho1 - rho2) a u' / rho, reached at h^2."""
    L, eps, A, G = 1.0, 0.03, 0.5, 1.7
    rho1, rho2 = 10.0, 1.0
    errs = []
    for n in (64, 128, 256):
        h = L / n
        g = grid(orc, n, 2, 2, L, 2 * h, 2 * h, (1, 0, 0))
        xc, xf = centres(n, L) - 0.5, (np.arange(n) + 1.0) * h - 0.5
        phi = (0.5 * (1 + np.tanh(xc / (4 * eps)))) * np.ones(g.shape)
        u = (A * np.sin(2 * math.pi * (xf + 0.5))) * np.ones(g.shape)
        u[..., -1] = 0.0
        z = np.zeros(g.shape)
        mk = lambda gam: orc.flow_params(rho1=rho1, rho2=rho2, mu1=0.0, mu2=0.0, sigma=0.0, gamma=gam, eps=eps)
        a = orc.momentum_rhs(g, mk(G), phi, u, z, z)[0]
        b = orc.momentum_rhs(g, mk(0.0), phi, u, z, z)[0]
        t = np.tanh(xf / (4 * eps))
        aex = G * (0.125 - 0.25) * (1 - t ** 2)
        rf = rho2 + (rho1 - rho2) * 0.5 * (1 + np.tanh(xf / (4 * eps)))
        want = (rho1 - rho2) * aex * A * 2 * math.pi * np.cos(2 * math.pi * (xf + 0.5)) / rf
        inner = slice(2, n - 3)
        errs.append(np.abs((a - b)[0, 0, inner] - want[inner]).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.7, errs


def test_static_drop_laplace_jump(orc):
    """A drop at rest with surface tension: after one substep the pressure
    jump across the interface is sigma kappa = 2 sigma / R (within 3 % at
    R = 8 h)."""
    n, L, R, sig = 32, 1.0, 0.25, 0.1
    eps = 0.51 * L / n
    g = grid(orc, n, n, n, L, L, L)
    phi, d = sphere_phi(n, L, R, eps)
    fl = orc.flow_params(rho1=1.0, rho2=1.0, mu1=0.0, mu2=0.0, sigma=sig, gamma=0.0, eps=eps)
    z = np.zeros(g.shape)
    hs = [np.zeros(g.shape) for _ in range(4)]
    out = orc.flow_substep(g, fl, 1, 1e-3, phi, z, z, z, z, z, 0.0, hs)
    p = out[4]
    jump = p[d < 0.1].mean() - p[d > 0.4].mean()
    assert abs(jump / (2 * sig / R) - 1) < 0.03
    assert np.array_equal(out[0], phi)  # Gamma = 0, u = 0: the phase field does not move


# --------------------------------------------------------------- substep

def test_rk3_coefficients_are_third_order(orc):
    """The low-storage scheme on y' = lam y over one step (three substeps)
    matches exp(lam Dt) to O(Dt^4): the error falls by 2^4 when Dt halves."""
    lam = -1.3 + 0.7j
    errs = []
    for Dt in (0.2, 0.1, 0.05):
        y, hprev = 1.0 + 0j, 0.0
        for s in (1, 2, 3):
            ga, ze, al = orc.rk3_coeffs(s)
            rr = lam * y
            y = y + Dt * (ga * rr + ze * hprev)
            hprev = rr
        errs.append(abs(y - np.exp(lam * Dt)))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18, errs
    assert abs(sum(orc.rk3_coeffs(s)[2] for s in (1, 2, 3)) - 1.0) <= 1e-15


def _taylor_green(orc, n, nu=0.05, T=0.5, cfl=0.2):
    L = 2 * math.pi
    h = L / n
    g = orc.Grid(n, n, 2, L, L, W.zf_uniform(2, 2 * h), 0, 0, 0)
    xc, xf = centres(n, L), (np.arange(n) + 1.0) * h

    def exact(t):
        e = math.exp(-2 * nu * t)
        u = np.broadcast_to(np.sin(xf)[None, :] * np.cos(xc)[:, None] * e, (2, n, n)).copy()
        v = np.broadcast_to(-np.cos(xc)[None, :] * np.sin(xf)[:, None] * e, (2, n, n)).copy()
        return u, v

    u, v = exact(0.0)
    w, phi = np.zeros_like(u), np.zeros_like(u)
    fl = orc.flow_params(rho1=1.0, rho2=1.0, mu1=nu, mu2=nu, gamma=1.0, eps=0.51 * h)
    nst = int(round(T / (cfl * h)))
    Dt = T / nst
    p1, p2, dtprev = np.zeros_like(u), np.zeros_like(u), None
    hs = [np.zeros_like(u) for _ in range(4)]
    for _ in range(nst):
        for s in (1, 2, 3):
            al = orc.rk3_coeffs(s)[2]
            r = 0.0 if dtprev is None else al * Dt / dtprev
            phi, u, v, w, p, d = orc.flow_substep(g, fl, s, Dt, phi, u, v, w, p1, p2, r, hs)
            assert d["max_div_rel"] <= 1e-12
            p2, p1, dtprev = p1, p, al * Dt
    ue, ve = exact(T)
    return max(np.abs(u - ue).max(), np.abs(v - ve).max())


def test_taylor_green_decay_second_order(orc):
    e16, e32 = _taylor_green(orc, 16), _taylor_green(orc, 32)
    assert e32 < 2e-4 and e16 / e32 > 3.7, (e16, e32)


def test_substep_conserves_phase_volume_and_projects(orc):
    rng = np.random.default_rng(4)
    n = 16
    g = grid(orc, n, n, 12, 1.0, 1.0, 0.75, (0, 0, 1), zf=W.zf_tanh(12, 0.75, 1.3))
    phi, _ = sphere_phi(n, 1.0, 0.2, 0.51 / n, centre=(0.45, 0.5, 0.4))
    phi = phi[:12].copy()
    u, v, w = (0.3 * rng.uniform(-1, 1, g.shape) for _ in range(3))
    w[-1] = 0.0
    fl = orc.flow_params(rho1=1000.0, rho2=1.0, mu1=1e-2, mu2=1e-4, sigma=0.05, g=(0, 0, -1.0), gamma=1.0,
                         eps=0.51 / n)
    hs = [np.zeros(g.shape) for _ in range(4)]
    p1 = np.zeros(g.shape)
    V = vol(g)
    m0 = (phi * V).sum()
    for s in (1, 2, 3):
        phi, u, v, w, p, d = orc.flow_substep(g, fl, s, 2e-3, phi, u, v, w, p1, p1, 0.0, hs)
        assert d["max_div_rel"] <= 1e-12
        assert np.all(w[-1] == 0.0)
        p1 = p
    assert abs((phi * V).sum() - m0) <= 1e-13 * m0


def test_substep_extrapolates_the_pressure_linearly(orc):
    """p* = (1 + r) p1 - r p2: (p1, p2 = 0, r = 1) and (2 p1, p2, r = 0) give
    the same substep, (q, q, any r) the same as (q, 0, r = 0)."""
    rng = np.random.default_rng(9)
    n = 12
    g = grid(orc, n, n, 8, 1.0, 1.0, 0.7, (0, 0, 1))
    phi, _ = sphere_phi(n, 1.0, 0.25, 0.51 / n, centre=(0.5, 0.5, 0.35))
    phi = phi[:8].copy()
    u, v, w = (0.2 * rng.uniform(-1, 1, g.shape) for _ in range(3))
    w[-1] = 0.0
    q = rng.normal(size=g.shape)
    fl = orc.flow_params(rho1=100.0, rho2=1.0, mu1=1e-3, mu2=1e-4, sigma=0.0, gamma=1.0, eps=0.51 / n)
    z = np.zeros(g.shape)

    def run(p1, p2, r):
        hs = [np.zeros(g.shape) for _ in range(4)]
        return orc.flow_substep(g, fl, 1, 1e-3, phi, u, v, w, p1, p2, r, hs)[:5]

    a, b = run(q, z, 1.0), run(2 * q, z, 0.0)
    c, d = run(q, q, 0.7), run(q, z, 0.0)
    e = run(z, z, 0.0)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * max(np.abs(y).max(), 1.0)
    for x, y in zip(c, d):
        assert np.abs(x - y).max() <= 1e-12 * max(np.abs(y).max(), 1.0)
    assert np.abs(a[4] - e[4]).max() > 1e-6  # p* matters at density ratio 100
