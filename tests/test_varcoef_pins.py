"""Pins of the variable-coefficient projection oracle (oracle/varcoef.c),
the comparator for the splitting error: at constant density it is the
split step; its operator is volume-symmetric, conservative and reduces to
L / rho0; its solve agrees with a dense solve; its output is
divergence-free; and the split step given the exact pressure as p*
reproduces it (the splitting is exact when p* = p).  No GPU."""
import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W


BCS = [(0, 0, 1), (0, 0, 0), (1, 1, 1), (1, 0, 0)]


def _case(orc, seed, nx, ny, nz, bc, stretch, ratio=100.0):
    c = W.random_case(seed, nx, ny, nz, *bc, stretch=stretch, ratio=ratio)
    return c, orc.Grid.from_workload(c.grid)


def vol(g):
    return (g.lx / g.nx) * (g.ly / g.ny) * np.diff(g.zf)[:, None, None] * np.ones(g.shape)


@pytest.mark.parametrize("bc", BCS)
def test_constant_density_is_the_split_step(orc, bc):
    c, g = _case(orc, 3, 12, 10, 8, bc, 1.3)
    rho = np.full(g.shape, 2.5)
    uo, vo, wo, p, it, rr = orc.varcoef_project(g, c.dt, rho, 2.5, c.u, c.v, c.w)
    ref = orc.step(g, c.dt, 2.5, rho, c.pstar, c.u, c.v, c.w)
    assert it == 1
    for a, b in zip((uo, vo, wo, p), ref[:4]):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("bc", BCS)
def test_operator_symmetric_conservative_and_constant_limit(orc, bc):
    c, g = _case(orc, 5, 6, 4, 5, bc, 1.2)
    n = c.grid.cells
    A = np.empty((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        A[:, q] = orc.varcoef_apply(g, c.rho, e.reshape(g.shape)).ravel()
    V = vol(g).ravel()
    VA = V[:, None] * A
    assert np.abs(VA - VA.T).max() <= 1e-12 * np.abs(VA).max()
    assert np.abs(V @ A).max() <= 1e-12 * np.abs(VA).max()
    p = np.random.default_rng(1).normal(size=g.shape)
    rho0 = 3.0
    assert np.abs(orc.varcoef_apply(g, np.full(g.shape, rho0), p) - orc.apply_L(g, p) / rho0).max() <= \
        1e-12 * np.abs(orc.apply_L(g, p)).max() / rho0


@pytest.mark.parametrize("bc", BCS)
def test_solve_matches_a_dense_solve(orc, bc):
    c, g = _case(orc, 7, 6, 4, 5, bc, 1.2, ratio=1000.0)
    n = c.grid.cells
    A = np.empty((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        A[:, q] = orc.varcoef_apply(g, c.rho, e.reshape(g.shape)).ravel()
    V = vol(g).ravel()
    rhs = orc.div(g, c.u, c.v, c.w).ravel() / c.dt
    # bordered system: [A, 1; V^T, 0] [p; s] = [rhs; 0]
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = A
    B[:n, n] = 1.0
    B[n, :n] = V
    want = np.linalg.solve(B, np.append(rhs, 0.0))[:n].reshape(g.shape)
    uo, vo, wo, p, it, rr = orc.varcoef_project(g, c.dt, c.rho, c.rho0, c.u, c.v, c.w, tol=1e-14)
    assert np.abs(p - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("bc", BCS)
def test_projection_is_divergence_free(orc, bc):
    c, g = _case(orc, 9, 16, 12, 10, bc, 1.4, ratio=1000.0)
    uo, vo, wo, p, it, rr = orc.varcoef_project(g, c.dt, c.rho, c.rho0, c.u, c.v, c.w, tol=1e-13)
    d0 = np.abs(orc.div(g, c.u, c.v, c.w)).max()
    assert np.abs(orc.div(g, uo, vo, wo)).max() <= 1e-11 * d0
    assert rr <= 1e-13 and 1 < it < 400


@pytest.mark.parametrize("bc", BCS)
def test_split_step_with_the_exact_pressure_is_exact(orc, bc):
    """With p* = the variable-coefficient pressure, the split step returns
    that pressure and the same velocity: the splitting error vanishes."""
    c, g = _case(orc, 11, 16, 12, 10, bc, 1.4, ratio=1000.0)
    uo, vo, wo, p, it, rr = orc.varcoef_project(g, c.dt, c.rho, c.rho0, c.u, c.v, c.w, tol=1e-14)
    su, sv, sw, sp, _ = orc.step(g, c.dt, c.rho0, c.rho, p, c.u, c.v, c.w)
    for a, b in zip((su, sv, sw, sp), (uo, vo, wo, p)):
        assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()
    # and with another p* it differs: the comparator measures something
    su2 = orc.step(g, c.dt, c.rho0, c.rho, c.pstar, c.u, c.v, c.w)[0]
    assert np.abs(su2 - uo).max() > 1e-6 * np.abs(uo).max()


@pytest.mark.parametrize("bc", BCS)
def test_reported_residual_is_the_volume_weighted_norm(orc, bc):
    """The stopping test measures the residual in the volume-weighted norm,
    the one the operator is symmetric in; stopped early, the reported
    relative residual is that norm of rhs - <rhs> - A p."""
    c, g = _case(orc, 13, 16, 12, 10, bc, 2.0, ratio=1000.0)
    uo, vo, wo, p, it, rr = orc.varcoef_project(g, c.dt, c.rho, c.rho0, c.u, c.v, c.w, tol=1e-4)
    V = vol(g)
    b = orc.div(g, c.u, c.v, c.w) / c.dt
    b = b - (V * b).sum() / V.sum()
    r = b - orc.varcoef_apply(g, c.rho, p)
    want = np.sqrt((V * r * r).sum() / (V * b * b).sum())
    assert rr <= 1e-4 and abs(rr - want) <= 1e-6 * want
