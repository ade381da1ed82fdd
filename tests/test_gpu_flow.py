"""GPU parity of the Runge-Kutta substep around the pressure correction
(phase-field transport, momentum predictor, whole substeps) through the C
ABI against the oracle (oracle/flow.c) on seeded inputs.

Tolerance: max-norm error relative to the field's max norm, 1e-11 for the
right-hand sides (the face fluxes take device log/tanh, which may differ
from the host's by an ulp, and the right-hand side is a difference of face
fluxes over a cell width, which amplifies that by up to the ratio of flux
to right-hand side: about 100 on these grids), 1e-11 for the substep's
outputs (the same plus the pressure step's own 1e-12)."""
import math
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests import manufactured as MF
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_04189_amd import pcx as P
    P.lib()
    return P


def _case(seed, nx, ny, nz, bc, stretch):
    """A drop (tanh profile, eps = 0.51 dx), a random solenoidal velocity,
    random pressures."""
    rng = np.random.default_rng(seed)
    lx, ly, lz = nx / 16.0, ny / 16.0, nz / 16.0
    zf = W.zf_tanh(nz, lz, stretch) if stretch > 0 else W.zf_uniform(nz, lz)
    gs = W.GridSpec(nx, ny, nz, lx, ly, zf, *bc)
    h = lx / nx
    xc, yc = (np.arange(nx) + 0.5) * h, (np.arange(ny) + 0.5) * (ly / ny)
    zc = 0.5 * (zf[:-1] + zf[1:])
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    R = 0.3 * min(lx, ly, lz)
    d = np.sqrt((X - 0.45 * lx) ** 2 + (Y - 0.55 * ly) ** 2 + (Z - 0.5 * lz) ** 2)
    eps = 0.51 * h
    phi = 0.5 * (1 + np.tanh((R - d) / (2 * eps)))
    # a discretely solenoidal velocity (the curl of a random edge
    # potential), largest component 0.5: below the ACDI velocity scale
    u, v, w = MF.divfree_field(rng, gs)
    scale = 0.5 / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    u, v, w = u * scale, v * scale, w * scale
    p1, p2 = rng.normal(size=gs.shape), rng.normal(size=gs.shape)
    return gs, eps, phi, u, v, w, p1, p2


CASES = [
    ((24, 18, 16), (0, 0, 1), 1.4),
    ((32, 32, 32), (0, 0, 0), 0.0),
    ((16, 12, 10), (1, 1, 1), 1.2),
    ((4, 6, 2), (0, 1, 0), 0.0),
    ((18, 24, 9), (1, 0, 0), 0.0),
]
# grids with interior tiles next to walls in x and y (and z): the interior
# kernels run beside the wall tiles, and the flux kernel's interior cells
# next to a wall tile store the normals the wall tiles read
CASES_INTERIOR = [
    ((144, 24, 12), (1, 1, 1), 1.3),
    ((144, 24, 10), (0, 1, 1), 0.0),
]
PARAMS = dict(rho1=1000.0, rho2=1.2, mu1=1e-2, mu2=2e-4, sigma=0.07, g=(0.0, 0.0, -9.81), gamma=1.5)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("dims,bc,stretch", CASES + CASES_INTERIOR)
def test_flow_rhs_vs_oracle(pcx, orc, dims, bc, stretch):
    gs, eps, phi, u, v, w, _, _ = _case(sum(dims), *dims, bc, stretch)
    _say(f"flow rhs {dims} bc {bc} stretch {stretch}")
    g = orc.Grid.from_workload(gs)
    fl = orc.flow_params(eps=eps, **{k: v_ for k, v_ in PARAMS.items()})
    ref_a = orc.acdi_rhs(g, fl, phi, u, v, w)
    ref_m = orc.momentum_rhs(g, fl, phi, u, v, w)
    F = pcx.Flow(gs, eps=eps, **PARAMS)
    dev = [to_dev(a) for a in (phi, u, v, w)]
    got_a = F.phase_rhs(*dev).cpu().numpy()
    got_m = [t.cpu().numpy() for t in F.momentum_rhs(*dev)]
    F.close()
    e = {"phase": _rel(got_a, ref_a)}
    e.update({n: _rel(x, y) for n, x, y in zip(("mu", "mv", "mw"), got_m, ref_m)})
    _say(f"  errors {e}")
    assert max(e.values()) <= TOL


@pytest.mark.parametrize("dims,bc,stretch", CASES[:3] + CASES_INTERIOR)
def test_flow_three_substeps_vs_oracle(pcx, orc, dims, bc, stretch):
    import torch
    gs, eps, phi, u, v, w, p1, p2 = _case(7 + sum(dims), *dims, bc, stretch)
    _say(f"flow substeps {dims} bc {bc}")
    g = orc.Grid.from_workload(gs)
    fl = orc.flow_params(eps=eps, **PARAMS)
    F = pcx.Flow(gs, eps=eps, **PARAMS)
    Dt = 0.1 * gs.lx / gs.nx
    st_o = [phi, u, v, w]
    st_g = [to_dev(a) for a in st_o]
    ho = [np.zeros(gs.shape) for _ in range(4)]
    hg = [torch.zeros(gs.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    po, pg = [p1, p2], [to_dev(p1), to_dev(p2)]
    dtprev = Dt / 3.0
    for s in (1, 2, 3):
        al = orc.rk3_coeffs(s)[2]
        r = al * Dt / dtprev
        *outs_o, d = orc.flow_substep(g, fl, s, Dt, *st_o, po[0], po[1], r, ho)
        outs_g = [torch.empty(gs.shape, dtype=torch.float64, device="cuda") for _ in range(5)]
        rep = F.substep(s, Dt, *st_g, pg[0], pg[1], r, hg, outs_g)
        got = [t.cpu().numpy() for t in outs_g]
        e = {n: _rel(x, y) for n, x, y in zip(("phi", "u", "v", "w", "p"), got, outs_o)}
        eh = max(_rel(a.cpu().numpy(), b) for a, b in zip(hg, ho))
        _say(f"  substep {s}: errors {e}, rhs {eh:.2e}, div {rep['max_div_rel']:.2e}")
        assert max(e.values()) <= TOL and eh <= TOL
        assert rep["max_div_rel"] <= 1e-12
        st_o, st_g = outs_o[:4], outs_g[:4]
        po, pg = [outs_o[4], po[0]], [outs_g[4], pg[0]]
        dtprev = al * Dt
    F.close()


def test_flow_taylor_green_on_the_gpu(pcx):
    """Single phase, the Taylor-Green vortex through whole steps on the GPU:
    the error against the exact decay at T = 0.5 is the oracle's
    second-order discretization error (below 2e-4 at 32^2, falling 4x)."""
    import torch
    errs = []
    for n in (32, 64):
        nu, T, cfl = 0.05, 0.5, 0.2
        L = 2 * math.pi
        h = L / n
        gs = W.GridSpec(n, n, 2, L, L, W.zf_uniform(2, 2 * h), 0, 0, 0)
        xc, xf = (np.arange(n) + 0.5) * h, (np.arange(n) + 1.0) * h
        ex = lambda t: (np.broadcast_to(np.sin(xf)[None, :] * np.cos(xc)[:, None] * math.exp(-2 * nu * t), (2, n, n)),
                        np.broadcast_to(-np.cos(xc)[None, :] * np.sin(xf)[:, None] * math.exp(-2 * nu * t), (2, n, n)))
        u0, v0 = ex(0.0)
        st = [torch.zeros(gs.shape, dtype=torch.float64, device="cuda"), to_dev(np.ascontiguousarray(u0)),
              to_dev(np.ascontiguousarray(v0)), torch.zeros(gs.shape, dtype=torch.float64, device="cuda")]
        F = pcx.Flow(gs, rho1=1.0, rho2=1.0, mu1=nu, mu2=nu, gamma=1.0, eps=0.51 * h)
        nst = int(round(T / (cfl * h)))
        Dt = T / nst
        hg = [torch.zeros(gs.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        p1 = torch.zeros(gs.shape, dtype=torch.float64, device="cuda")
        p2 = p1.clone()
        dtprev = None
        for _ in range(nst):
            for s in (1, 2, 3):
                al = (8 / 15, 2 / 15, 1 / 3)[s - 1]
                r = 0.0 if dtprev is None else al * Dt / dtprev
                outs = [torch.empty(gs.shape, dtype=torch.float64, device="cuda") for _ in range(5)]
                F.substep(s, Dt, *st, p1, p2, r, hg, outs, report=False)
                st, p2, p1, dtprev = outs[:4], p1, outs[4], al * Dt
        torch.cuda.synchronize()
        ue, ve = ex(T)
        errs.append(max(np.abs(st[1].cpu().numpy() - ue).max(), np.abs(st[2].cpu().numpy() - ve).max()))
        F.close()
    _say(f"Taylor-Green errors {errs}")
    assert errs[0] < 2e-4 and errs[0] / errs[1] > 3.7


def test_flow_bubble_channel_vs_oracle(pcx, orc):
    """The benchmark's setup at 128^3: the bubble channel's phase field and
    the velocity its pressure step corrects, gas/liquid properties, surface
    tension and gravity; three substeps on the GPU against the oracle."""
    import torch
    c = W.channel_bubbles(128, 4, 1003, "channel128")
    g = orc.Grid.from_workload(c.grid)
    u, v, w, _, _ = orc.step(g, c.dt, c.rho0, *c.fields())
    phi = (1000.0 - c.fields()[0]) / 999.0
    umax = max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    eps = 0.51 * c.grid.lx / c.grid.nx
    prm = dict(rho1=1.0, rho2=1000.0, mu1=1e-5, mu2=1e-3, sigma=0.07, g=(0.0, 0.0, -9.81), gamma=2 * umax)
    fl = orc.flow_params(eps=eps, **prm)
    F = pcx.Flow(c.grid, eps=eps, **prm)
    # the benchmark's step rule (advective and diffusive limits)
    import bench
    Dt = bench.flow_dt(c.grid, dict(prm, eps=eps), umax)
    st_o, st_g = [phi, u, v, w], [to_dev(a) for a in (phi, u, v, w)]
    ho = [np.zeros(c.grid.shape) for _ in range(4)]
    hg = [torch.zeros(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    z = np.zeros(c.grid.shape)
    po, pg = [z, z], [to_dev(z), to_dev(z)]
    dtprev = None
    for s in (1, 2, 3):
        al = orc.rk3_coeffs(s)[2]
        r = 0.0 if dtprev is None else al * Dt / dtprev
        *outs_o, d = orc.flow_substep(g, fl, s, Dt, *st_o, po[0], po[1], r, ho)
        outs_g = [torch.empty(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(5)]
        rep = F.substep(s, Dt, *st_g, pg[0], pg[1], r, hg, outs_g)
        got = [t.cpu().numpy() for t in outs_g]
        e = {n: _rel(x, y) for n, x, y in zip(("phi", "u", "v", "w", "p"), got, outs_o)}
        # divergence after the correction relative to the scale of the
        # velocity differences, max|u|/h_min (with p* = 0 and a nearly
        # solenoidal u*, f is small and the residual relative to ||f|| says
        # little); the oracle's own value on the same inputs beside it
        hmin = min(c.grid.lx / c.grid.nx, float(np.diff(c.grid.zf).min()))
        uscale = max(np.abs(a).max() for a in got[1:4]) / hmin
        _say(f"  channel substep {s}: errors {e}, phi in [{got[0].min():.3e}, {got[0].max():.9f}], "
             f"max|Du| {rep['max_div_abs']:.3e} (relative to max|u|/h {rep['max_div_abs'] / uscale:.2e}; "
             f"residual/||f|| {rep['max_div_rel']:.2e}, oracle's {d['max_div_rel']:.2e})")
        assert max(e.values()) <= TOL
        assert rep["max_div_abs"] <= 1e-12 * uscale
        assert 0.0 <= got[0].min() + 1e-12 and got[0].max() <= 1.0
        st_o, st_g = outs_o[:4], outs_g[:4]
        po, pg = [outs_o[4], po[0]], [outs_g[4], pg[0]]
        dtprev = al * Dt
    F.close()


def test_predict_then_step_is_the_substep(pcx):
    """pcx_flow_predict returns the inputs of the substep's correction: the
    pressure-correction step applied to them gives the substep's outputs
    bit for bit (same kernels, same order)."""
    import torch
    gs, eps, phi, u, v, w, p1, p2 = _case(41, 32, 24, 16, (0, 0, 1), 1.3)
    F = pcx.Flow(gs, eps=eps, **PARAMS)
    st = [to_dev(a) for a in (phi, u, v, w)]
    pg = [to_dev(p1), to_dev(p2)]
    Dt, r = 0.1 * gs.lx / gs.nx, 0.7
    h0 = [torch.zeros(gs.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    for s in (1, 2):
        # substep 2 takes substep 1's right-hand sides (bitwise the same on
        # both paths, checked below)
        ha, hb = [t.clone() for t in h0], [t.clone() for t in h0]
        outs = [torch.empty(gs.shape, dtype=torch.float64, device="cuda") for _ in range(5)]
        F.substep(s, Dt, *st, *pg, r, ha, outs, report=False)
        phi_b = torch.empty_like(outs[0])
        us, vs, ws, rho, ps, rho0, dt = F.predict(s, Dt, *st, *pg, r, hb, phi_b)
        plan = pcx.Plan(gs, "fp64")
        uo, vo, wo, po, _ = plan.step(dt, rho0, rho, ps, us, vs, ws)
        plan.close()
        torch.cuda.synchronize()
        same = [torch.equal(a, b) for a, b in zip(outs + ha, [phi_b, uo, vo, wo, po] + hb)]
        _say(f"  predict + step vs substep {s}: bitwise equal {same}, rho0 {rho0:.4g}, dt/Dt {dt / Dt:.4f}")
        assert all(same)
        assert abs(rho0 - float(rho.min())) == 0.0
        h0 = ha
    F.close()


def test_substep_rejects_aliased_fields(pcx):
    """Right-hand-side buffers and outputs that alias an input or each other
    are rejected before any launch."""
    import torch
    gs, eps, phi, u, v, w, p1, p2 = _case(43, 16, 12, 8, (0, 0, 1), 0.0)
    F = pcx.Flow(gs, eps=eps, **PARAMS)
    st = [to_dev(a) for a in (phi, u, v, w)]
    pg = [to_dev(p1), to_dev(p2)]
    z = lambda: torch.zeros(gs.shape, dtype=torch.float64, device="cuda")
    h = [z() for _ in range(4)]
    outs = [z() for _ in range(5)]
    for bad_h, bad_o in (([st[0]] + h[1:], outs), (h, [h[0]] + outs[1:]), (h, [outs[0], outs[0]] + outs[2:]),
                         ([h[0], h[0]] + h[2:], outs)):
        with pytest.raises(pcx.PcxError):
            F.substep(1, 1e-3, *st, *pg, 0.0, bad_h, bad_o, report=False)
    F.substep(1, 1e-3, *st, *pg, 0.0, h, outs, report=False)  # the valid call still runs
    torch.cuda.synchronize()
    F.close()
