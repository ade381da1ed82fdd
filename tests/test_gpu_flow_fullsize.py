"""The substep at the benchmark's full size and launch configuration: one
Runge-Kutta substep of the 512^3 bubble channel exactly as bench.py runs it
(state from one pressure-correction step, the same parameters and step),
checked against the oracle on sampled windows.

The right-hand sides are local: a cell's phase-field and momentum
right-hand sides depend on the inputs within 4 cells (psi -> normals ->
flux and curvature -> right-hand side).  So the oracle runs on windows of
20 x 20 columns x all nz planes, cut out of the full inputs with the
periodic wrap in x and y and taken as periodic grids themselves: its
results in the 10 x 10 columns 5 cells or more from a window's edge are
exactly the full grid's.  Windows sit at seeded positions, two of them
across the periodic seams, and span both walls in z.  Checked per window:
the phase and momentum right-hand sides the substep stores (hphi, hu, hv,
hw) within 1e-11 of each field's max norm (as the 128^3 substep tests),
and the updated phase field (phi + Dt gamma_1 R for the first substep)
within that tolerance carried through the update plus its rounding."""
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-11
WIN, MARGIN = 20, 5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_substep_512_on_sampled_windows(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_04189_amd import pcx
    import bench
    case = W.config3()
    gs = case.grid
    st, prm, umax = bench.flow_setup(case)
    Dt = bench.flow_dt(gs, prm, umax)
    _say(f"512^3 substep: umax {umax:.3e}, Dt {Dt:.3e}")
    F = pcx.Flow(gs, **prm)
    z = torch.zeros(gs.shape, dtype=torch.float64, device="cuda")
    h = [torch.zeros_like(z) for _ in range(4)]
    outs = [torch.empty_like(z) for _ in range(5)]
    F.substep(1, Dt, *st, z, z, 0.0, h, outs)
    torch.cuda.synchronize()
    F.close()
    host = [t.cpu().numpy() for t in st]            # phi, u, v, w
    hh = [t.cpu().numpy() for t in h]               # hphi, hu, hv, hw
    phi_out = outs[0].cpu().numpy()
    del st, h, outs, z
    torch.cuda.empty_cache()
    scale = [max(np.abs(a).max(), 1e-300) for a in hh]
    gamma1 = orc.rk3_coeffs(1)[0]
    fl = orc.flow_params(eps=prm["eps"], rho1=prm["rho1"], rho2=prm["rho2"], mu1=prm["mu1"], mu2=prm["mu2"],
                         sigma=prm["sigma"], g=prm["g"], gamma=prm["gamma"])
    wg = orc.Grid(WIN, WIN, gs.nz, WIN * gs.lx / gs.nx, WIN * gs.ly / gs.ny, gs.zf, 0, 0, gs.bcz)
    rng = np.random.default_rng(5120)
    starts = [(gs.nx - 7, gs.ny - 9), (3, gs.ny - 12)] + [tuple(int(x) for x in rng.integers(0, 512, 2))
                                                         for _ in range(6)]
    worst = 0.0
    for (i0, j0) in starts:
        ix = np.arange(i0, i0 + WIN) % gs.nx
        jy = np.arange(j0, j0 + WIN) % gs.ny
        cut = lambda a: np.ascontiguousarray(a[:, jy][:, :, ix])
        phi, u, v, w = (cut(a) for a in host)
        ra = orc.acdi_rhs(wg, fl, phi, u, v, w)
        rm = orc.momentum_rhs(wg, fl, phi, u, v, w)
        inner = (slice(None), slice(MARGIN, WIN - MARGIN), slice(MARGIN, WIN - MARGIN))
        errs = [float(np.abs(cut(g)[inner] - r[inner]).max() / s)
                for g, r, s in zip(hh, [ra, *rm], scale)]
        ephi = float(np.abs(cut(phi_out)[inner] - (phi + Dt * gamma1 * ra)[inner]).max())
        _say(f"  window at ({i0}, {j0}): hphi hu hv hw errors {' '.join(f'{e:.2e}' for e in errs)}, "
             f"phi_out {ephi:.2e}")
        # phi_out = phi + Dt gamma_1 R: R's own tolerance carried through, plus
        # the rounding of the update (phi is in [0, 1])
        assert max(errs) <= TOL and ephi <= Dt * gamma1 * TOL * scale[0] + 1e-15
        worst = max(worst, max(errs))
    _say(f"  worst {worst:.2e}")
