"""Helpers shared by the GPU tests: move a seeded case to the GPU, run the
library through the C ABI, compare with the oracle."""
import numpy as np

from tests import manufactured as M


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_plan(plan, case, inplace=False):
    import torch
    rho, ps, u, v, w = [to_dev(a) for a in case.fields()]
    if inplace:
        uo, vo, wo, p, rep = plan.step(case.dt, case.rho0, rho, ps, u, v, w, u_out=u, v_out=v, w_out=w)
    else:
        uo, vo, wo, p, rep = plan.step(case.dt, case.rho0, rho, ps, u, v, w)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (uo, vo, wo, p)], rep


def errors(got, ref):
    """max-norm relative error per field (u, v, w, p)."""
    return {n: M.relerr(g, r) for n, g, r in zip("uvwp", got, ref)}


EPS = np.finfo(np.float64).eps


def div_terms_max(case, u, v, w):
    """max over cells of |du/dx| + |dv/dy| + |dw/dz| (the three face
    differences of the divergence, each divided by its spacing): the scale
    of the rounding noise in any evaluation of D u."""
    g = case.grid
    dx, dy = g.lx / g.nx, g.ly / g.ny
    dzf = np.diff(np.asarray(g.zf, dtype=np.float64))[:, None, None]

    def back(a, axis, wall):
        b = np.roll(a, 1, axis=axis)
        if wall:
            idx = [slice(None)] * 3
            idx[axis] = 0
            b[tuple(idx)] = 0.0
        return b

    t = (np.abs(u - back(u, 2, g.bcx == 1)) / dx + np.abs(v - back(v, 1, g.bcy == 1)) / dy +
         np.abs(w - back(w, 0, g.bcz == 1)) / dzf)
    return float(t.max())


def check_div(orc, case, got, rep, what=""):
    """The divergence the GPU reports is max |D u_out| of the velocity it
    stored: compared with the oracle's D applied to the GPU's own u_out, to
    1 % of the value plus the rounding noise of evaluating D in two different
    operation orders (8 eps times the largest sum of face-difference terms)."""
    g = orc.Grid.from_workload(case.grid)
    dv = float(np.abs(orc.div(g, got[0], got[1], got[2])).max())
    noise = 8 * EPS * div_terms_max(case, got[0], got[1], got[2])
    diff = abs(rep["max_div_abs"] - dv)
    assert diff <= 0.01 * dv + noise, (what, rep["max_div_abs"], dv, noise)
    return dv, noise
