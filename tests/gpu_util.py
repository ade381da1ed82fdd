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
