"""GPU parity of the fused stencil + forward x passes (the RHS, and the
residual of the refined form, evaluated inside the x transform and never
stored) against the oracle, beside the separate stencil and x-transform
launches on the same inputs (PCX_FUSE / PCX_FUSE_RHS at plan creation; the
residual's fusion is on by default, the RHS's opt-in).  The fused form
runs where the x pass takes one row per wave: half lengths 256 and 512
(nx = 512, 1024); the cases cover partial row tiles, walls in x and y (odd
ny), periodic and stretched z."""
import os
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests.gpu_util import check_div, errors, run_plan

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
REF_TOL = 1e-10

CASES = [
    ((512, 18, 6), (0, 0, 1), 1.6),
    ((512, 9, 5), (1, 1, 0), 0.0),
    ((1024, 16, 4), (0, 0, 0), 0.0),
    ((512, 27, 7), (0, 1, 1), 1.2),
    ((1024, 12, 6), (0, 1, 1), 1.4),
]


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


def _plan(pcx, grid, prec, fuse):
    """A plan with both fused passes (the RHS one is opt-in) or neither."""
    old = {k: os.environ.get(k) for k in ("PCX_FUSE", "PCX_FUSE_RHS")}
    os.environ["PCX_FUSE"] = "1" if fuse else "0"
    os.environ["PCX_FUSE_RHS"] = "1" if fuse else "0"
    try:
        return pcx.Plan(grid, prec)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("dims,bc,stretch", CASES)
def test_fused_vs_oracle_and_unfused(pcx, orc, dims, bc, stretch):
    case = W.random_case(11 + sum(dims), *dims, *bc, stretch=stretch)
    g = orc.Grid.from_workload(case.grid)
    ref = list(orc.step(g, case.dt, case.rho0, *case.fields())[:4])
    for prec, tol in (("fp64", FP64_TOL), ("fp32_refined", REF_TOL)):
        res = {}
        for fuse in (True, False):
            _say(f"case {case.name} {prec} fused={fuse}")
            plan = _plan(pcx, case.grid, prec, fuse)
            plan.set_timing(True)
            got, rep = run_plan(plan, case)
            names = {n for n, _ in plan.pass_times()}
            plan.close()
            assert ("rhs_fftx" in names) == fuse, names
            if prec == "fp32_refined":
                assert ("resid_fftx" in names) == fuse, names
            e = errors(got, ref)
            _say(f"  errors {e} div {rep['max_div_rel']:.3e} solves {rep['solves']}")
            assert max(e.values()) <= tol
            assert rep["max_div_rel"] <= tol
            check_div(orc, case, got, rep, f"{case.name} {prec} fused={fuse}")
            res[fuse] = (got, rep)
        # the same f (and residuals) either way: same norms up to rounding
        rf, ru = res[True][1], res[False][1]
        assert abs(rf["f_inf"] - ru["f_inf"]) <= 1e-14 * ru["f_inf"]
        assert rf["solves"] == ru["solves"]
