"""The allocation-free step (pcx_step_noalloc, tables and workspace in the
library's fixed device array) against the allocating entry point
(pcx_plan_create + pcx_step) on the same seeded inputs, through the C ABI:
two calls in a row, the second on a smaller grid, in both precisions.  The
two paths run the same kernels on the same tables and tile shapes, so the
outputs must agree bit for bit (which also meets the 1e-12 / 1e-10 bars)."""
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests.gpu_util import errors

pytestmark = pytest.mark.gpu


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


def _cases():
    # a bubble channel (wall z, stretched) and a smaller triply periodic box
    big = W.random_case(31, 96, 64, 48, bcz=W.WALL, stretch=1.8)
    small = W.random_case(5, 24, 18, 10, bcz=W.PERIODIC)
    return big, small


def _run_both(pcx, case, prec):
    import torch
    from tests.gpu_util import to_dev
    rho, ps, u, v, w = [to_dev(a) for a in case.fields()]
    plan = pcx.Plan(case.grid, prec)
    ref = plan.step(case.dt, case.rho0, rho, ps, u, v, w)
    torch.cuda.synchronize()
    plan.close()
    outs = [torch.full(case.grid.shape, float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
    st, rep = pcx.step_noalloc(case.grid, case.dt, case.rho0, rho, ps, u, v, w, *outs, precision=prec)
    torch.cuda.synchronize()
    assert st == pcx.PCX_OK, pcx.lib().pcx_last_error().decode()
    return [t.cpu().numpy() for t in ref[:4]], ref[4], [t.cpu().numpy() for t in outs], rep


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_noalloc_matches_plan_step_two_calls(pcx, prec):
    big, small = _cases()
    for case in (big, small):
        need = pcx.noalloc_scratch_need(case.grid, prec)
        _say(f"noalloc {prec}: {case.name} {case.grid.shape}, scratch need {need} bytes")
        want, rep_w, got, rep_g = _run_both(pcx, case, prec)
        e = errors(got, want)
        _say(f"  vs pcx_step: errors {e}, solves {rep_g['solves']} / {rep_w['solves']}")
        assert max(e.values()) <= (1e-12 if prec == "fp64" else 1e-10)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
        for k in ("solves", "converged", "f_inf", "max_div_abs", "mean_p"):
            assert rep_g[k] == rep_w[k], k
