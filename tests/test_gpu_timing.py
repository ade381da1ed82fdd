"""Per-pass timing of a plan on the GPU: the timing modes report the passes
they promise (every pass, or the velocity correction alone, once per step),
and timing does not change the step's results (bit for bit)."""
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests.gpu_util import run_plan

pytestmark = pytest.mark.gpu

FP64_PASSES = {"rhs_stencil", "x_fft_fwd", "y_fft_fwd", "z_solve", "y_fft_inv", "x_fft_inv_store_p", "x_max",
               "correct_div"}


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


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_timing_modes(pcx, prec):
    case = W.random_case(41, 96, 64, 24, stretch=1.3)
    _say(f"timing modes {case.name} {prec}")
    plan = pcx.Plan(case.grid, prec)
    ref, _ = run_plan(plan, case)
    steps = 3
    # every pass
    plan.set_timing(True)
    for _ in range(steps):
        got, _ = run_plan(plan, case)
    allp = plan.pass_times()
    names = [n for n, _ in allp]
    # the refined form with a report may correct again after an extra solve
    ncorr = names.count("correct_div")
    assert ncorr == steps if prec == "fp64" else ncorr >= steps
    if prec == "fp64":
        assert set(names) == FP64_PASSES
        assert len(names) == steps * len(FP64_PASSES)
    assert all(t > 0.0 for _, t in allp)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
    # the correction only: one duration per step
    plan.set_timing(True, correction_only=True)
    for _ in range(steps):
        got, _ = run_plan(plan, case)
    corr = plan.pass_times()
    assert [n for n, _ in corr] == ["correct_div"] * len(corr)
    assert len(corr) == ncorr
    assert all(t > 0.0 for _, t in corr)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
    # off: nothing recorded
    plan.set_timing(False)
    run_plan(plan, case)
    assert plan.pass_times() == []
    plan.close()
