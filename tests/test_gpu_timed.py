"""GPU parity on exactly the inputs and launch configurations bench.py times:

* the 512^3 wall-channel case with 512 bubbles (the headline workload), one
  FP64 step and one refined step, each compared element by element with one
  oracle step on the same inputs;
* all 192 domains of the batch recipe (seed 1004), batched with autotuned
  shapes (the tune cache bench.py uses) in the refined form and in FP64,
  every domain compared element by element with the oracle.

The reported divergence is checked against the oracle's D applied to the
GPU's own velocity output in every case.
"""
import sys
import time

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests import manufactured as M
from tests.gpu_util import check_div, errors, run_plan, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
REF_TOL = 1e-10


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


@pytest.mark.timeout(1200)
def test_config3_512_fp64_and_refined_vs_oracle(pcx, orc):
    import torch
    t0 = time.perf_counter()
    c = W.config3()
    _say(f"case {c.name}: generated in {time.perf_counter() - t0:.1f} s")
    got = {}
    reps = {}
    for prec in ("fp64", "fp32_refined"):
        plan = pcx.Plan(c.grid, prec)
        got[prec], reps[prec] = run_plan(plan, c)
        plan.close()
        torch.cuda.empty_cache()
        _say(f"GPU {prec} step done, report {reps[prec]}")
    t0 = time.perf_counter()
    g = orc.Grid.from_workload(c.grid)
    ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
    _say(f"oracle step (single thread) at 512^3 in {time.perf_counter() - t0:.1f} s")
    for prec, tol in (("fp64", FP64_TOL), ("fp32_refined", REF_TOL)):
        e = errors(got[prec], ref)
        dv, noise = check_div(orc, c, got[prec], reps[prec], f"{c.name} {prec}")
        _say(f"{prec}: errors {e}, reported max|D u| {reps[prec]['max_div_abs']:.3e}, "
             f"oracle D of the GPU output {dv:.3e} (noise bound {noise:.1e})")
        assert max(e.values()) <= tol
        assert reps[prec]["max_div_rel"] <= tol
    assert reps["fp32_refined"]["converged"] == 1


def _domains(cases):
    import torch
    doms = []
    for c in cases:
        rho, ps, u, v, w = [to_dev(a) for a in c.fields()]
        outs = [torch.zeros(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        doms.append({"grid": c.grid, "dt": c.dt, "rho0": c.rho0, "rho": rho, "pstar": ps, "u": u, "v": v,
                     "w": w, "u_out": outs[0], "v_out": outs[1], "w_out": outs[2], "p_out": outs[3]})
    return doms


@pytest.mark.timeout(1200)
def test_config4_all_192_domains_vs_oracle(pcx, orc):
    import torch
    t0 = time.perf_counter()
    cases = W.config4()
    assert len(cases) == 192
    _say(f"batch recipe: {len(cases)} domains, {sum(c.grid.cells for c in cases)} cells, generated in "
         f"{time.perf_counter() - t0:.1f} s")
    doms = _domains(cases)
    cache = pcx.batch_tune_cache_path()
    outs = {}
    reps = {}
    for prec, tune in (("fp32_refined", True), ("fp64", True)):
        t0 = time.perf_counter()
        b = pcx.Batch(doms, prec, autotune=tune, tune_cache=cache)
        b.launch()
        torch.cuda.synchronize()
        reps[prec], st = b.reports()
        assert st == pcx.PCX_OK, prec
        outs[prec] = [[d[k].cpu().numpy() for k in ("u_out", "v_out", "w_out", "p_out")] for d in doms]
        _say(f"batch {prec} (autotune={tune}, cache {cache}) created and run in {time.perf_counter() - t0:.1f} s")
        b.close()
    t0 = time.perf_counter()
    worst = {"fp64": 0.0, "fp32_refined": 0.0}
    for i, c in enumerate(cases):
        g = orc.Grid.from_workload(c.grid)
        ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
        for prec, tol in (("fp64", FP64_TOL), ("fp32_refined", REF_TOL)):
            e = errors(outs[prec][i], ref)
            r = reps[prec][i]
            worst[prec] = max(worst[prec], max(e.values()))
            assert max(e.values()) <= tol, (c.name, prec, e)
            assert r["max_div_rel"] <= tol, (c.name, prec, r)
            check_div(orc, c, outs[prec][i], r, f"{c.name} {prec}")
        if i % 32 == 31:
            _say(f"  {i + 1} domains checked against the oracle ({time.perf_counter() - t0:.1f} s)")
    _say(f"worst max-norm relative errors over the 192 domains: {worst}")
