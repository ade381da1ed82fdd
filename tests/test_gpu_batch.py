"""GPU tests of the batched form (persistent kernel in a HIP graph) against
the CPU oracle and against the single-domain plans."""
import os
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests import manufactured as M
from tests.gpu_util import check_div, to_dev

pytestmark = pytest.mark.gpu
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


def _domains(cases):
    import torch
    doms = []
    for c in cases:
        rho, ps, u, v, w = [to_dev(a) for a in c.fields()]
        outs = [torch.zeros(c.grid.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        doms.append({"grid": c.grid, "dt": c.dt, "rho0": c.rho0, "rho": rho, "pstar": ps, "u": u, "v": v,
                     "w": w, "u_out": outs[0], "v_out": outs[1], "w_out": outs[2], "p_out": outs[3]})
    return doms


def _outs(d):
    return [d[k].cpu().numpy() for k in ("u_out", "v_out", "w_out", "p_out")]


def test_batch_refined_vs_oracle(pcx, orc):
    import torch
    cases = W.config4(ndom=10)
    _say("batch refined: 10 domains drawn by the batch recipe (seed 1004, ndom=10): " +
         ", ".join(c.name for c in cases))
    doms = _domains(cases)
    b = pcx.Batch(doms, "fp32_refined")
    b.launch()
    torch.cuda.synchronize()
    reps, st = b.reports()
    for c, d, r in zip(cases, doms, reps):
        g = orc.Grid.from_workload(c.grid)
        ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
        e = {n: M.relerr(x, y) for n, x, y in zip("uvwp", _outs(d), ref)}
        _say(f"{c.name}: errors {e} div {r['max_div_rel']:.2e} converged {r['converged']}")
        assert max(e.values()) <= REF_TOL
        assert r["max_div_rel"] <= REF_TOL
        check_div(orc, c, _outs(d), r, c.name)
    assert st == pcx.PCX_OK


def test_batch_fp64_matches_plans_bitwise(pcx):
    import torch
    cases = W.config4(ndom=6)
    _say("batch fp64 vs single plans, 6 domains")
    doms = _domains(cases)
    b = pcx.Batch(doms, "fp64")
    b.launch()
    torch.cuda.synchronize()
    for c, d in zip(cases, doms):
        plan = pcx.Plan(c.grid, "fp64")
        uo, vo, wo, p, _ = plan.step(c.dt, c.rho0, d["rho"], d["pstar"], d["u"], d["v"], d["w"])
        for x, y in zip((uo, vo, wo, p), (d["u_out"], d["v_out"], d["w_out"], d["p_out"])):
            assert torch.equal(x, y), c.name


def test_batch_graph_replays(pcx):
    """Replaying the graph (reset kernels + persistent kernel) gives the same
    outputs every time, with eager work and synchronisations in between."""
    import torch
    cases = W.config4(ndom=12)
    doms = _domains(cases)
    b = pcx.Batch(doms, "fp32_refined")
    b.launch()
    torch.cuda.synchronize()
    first = [d["p_out"].clone() for d in doms]
    for rep in range(3):
        for d in doms:
            d["p_out"].fill_(float("nan"))
            d["u_out"].zero_()
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for d, f in zip(doms, first):
            assert torch.equal(d["p_out"], f)
        _say(f"replay {rep} identical")


def test_batch_autotune_and_cache(pcx, orc, tmp_path):
    import torch
    cases = W.config4(ndom=4)
    cache = str(tmp_path / "tune.txt")
    doms = _domains(cases)
    b = pcx.Batch(doms, "fp32_refined", autotune=True, tune_cache=cache)
    b.launch()
    torch.cuda.synchronize()
    txt = open(cache).read()
    _say("tune cache:\n" + txt)
    assert len([l for l in txt.splitlines() if not l.startswith("#")]) >= 1
    for c, d in zip(cases, doms):
        g = orc.Grid.from_workload(c.grid)
        ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
        assert max(M.relerr(x, y) for x, y in zip(_outs(d), ref)) <= REF_TOL
    # re-created from the cache only
    doms2 = _domains(cases)
    b2 = pcx.Batch(doms2, "fp32_refined", tune_cache=cache)
    b2.launch()
    torch.cuda.synchronize()
    for d, d2 in zip(doms, doms2):
        assert torch.equal(d["p_out"], d2["p_out"])


def test_batch_mixed_walls_vs_oracle(pcx, orc):
    """Domains with walls in x and/or y (cosine transforms) batched with
    periodic ones, in both precisions."""
    import torch
    specs = [((32, 48, 32), (1, 0, 1), 1.5), ((48, 32, 64), (0, 1, 0), 0.0), ((64, 64, 32), (1, 1, 1), 1.2),
             ((32, 32, 32), (0, 0, 1), 0.0), ((96, 32, 33), (1, 1, 0), 0.0)]
    cases = [W.random_case(900 + i, *d, *bc, stretch=s) for i, (d, bc, s) in enumerate(specs)]
    for prec, tol in (("fp64", 1e-12), ("fp32_refined", REF_TOL)):
        _say(f"mixed-wall batch {prec}: " + ", ".join(c.name for c in cases))
        doms = _domains(cases)
        b = pcx.Batch(doms, prec)
        b.launch()
        torch.cuda.synchronize()
        reps, st = b.reports()
        for c, d, r in zip(cases, doms, reps):
            g = orc.Grid.from_workload(c.grid)
            ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
            e = {n: M.relerr(x, y) for n, x, y in zip("uvwp", _outs(d), ref)}
            _say(f"  {c.name}: errors {e} report {r}")
            assert max(e.values()) <= tol
            assert r["max_div_rel"] <= tol
            check_div(orc, c, _outs(d), r, c.name)
        assert st == pcx.PCX_OK
