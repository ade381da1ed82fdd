"""GPU tests at the workload sizes, in the launch configuration bench.py times:
256^3 against the oracle element by element; 512^3 (and a triply periodic
512^3) through the manufactured fixed point, which holds at any size;
determinism and in-place operation."""
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests import manufactured as M
from tests.gpu_util import errors, run_plan

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


@pytest.fixture(scope="module")
def case256():
    return W.config1()


def test_config1_256_fp64_vs_oracle(pcx, orc, case256):
    c = case256
    _say(f"case {c.name}: GPU FP64 step")
    plan = pcx.Plan(c.grid, "fp64")
    got, rep = run_plan(plan, c)
    plan.close()
    _say("oracle step (single thread)...")
    g = orc.Grid.from_workload(c.grid)
    ref = orc.step(g, c.dt, c.rho0, *c.fields())[:4]
    e = errors(got, ref)
    _say(f"errors {e} div {rep['max_div_rel']:.2e}")
    assert max(e.values()) <= 1e-12
    assert rep["max_div_rel"] <= 1e-12


def test_config1_256_refined_vs_fp64(pcx, case256):
    import torch
    c = case256
    p64 = pcx.Plan(c.grid, "fp64")
    g64, _ = run_plan(p64, c)
    p64.close()
    pr = pcx.Plan(c.grid, "fp32_refined")
    gr, rep = run_plan(pr, c)
    e = errors(gr, g64)
    _say(f"refined vs fp64 at 256^3: {e}, solves {rep['solves']}, div {rep['max_div_rel']:.2e}")
    assert rep["converged"] == 1
    assert max(e.values()) <= 1e-10 and rep["max_div_rel"] <= 1e-10


def test_determinism_and_inplace_256(pcx, case256):
    import torch
    c = case256
    dev = [torch.from_numpy(a).to("cuda") for a in c.fields()]
    plan = pcx.Plan(c.grid, "fp64")
    a = plan.step(c.dt, c.rho0, *dev)
    b = plan.step(c.dt, c.rho0, *dev)
    for x, y in zip(a[:4], b[:4]):
        assert torch.equal(x, y)
    u2, v2, w2 = dev[2].clone(), dev[3].clone(), dev[4].clone()
    _, _, _, p_in, rep_in = plan.step(c.dt, c.rho0, dev[0], dev[1], u2, v2, w2, u_out=u2, v_out=v2, w_out=w2)
    for x, y in zip((u2, v2, w2, p_in), a[:4]):
        assert torch.equal(x, y)
    assert abs(rep_in["max_div_rel"] - a[4]["max_div_rel"]) <= 1e-3 * a[4]["max_div_rel"] + 1e-18
    _say(f"deterministic; in place identical; div {rep_in['max_div_rel']:.2e}")


@pytest.mark.parametrize("bc,stretch", [((0, 0, 1), 1.8), ((0, 0, 0), 0.0), ((1, 1, 1), 1.8)])
def test_512_manufactured_fixed_point(pcx, bc, stretch):
    """p* = q and u* = u_df + dt G q / rho_face on the 512^3 bubble density:
    the exact step returns p = q and u_out = u_df."""
    import torch
    n = 512
    g = W.GridSpec(n, n, n, 2 * np.pi, 2 * np.pi, W.zf_tanh(n, 2.0, 1.8) if stretch else W.zf_uniform(n, 2.0),
                   *bc)
    rng = np.random.Generator(np.random.PCG64(77))
    bub = W.place_bubbles(rng, g, [8 * g.dx] * 512)
    rho = torch.from_numpy(1000.0 + (1.0 - 1000.0) * W.phase_field(g, bub)).to("cuda")
    rho0 = float(rho.min())
    dt = (8 / 15) * 0.5 * min(g.dx, float(np.diff(g.zf).min()))
    _say(f"512^3 fixed point bc={bc}: building inputs on the GPU")
    ps, us, vs, ws, q, ud, vd, wd = M.fixed_point_inputs_torch(1234 + bc[0] + 2 * bc[2], g, rho, dt)
    for prec, tol in (("fp64", 1e-12), ("fp32_refined", 1e-10)):
        plan = pcx.Plan(g, prec)
        uo, vo, wo, p, rep = plan.step(dt, rho0, rho, ps, us, vs, ws)
        torch.cuda.synchronize()
        ep = M.relerr_t(p, q)
        vmax = max(float(ud.abs().max()), float(vd.abs().max()), float(wd.abs().max()))
        eu = max(float((o - r).abs().max()) for o, r in ((uo, ud), (vo, vd), (wo, wd))) / vmax
        _say(f"  {prec}: |p-q|/|q| {ep:.2e}  |u-u_df|/|u_df| {eu:.2e}  div {rep['max_div_rel']:.2e} "
             f"solves {rep['solves']}")
        assert ep <= tol and eu <= tol and rep["max_div_rel"] <= tol
        del uo, vo, wo, p
        plan.close()
