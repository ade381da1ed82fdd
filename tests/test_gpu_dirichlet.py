"""GPU parity of the plan's Poisson solve (pcx_poisson_solve) with
homogeneous Dirichlet directions (sine transforms through the cosine path
with alternating signs) against the explicit-eigenvector oracle
(oracle/dirichlet.c), and with periodic / wall directions against the
step oracle's solve (oracle.c).  FP64, max-norm error relative to max |p|
within 1e-12; the step and the refined solve reject Dirichlet plans."""
import sys

import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


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


CASES = [
    ((32, 24, 12), (2, 0, 1), 1.3),
    ((24, 18, 10), (0, 2, 0), 0.0),
    ((16, 12, 8), (2, 2, 2), 1.2),
    ((32, 27, 9), (1, 2, 2), 0.0),
    ((48, 16, 7), (2, 1, 0), 0.0),
    ((6, 9, 4), (2, 2, 1), 0.0),
    # wave-level FFT paths: x half length 256 with a Dirichlet x, y length 256 with a Dirichlet y
    ((512, 12, 6), (2, 0, 1), 1.1),
    ((16, 256, 4), (0, 2, 0), 0.0),
]


def _grid(dims, bc, stretch):
    nx, ny, nz = dims
    zf = W.zf_tanh(nz, 0.9, stretch) if stretch > 0 else W.zf_uniform(nz, 0.9)
    return W.GridSpec(nx, ny, nz, 1.0, 0.8, zf, *bc)


@pytest.mark.parametrize("dims,bc,stretch", CASES)
def test_dirichlet_solve_vs_oracle(pcx, orc, dims, bc, stretch):
    gs = _grid(dims, bc, stretch)
    f = np.random.default_rng(sum(dims)).normal(size=gs.shape)
    ref = orc.poisson_bc(orc.Grid.from_workload(gs), f)
    plan = pcx.Plan(gs, "fp64")
    p = plan.poisson_solve(to_dev(f)).cpu().numpy()
    plan.close()
    e = float(np.abs(p - ref).max() / np.abs(ref).max())
    _say(f"dirichlet {dims} bc {bc}: max rel error {e:.2e}")
    assert e <= TOL


@pytest.mark.parametrize("dims,bc", [((32, 24, 12), (0, 0, 1)), ((24, 18, 10), (1, 1, 0)), ((16, 12, 8), (0, 1, 1))])
def test_poisson_solve_without_dirichlet_vs_step_oracle(pcx, orc, dims, bc):
    gs = _grid(dims, bc, 1.2)
    f = np.random.default_rng(7).normal(size=gs.shape)
    ref = orc.poisson(orc.Grid.from_workload(gs), f)
    plan = pcx.Plan(gs, "fp64")
    p = plan.poisson_solve(to_dev(f)).cpu().numpy()
    plan.close()
    e = float(np.abs(p - ref).max() / np.abs(ref).max())
    _say(f"neumann/periodic {dims} bc {bc}: max rel error {e:.2e}")
    assert e <= TOL


def test_dirichlet_plans_reject_the_step_and_refined_solve(pcx):
    import torch
    gs = _grid((16, 12, 8), (2, 0, 1), 0.0)
    plan = pcx.Plan(gs, "fp64")
    z = [torch.zeros(gs.shape, dtype=torch.float64, device="cuda") for _ in range(5)]
    z[0] += 1.0
    with pytest.raises(pcx.PcxError) as e:
        plan.step(1e-3, 1.0, *z)
    assert e.value.status == pcx.PCX_ERR_UNSUPPORTED
    plan.close()
    rplan = pcx.Plan(gs, "fp32_refined")
    with pytest.raises(pcx.PcxError) as e:
        rplan.poisson_solve(z[1])
    assert e.value.status == pcx.PCX_ERR_UNSUPPORTED
    rplan.close()


@pytest.mark.parametrize("bc", [(0, 0, 1), (2, 2, 1)], ids=["periodic_xy", "dirichlet_xy"])
def test_solve_at_512_residual(pcx, orc, bc):
    """pcx_poisson_solve on the benchmark's 512^3 grid (tanh z, walls in z)
    as bench.py times it, with its x/y boundaries and with Dirichlet x and
    y: the oracle's operator applied to the GPU's p gives back f (minus its
    volume mean where the problem is singular).  A direct transform solve is
    backward stable: the residual is bounded by a modest multiple of
    eps ||L||inf ||p||inf (||L||inf: the largest absolute row sum of the
    7-point operator); 64 allows for the log2 n stages of each transform."""
    import torch
    gs0 = W.config3().grid
    gs = W.GridSpec(gs0.nx, gs0.ny, gs0.nz, gs0.lx, gs0.ly, gs0.zf, *bc)
    f = np.random.default_rng(512).normal(size=gs.shape)
    plan = pcx.Plan(gs, "fp64")
    p = plan.poisson_solve(to_dev(f)).cpu().numpy()
    plan.close()
    torch.cuda.synchronize()
    g = orc.Grid.from_workload(gs)
    lp = orc.apply_L_bc(g, p)
    want = f if 2 in bc else f - orc.volume_mean(g, f)
    dzf = np.diff(gs.zf)
    dzc = 0.5 * (dzf[:-1] + dzf[1:])
    lo = np.concatenate([[dzf[0]], dzc])
    hi = np.concatenate([dzc, [dzf[-1]]])
    linf = 4.0 / gs.dx ** 2 + 4.0 / gs.dy ** 2 + float(np.max(2.0 * (1.0 / lo + 1.0 / hi) / dzf))
    r = float(np.abs(lp - want).max())
    bound = 64 * np.finfo(np.float64).eps * linf * float(np.abs(p).max())
    _say(f"512^3 solve bc {bc}: max|L p - f| = {r:.2e} ({r / np.abs(f).max():.2e} of max|f|), "
         f"{r / bound * 64:.1f} eps ||L|| ||p||")
    assert r <= bound
