"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (max-norm relative error per field): FP64 path 1e-12; FP32 with
FP64 refinement 1e-10; relative post-correction divergence likewise.
"""
import sys

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


def _oracle(orc, case):
    g = orc.Grid.from_workload(case.grid)
    uo, vo, wo, p, d = orc.step(g, case.dt, case.rho0, *case.fields())
    return [uo, vo, wo, p], d


def test_config0_fp64(pcx, orc):
    case = W.config0()
    _say("case config0 fp64 32^3")
    plan = pcx.Plan(case.grid, "fp64")
    got, rep = run_plan(plan, case)
    ref, d = _oracle(orc, case)
    e = errors(got, ref)
    _say(f"errors {e} report {rep}")
    assert max(e.values()) <= FP64_TOL
    assert rep["max_div_rel"] <= FP64_TOL
    check_div(orc, case, got, rep, case.name)
    assert abs(rep["mean_p"]) <= 1e-13 * np.abs(ref[3]).max()
    assert np.all(got[2][-1] == 0.0)


SMALL = [
    ((48, 36, 20), (0, 0, 1), 1.8),
    ((64, 96, 33), (0, 0, 0), 0.0),
    ((96, 48, 64), (0, 0, 1), 1.2),
    ((6, 4, 5), (0, 0, 1), 1.5),
    ((8, 8, 3), (0, 0, 0), 0.0),
    ((2, 2, 2), (0, 0, 1), 0.0),
    ((24, 18, 7), (0, 0, 0), 1.1),
    ((128, 32, 96), (0, 0, 0), 0.0),
    # wall x and/or y: cosine transforms in the walled directions
    ((48, 36, 20), (1, 0, 1), 1.8),
    ((32, 48, 17), (0, 1, 0), 0.0),
    ((64, 54, 24), (1, 1, 1), 1.2),
    ((96, 64, 33), (1, 1, 0), 0.0),
    ((6, 9, 5), (1, 1, 1), 0.0),
    ((2, 3, 2), (1, 1, 0), 0.0),
    ((24, 27, 7), (0, 1, 1), 1.1),
    ((96, 162, 5), (1, 1, 0), 0.0),
    ((96, 18, 9), (0, 0, 1), 1.4),
    # wave-level FFT paths: x half length 256 and y length 256 (4.4.4.4),
    # y length 512 (8.8.8); z both on and off the full-chunk fast path
    ((512, 256, 12), (0, 0, 1), 1.3),
    ((512, 512, 8), (0, 0, 0), 0.0),
    # narrow and tall: the stencil halos outnumber the threads (two items each)
    ((4, 192, 6), (0, 0, 1), 1.2),
    ((6, 144, 4), (1, 1, 0), 0.0),
]


@pytest.mark.parametrize("dims,bc,stretch", SMALL)
def test_small_fp64(pcx, orc, dims, bc, stretch):
    case = W.random_case(3 + sum(dims), *dims, *bc, stretch=stretch)
    _say(f"case {case.name} fp64")
    plan = pcx.Plan(case.grid, "fp64")
    got, rep = run_plan(plan, case)
    ref, d = _oracle(orc, case)
    e = errors(got, ref)
    _say(f"errors {e} div {rep['max_div_rel']:.3e}")
    assert max(e.values()) <= FP64_TOL
    assert rep["max_div_rel"] <= FP64_TOL
    check_div(orc, case, got, rep, case.name)
    # the FP64 solve stores p itself as the update: the wave and workgroup
    # maxima of the x inverse must give max |p| exactly
    assert rep["last_update_inf"] == np.abs(got[3]).max()


@pytest.mark.parametrize("dims,bc,stretch", [((32, 32, 32), (0, 0, 1), 0.0), ((48, 36, 20), (0, 0, 1), 1.8),
                                             ((64, 96, 33), (0, 0, 0), 0.0),
                                             ((64, 48, 40), (1, 1, 1), 1.5),
                                             # partial stencil tiles in x and y (last tiles of 32 and 2)
                                             ((64, 18, 12), (0, 0, 1), 1.3), ((96, 162, 5), (1, 1, 0), 0.0),
                                             # wave-level FFT paths in FP32 (x half length and y length 256)
                                             ((512, 256, 16), (0, 0, 1), 1.2)])
def test_small_refined(pcx, orc, dims, bc, stretch):
    case = W.config0() if dims == (32, 32, 32) else W.random_case(5 + sum(dims), *dims, *bc, stretch=stretch)
    _say(f"case {case.name} fp32_refined")
    plan = pcx.Plan(case.grid, "fp32_refined")
    got, rep = run_plan(plan, case)
    ref, d = _oracle(orc, case)
    e = errors(got, ref)
    _say(f"errors {e} report {rep}")
    assert rep["converged"] == 1
    assert max(e.values()) <= REF_TOL
    assert rep["max_div_rel"] <= REF_TOL
    check_div(orc, case, got, rep, case.name)


@pytest.mark.parametrize("dims,ndrops,kmax", [((64, 64, 32), 6, 8.0), ((96, 96, 48), 12, 12.0)])
def test_emulsion_small(pcx, orc, dims, ndrops, kmax):
    """The triply periodic emulsion recipe (k^-5/3 solenoidal velocity,
    density ratio 10) at sizes the oracle runs in seconds, both forms."""
    case = W.emulsion(*dims, ndrops, 31 + dims[0], f"emulsion_{dims}", kmax=kmax)
    ref, d = _oracle(orc, case)
    for prec, tol in (("fp64", FP64_TOL), ("fp32_refined", REF_TOL)):
        _say(f"case {case.name} {prec}")
        plan = pcx.Plan(case.grid, prec)
        got, rep = run_plan(plan, case)
        e = errors(got, ref)
        _say(f"errors {e} div {rep['max_div_rel']:.3e} solves {rep['solves']}")
        assert max(e.values()) <= tol
        assert rep["max_div_rel"] <= tol
        check_div(orc, case, got, rep, case.name)
