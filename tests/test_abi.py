"""C-ABI library checks that need no GPU: the library loads, exports every
function include/pcx.h declares, validates descriptors on the host and
reports a missing device as PCX_ERR_HIP."""
import ctypes as C

import numpy as np
import pytest

from paper_2502_04189_amd import pcx as P
from paper_2502_04189_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    return P.lib()


def test_exports_every_declared_symbol(L):
    syms = P.header_symbols()
    assert len(syms) >= 15
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert L.pcx_abi_version() == 1


def test_status_strings(L):
    for s in range(7):
        assert L.pcx_status_str(s).decode().startswith("PCX_")


def _create(L, gs, opts=None):
    g = P.make_grid(gs)
    h = C.c_void_p()
    st = L.pcx_plan_create(C.byref(g), C.byref(opts) if opts is not None else None, C.byref(h))
    if st == 0:
        L.pcx_plan_destroy(h)
    return st


def test_descriptor_validation(L):
    ok = W.GridSpec(32, 32, 16, 1.0, 1.0, W.zf_uniform(16, 1.0))
    bad_z = ok.zf.copy()
    bad_z[5] = bad_z[4]
    cases = [
        (W.GridSpec(1, 32, 16, 1.0, 1.0, ok.zf), P.PCX_ERR_INVALID),
        (W.GridSpec(32, 32, 16, 0.0, 1.0, ok.zf), P.PCX_ERR_INVALID),
        (W.GridSpec(31, 32, 16, 1.0, 1.0, ok.zf), P.PCX_ERR_INVALID),      # odd periodic nx
        (W.GridSpec(27, 32, 16, 1.0, 1.0, ok.zf, 1, 0, 1), P.PCX_ERR_INVALID),  # odd walled nx
        (W.GridSpec(32, 27, 16, 1.0, 1.0, ok.zf, 0, 0, 1), P.PCX_ERR_INVALID),  # odd periodic ny
        (W.GridSpec(32, 32, 16, 1.0, 1.0, bad_z), P.PCX_ERR_INVALID),      # non-increasing zf
        (W.GridSpec(32, 32, 16, 1.0, 1.0, ok.zf, 0, 0, 7), P.PCX_ERR_INVALID),
        (W.GridSpec(40, 32, 16, 1.0, 1.0, ok.zf), P.PCX_ERR_UNSUPPORTED),  # 40 = 2^3 5
        (W.GridSpec(8192, 32, 16, 1.0, 1.0, ok.zf), P.PCX_ERR_UNSUPPORTED),
        (W.GridSpec(32, 32, 2048, 1.0, 1.0, W.zf_uniform(2048, 1.0)), P.PCX_ERR_UNSUPPORTED),
    ]
    for gs, want in cases:
        assert _create(L, gs) == want, (gs.nx, gs.ny, gs.nz)
    assert "must" in L.pcx_last_error().decode() or "support" in L.pcx_last_error().decode()
    h = C.c_void_p()
    assert L.pcx_plan_create(None, None, C.byref(h)) == P.PCX_ERR_INVALID
    assert L.pcx_step(None, 1.0, 1.0, *([None] * 9), None, None) == P.PCX_ERR_INVALID


def test_cell_count_limit(L):
    """Cell offsets in the kernels are 32-bit: a grid of 2^31 cells or more
    is rejected as UNSUPPORTED before any device work (checked here without a
    GPU: a grid just below the limit passes validation and then reports the
    missing device, or is created when a GPU is present)."""
    import torch
    big = W.GridSpec(2048, 2048, 512, 1.0, 1.0, W.zf_uniform(512, 1.0))
    assert _create(L, big) == P.PCX_ERR_UNSUPPORTED
    assert "2^31" in L.pcx_last_error().decode()
    big_wall = W.GridSpec(4096, 1024, 512, 1.0, 1.0, W.zf_uniform(512, 1.0), 1, 1, 1)
    assert _create(L, big_wall) == P.PCX_ERR_UNSUPPORTED
    if not torch.cuda.is_available():
        under = W.GridSpec(2048, 2048, 511, 1.0, 1.0, W.zf_uniform(511, 1.0))
        assert _create(L, under) == P.PCX_ERR_HIP


def test_missing_device_is_hip_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    gs = W.GridSpec(32, 32, 16, 1.0, 1.0, W.zf_uniform(16, 1.0))
    assert _create(L, gs) == P.PCX_ERR_HIP
    assert "device" in L.pcx_last_error().decode()


def test_refine_stop_logic(L):
    """Host stop test on fake residual/update sequences: the residual must be
    within rtol and the error left after the last update, estimated from the
    observed contraction q = |e_s|/|e_s-1| as q |e_s| / (1 - q), must be below
    0.1 rtol |p|."""
    rtol = 1e-10
    # (rel_residual, |e_s|, |e_s-1|) with |p| = 1
    seq = [(4e-6, 1.0, 0.0),        # first solve: no rate yet
           (2e-11, 1e-4, 1.0),      # residual fine, but q |e| = 1e-8 left
           (2e-11, 1e-8, 1e-4),     # q = 1e-4: about 1e-12 left -> stop
           (5e-10, 1e-12, 1e-8),    # residual above rtol
           (1e-12, 9e-9, 1e-8)]     # q = 0.9: about 8e-8 left
    got = [L.pcx_refine_should_stop(r, e, ep, 1.0, rtol) for r, e, ep in seq]
    assert got == [0, 0, 1, 0, 0]
    assert L.pcx_refine_should_stop(float("nan"), 0.0, 1.0, 1.0, rtol) == 0
    assert L.pcx_refine_should_stop(1e-12, 2.0, 1.0, 1.0, rtol) == 0     # diverging


def test_noalloc_sizes_and_rejections(L):
    """The allocation-free step: scratch need of the stated sizes, and the
    host-side rejections that come before any device call."""
    fits = W.GridSpec(128, 128, 128, 1.0, 1.0, W.zf_uniform(128, 1.0))
    big = W.GridSpec(256, 256, 256, 1.0, 1.0, W.zf_uniform(256, 1.0))
    cap = 64 << 20
    for prec in ("fp64", "fp32_refined"):
        assert 0 < P.noalloc_scratch_need(fits, prec) <= cap
        assert P.noalloc_scratch_need(big, prec) > cap
    # a grid beyond the array: UNSUPPORTED before any device call (this
    # host has no GPU; the dummy pointers are never dereferenced)
    dummy = [C.c_void_p(4096 * (i + 1)) for i in range(9)]
    g = P.make_grid(big)
    o = P.make_options("fp64")
    st = L.pcx_step_noalloc(C.byref(g), C.byref(o), 1e-3, 1.0, *dummy, None, None)
    assert st == P.PCX_ERR_UNSUPPORTED
    assert "scratch" in L.pcx_last_error().decode()
    o = P.make_options("fp64", autotune=True)
    g = P.make_grid(fits)
    assert L.pcx_step_noalloc(C.byref(g), C.byref(o), 1e-3, 1.0, *dummy, None, None) == P.PCX_ERR_INVALID
    bad = W.GridSpec(40, 32, 16, 1.0, 1.0, W.zf_uniform(16, 1.0))
    g = P.make_grid(bad)
    o = P.make_options("fp64")
    assert L.pcx_step_noalloc(C.byref(g), C.byref(o), 1e-3, 1.0, *dummy, None, None) == P.PCX_ERR_UNSUPPORTED


def test_flow_create_validation(L):
    """pcx_flow_create rejects bad parameters on the host and reports a
    missing device; the substep entry points reject NULL flows."""
    gs = W.GridSpec(16, 16, 8, 1.0, 1.0, W.zf_uniform(8, 0.5))
    g = P.make_grid(gs)
    good = P.PcxFlowParams(1000.0, 1.0, 1e-2, 1e-4, 0.07, 0.0, 0.0, -9.81, 1.0, 0.04, 1e-100)
    h = C.c_void_p()
    inf = float("inf")
    for field, bad in (("rho1", 0.0), ("mu2", -1.0), ("eps", 0.0), ("gamma", -1.0), ("gz", float("nan")),
                       ("eps_s", -1e-3), ("eps_s", inf), ("sigma", inf), ("rho2", inf)):
        p = P.PcxFlowParams(*[getattr(good, f) for f, _ in P.PcxFlowParams._fields_])
        setattr(p, field, bad)
        assert L.pcx_flow_create(C.byref(g), C.byref(p), None, C.byref(h)) == P.PCX_ERR_INVALID, field
    assert L.pcx_flow_create(C.byref(g), None, None, C.byref(h)) == P.PCX_ERR_INVALID
    st = L.pcx_flow_create(C.byref(g), C.byref(good), None, C.byref(h))
    assert st in (P.PCX_OK, P.PCX_ERR_HIP)
    if st == P.PCX_OK:
        L.pcx_flow_destroy(h)
    assert L.pcx_flow_phase_rhs(None, *[None] * 5, None) == P.PCX_ERR_INVALID


def test_varcoef_create_validation(L):
    """pcx_varcoef_create rejects a Dirichlet grid and a non-FP64 precision on
    the host and reports a missing device; the entry points reject NULL."""
    h = C.c_void_p()
    dg = P.make_grid(W.GridSpec(16, 16, 8, 1.0, 1.0, W.zf_uniform(8, 0.5), 2, 0, 1))
    assert L.pcx_varcoef_create(C.byref(dg), None, C.byref(h)) == P.PCX_ERR_UNSUPPORTED
    g = P.make_grid(W.GridSpec(16, 16, 8, 1.0, 1.0, W.zf_uniform(8, 0.5)))
    o = P.make_options("fp32_refined")
    assert L.pcx_varcoef_create(C.byref(g), C.byref(o), C.byref(h)) == P.PCX_ERR_UNSUPPORTED
    assert L.pcx_varcoef_create(C.byref(g), None, None) == P.PCX_ERR_INVALID
    st = L.pcx_varcoef_create(C.byref(g), None, C.byref(h))
    assert st in (P.PCX_OK, P.PCX_ERR_HIP)
    if st == P.PCX_OK:
        L.pcx_varcoef_destroy(h)
    assert L.pcx_varcoef_apply(None, None, None, None, None) == P.PCX_ERR_INVALID
    it, rr = C.c_int32(), C.c_double()
    assert L.pcx_varcoef_project(None, 1.0, 1.0, *[None] * 4, 1e-12, 10, *[None] * 4, None, C.byref(it),
                                 C.byref(rr)) == P.PCX_ERR_INVALID


def test_flow_predict_rejects_null(L):
    """pcx_flow_predict rejects a NULL flow on the host."""
    r0, dt = C.c_double(), C.c_double()
    assert L.pcx_flow_predict(None, 1, 1e-3, *[None] * 6, 0.0, *[None] * 10, C.byref(r0), C.byref(dt),
                              None) == P.PCX_ERR_INVALID
