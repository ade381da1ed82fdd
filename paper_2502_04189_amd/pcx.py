"""Python binding of libpcx (ctypes).  Argument marshalling only: every pass
of the step runs in the HIP library; torch provides device memory and
streams.  Raises ImportError when the library has not been built."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pcx.h")
HEADERS = [HEADER] + [os.path.join(os.path.dirname(HERE), "include", h) for h in ("pcx_flow.h", "pcx_varcoef.h")]

PCX_OK, PCX_ERR_INVALID, PCX_ERR_UNSUPPORTED, PCX_ERR_NOMEM, PCX_ERR_HIP = 0, 1, 2, 3, 4
PCX_ERR_NOT_CONVERGED, PCX_ERR_NONFINITE = 5, 6
PCX_FP64, PCX_FP32_REFINED = 0, 1
PCX_BC_PERIODIC, PCX_BC_WALL, PCX_BC_DIRICHLET = 0, 1, 2

_DP = C.POINTER(C.c_double)


class PcxGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("zf", _DP),
                ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("bc_z", C.c_int32)]


class PcxOptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rtol", C.c_double), ("max_iters", C.c_int32),
                ("fixed_iters", C.c_int32), ("check_finite", C.c_int32), ("autotune", C.c_int32),
                ("tune_cache", C.c_char_p)]


class PcxReport(C.Structure):
    _fields_ = [("solves", C.c_int32), ("converged", C.c_int32), ("f_inf", C.c_double),
                ("rel_residual", C.c_double), ("max_div_abs", C.c_double),
                ("max_div_rel", C.c_double), ("mean_p", C.c_double),
                ("last_update_inf", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PcxFlowParams(C.Structure):
    _fields_ = [("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double),
                ("sigma", C.c_double), ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
                ("gamma", C.c_double), ("eps", C.c_double), ("eps_s", C.c_double)]


class PcxDomain(C.Structure):
    _fields_ = [("grid", PcxGrid), ("dt", C.c_double), ("rho0", C.c_double),
                ("rho", C.c_void_p), ("p_star", C.c_void_p), ("u", C.c_void_p),
                ("v", C.c_void_p), ("w", C.c_void_p), ("u_out", C.c_void_p),
                ("v_out", C.c_void_p), ("w_out", C.c_void_p), ("p_out", C.c_void_p)]


_lib = None


def header_symbols():
    """Function names declared in the library's headers (include/*.h)."""
    txt = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"\b(pcx_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpcx.so is not built ({LIB_PATH}); run paper_2502_04189_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    st = C.c_int
    sig = {
        "pcx_plan_create": (st, [C.POINTER(PcxGrid), C.POINTER(PcxOptions), C.POINTER(vp)]),
        "pcx_plan_workspace_bytes": (st, [vp, C.POINTER(C.c_size_t)]),
        "pcx_step": (st, [vp, dbl, dbl] + [vp] * 9 + [vp, C.POINTER(PcxReport)]),
        "pcx_plan_destroy": (st, [vp]),
        "pcx_plan_set_timing": (st, [vp, i32]),
        "pcx_plan_pass_times": (st, [vp, _DP, i32, C.POINTER(i32)]),
        "pcx_plan_pass_name": (C.c_char_p, [vp, i32]),
        "pcx_batch_create": (st, [C.POINTER(PcxDomain), i32, C.POINTER(PcxOptions), vp, C.POINTER(vp)]),
        "pcx_batch_launch": (st, [vp, vp]),
        "pcx_batch_reports": (st, [vp, C.POINTER(PcxReport)]),
        "pcx_batch_destroy": (st, [vp]),
        "pcx_rho_min": (st, [vp, C.c_int64, vp, _DP]),
        "pcx_poisson_solve": (st, [vp, vp, vp, vp]),
        "pcx_step_noalloc": (st, [C.POINTER(PcxGrid), C.POINTER(PcxOptions), dbl, dbl] + [vp] * 9 +
                             [vp, C.POINTER(PcxReport)]),
        "pcx_noalloc_scratch_need": (st, [C.POINTER(PcxGrid), C.POINTER(PcxOptions), C.POINTER(C.c_size_t)]),
        "pcx_flow_create": (st, [C.POINTER(PcxGrid), C.POINTER(PcxFlowParams), C.POINTER(PcxOptions), C.POINTER(vp)]),
        "pcx_flow_destroy": (st, [vp]),
        "pcx_flow_phase_rhs": (st, [vp] + [vp] * 5 + [vp]),
        "pcx_flow_momentum_rhs": (st, [vp] + [vp] * 7 + [vp]),
        "pcx_flow_substep": (st, [vp, i32, dbl] + [vp] * 6 + [dbl] + [vp] * 9 + [vp, C.POINTER(PcxReport)]),
        "pcx_flow_predict": (st, [vp, i32, dbl] + [vp] * 6 + [dbl] + [vp] * 10 + [_DP, _DP, vp]),
        "pcx_varcoef_create": (st, [C.POINTER(PcxGrid), C.POINTER(PcxOptions), C.POINTER(vp)]),
        "pcx_varcoef_destroy": (st, [vp]),
        "pcx_varcoef_apply": (st, [vp, vp, vp, vp, vp]),
        "pcx_varcoef_project": (st, [vp, dbl, dbl] + [vp] * 4 + [dbl, i32] + [vp] * 4 +
                                [vp, C.POINTER(i32), _DP]),
        "pcx_refine_should_stop": (i32, [dbl, dbl, dbl, dbl, dbl]),
        "pcx_status_str": (C.c_char_p, [st]),
        "pcx_last_error": (C.c_char_p, []),
        "pcx_abi_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
    _lib = L
    return L


class PcxError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        msg = L.pcx_last_error().decode()
        super().__init__(f"{where}: {L.pcx_status_str(status).decode()}: {msg}")
        self.status = status


def _check(status, where):
    if status != PCX_OK:
        raise PcxError(status, where)


def make_grid(gs):
    """pcx_grid from a workloads.GridSpec (keeps zf alive on the struct)."""
    import numpy as np
    zf = np.ascontiguousarray(gs.zf, dtype=np.float64)
    g = PcxGrid(gs.nx, gs.ny, gs.nz, gs.lx, gs.ly, zf.ctypes.data_as(_DP), gs.bcx, gs.bcy, gs.bcz)
    g._zf_keep = zf
    return g


def make_options(precision="fp64", rtol=1e-10, max_iters=8, fixed_iters=0, check_finite=False,
                 autotune=False, tune_cache=None):
    p = PCX_FP64 if precision in ("fp64", PCX_FP64) else PCX_FP32_REFINED
    return PcxOptions(p, rtol, max_iters, fixed_iters, 1 if check_finite else 0, 1 if autotune else 0,
                      tune_cache.encode() if tune_cache else None)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


class Plan:
    """pcx_plan for one grid.  step() takes torch float64 CUDA tensors of
    shape (nz, ny, nx)."""

    def __init__(self, grid, precision="fp64", rtol=1e-10, max_iters=8, fixed_iters=0, check_finite=False,
                 autotune=False, tune_cache=None):
        L = lib()
        self.gs = grid
        self._g = make_grid(grid)
        self._o = make_options(precision, rtol, max_iters, fixed_iters, check_finite, autotune, tune_cache)
        h = C.c_void_p()
        _check(L.pcx_plan_create(C.byref(self._g), C.byref(self._o), C.byref(h)), "pcx_plan_create")
        self._L = L
        self._h = h
        self.shape = (grid.nz, grid.ny, grid.nx)

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcx_plan_destroy(self._h)  # the library handle outlives module teardown
            self._h = None

    __del__ = close

    def workspace_bytes(self):
        n = C.c_size_t()
        _check(lib().pcx_plan_workspace_bytes(self._h, C.byref(n)), "pcx_plan_workspace_bytes")
        return n.value

    def step(self, dt, rho0, rho, pstar, u, v, w, u_out=None, v_out=None, w_out=None, p_out=None,
             stream=None, report=True, raise_on_status=True):
        import torch
        sh = self.shape
        outs = []
        for o in (u_out, v_out, w_out, p_out):
            outs.append(o if o is not None else torch.empty(sh, dtype=torch.float64, device=rho.device))
        ptrs = [_ptr(t, sh, n) for t, n in zip((rho, pstar, u, v, w) + tuple(outs),
                                               ("rho", "pstar", "u", "v", "w", "u_out", "v_out", "w_out", "p_out"))]
        rep = PcxReport()
        st = lib().pcx_step(self._h, float(dt), float(rho0), *ptrs, _stream_handle(stream),
                            C.byref(rep) if report else None)
        self.last_status = st
        if raise_on_status and st != PCX_OK:
            raise PcxError(st, "pcx_step")
        return outs[0], outs[1], outs[2], outs[3], (rep.as_dict() if report else None)

    def poisson_solve(self, f, p=None, stream=None):
        """pcx_poisson_solve: L p = f with the plan's boundary conditions."""
        import torch
        p = p if p is not None else torch.empty(self.shape, dtype=torch.float64, device=f.device)
        _check(lib().pcx_poisson_solve(self._h, _ptr(f, self.shape, "f"), _ptr(p, self.shape, "p"),
                                       _stream_handle(stream)), "pcx_poisson_solve")
        return p

    def set_timing(self, on=True, correction_only=False):
        mode = (2 if correction_only else 1) if on else 0
        _check(lib().pcx_plan_set_timing(self._h, mode), "pcx_plan_set_timing")

    def pass_times(self, cap=4096):
        """(pass name, ms) of every pass of every step since set_timing()."""
        buf = (C.c_double * cap)()
        n = C.c_int32()
        _check(lib().pcx_plan_pass_times(self._h, buf, cap, C.byref(n)), "pcx_plan_pass_times")
        return [(lib().pcx_plan_pass_name(self._h, i).decode(), buf[i]) for i in range(min(n.value, cap))]


def noalloc_scratch_need(grid, precision="fp64"):
    """Device bytes pcx_step_noalloc needs for `grid` (host-only)."""
    g = make_grid(grid)
    o = make_options(precision)
    n = C.c_size_t()
    _check(lib().pcx_noalloc_scratch_need(C.byref(g), C.byref(o), C.byref(n)), "pcx_noalloc_scratch_need")
    return n.value


def step_noalloc(grid, dt, rho0, rho, pstar, u, v, w, u_out, v_out, w_out, p_out, precision="fp64",
                 rtol=1e-10, max_iters=8, fixed_iters=0, check_finite=False, stream=None, report=True):
    """pcx_step_noalloc: one step with the library's fixed device scratch array
    (no device allocation).  Outputs are caller tensors; returns (status,
    report dict or None)."""
    g = make_grid(grid)
    o = make_options(precision, rtol, max_iters, fixed_iters, check_finite)
    sh = (grid.nz, grid.ny, grid.nx)
    ptrs = [_ptr(t, sh, n) for t, n in zip((rho, pstar, u, v, w, u_out, v_out, w_out, p_out),
                                           ("rho", "pstar", "u", "v", "w", "u_out", "v_out", "w_out", "p_out"))]
    rep = PcxReport()
    st = lib().pcx_step_noalloc(C.byref(g), C.byref(o), float(dt), float(rho0), *ptrs, _stream_handle(stream),
                                C.byref(rep) if report else None)
    return st, (rep.as_dict() if report else None)


class Batch:
    """pcx_batch over a list of (GridSpec, dt, rho0, tensors...) domains."""

    def __init__(self, domains, precision="fp32_refined", rtol=1e-10, max_iters=8, fixed_iters=0,
                 stream=None, autotune=False, tune_cache=None):
        L = lib()
        self._keep = []
        arr = (PcxDomain * len(domains))()
        for i, d in enumerate(domains):
            g = make_grid(d["grid"])
            self._keep.append(g)
            sh = (d["grid"].nz, d["grid"].ny, d["grid"].nx)
            names = ("rho", "pstar", "u", "v", "w", "u_out", "v_out", "w_out", "p_out")
            ptrs = [_ptr(d[n], sh, n).value for n in names]
            arr[i] = PcxDomain(g, float(d["dt"]), float(d["rho0"]), *ptrs)
        self._arr = arr
        self._o = make_options(precision, rtol, max_iters, fixed_iters, False, autotune, tune_cache)
        h = C.c_void_p()
        _check(L.pcx_batch_create(arr, len(domains), C.byref(self._o), _stream_handle(stream), C.byref(h)),
               "pcx_batch_create")
        self._L = L
        self._h = h
        self.n = len(domains)

    def launch(self, stream=None):
        _check(lib().pcx_batch_launch(self._h, _stream_handle(stream)), "pcx_batch_launch")

    def reports(self, raise_on_status=False):
        reps = (PcxReport * self.n)()
        st = lib().pcx_batch_reports(self._h, reps)
        if raise_on_status or st not in (PCX_OK, PCX_ERR_NOT_CONVERGED):
            _check(st, "pcx_batch_reports")
        return [r.as_dict() for r in reps], st

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcx_batch_destroy(self._h)  # the library handle outlives module teardown
            self._h = None

    __del__ = close


def batch_tune_cache_path():
    """Tune cache of the batch's size classes, kept between runs on one
    machine (the benchmark and the GPU tests use the same file)."""
    import tempfile
    return os.path.join(tempfile.gettempdir(), "pcx_batch_tune_cache.txt")


def rho_min(rho, stream=None):
    out = C.c_double()
    _check(lib().pcx_rho_min(C.c_void_p(rho.data_ptr()), rho.numel(), _stream_handle(stream), C.byref(out)),
           "pcx_rho_min")
    return out.value


class Flow:
    """pcx_flow: the Runge-Kutta substep around the pressure correction on
    one grid.  Fields are torch float64 CUDA tensors of shape (nz, ny, nx)."""

    def __init__(self, grid, rho1, rho2, mu1, mu2, sigma=0.0, g=(0.0, 0.0, 0.0), gamma=1.0, eps=None,
                 eps_s=1e-100, precision="fp64"):
        L = lib()
        self.gs = grid
        self._g = make_grid(grid)
        if eps is None:
            eps = 0.51 * grid.lx / grid.nx
        self._p = PcxFlowParams(rho1, rho2, mu1, mu2, sigma, g[0], g[1], g[2], gamma, eps, eps_s)
        self._o = make_options(precision)
        h = C.c_void_p()
        _check(L.pcx_flow_create(C.byref(self._g), C.byref(self._p), C.byref(self._o), C.byref(h)),
               "pcx_flow_create")
        self._L = L
        self._h = h
        self.shape = (grid.nz, grid.ny, grid.nx)

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcx_flow_destroy(self._h)  # the library handle outlives module teardown
            self._h = None

    __del__ = close

    def _ptrs(self, ts, names):
        return [_ptr(t, self.shape, n) for t, n in zip(ts, names)]

    def phase_rhs(self, phi, u, v, w, out=None, stream=None):
        import torch
        out = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=phi.device)
        p = self._ptrs((phi, u, v, w, out), ("phi", "u", "v", "w", "rhs"))
        _check(lib().pcx_flow_phase_rhs(self._h, *p, _stream_handle(stream)), "pcx_flow_phase_rhs")
        return out

    def momentum_rhs(self, phi, u, v, w, stream=None):
        import torch
        outs = [torch.empty(self.shape, dtype=torch.float64, device=phi.device) for _ in range(3)]
        p = self._ptrs((phi, u, v, w, *outs), ("phi", "u", "v", "w", "ru", "rv", "rw"))
        _check(lib().pcx_flow_momentum_rhs(self._h, *p, _stream_handle(stream)), "pcx_flow_momentum_rhs")
        return tuple(outs)

    def substep(self, s, Dt, phi, u, v, w, p1, p2, r, h, outs, stream=None, report=True):
        """h = [hphi, hu, hv, hw] (updated in place); outs = [phi, u, v, w, p]."""
        p = self._ptrs((phi, u, v, w, p1, p2), ("phi", "u", "v", "w", "p1", "p2"))
        ph = self._ptrs(h, ("hphi", "hu", "hv", "hw"))
        po = self._ptrs(outs, ("phi_out", "u_out", "v_out", "w_out", "p_out"))
        rep = PcxReport()
        st = lib().pcx_flow_substep(self._h, int(s), float(Dt), *p, float(r), *ph, *po, _stream_handle(stream),
                                    C.byref(rep) if report else None)
        _check(st, "pcx_flow_substep")
        return rep.as_dict() if report else None

    def predict(self, s, Dt, phi, u, v, w, p1, p2, r, h, phi_out, stream=None):
        """pcx_flow_predict: the substep up to the correction.  h = [hphi,
        hu, hv, hw] (updated in place).  Returns (u*, v*, w*, rho, p*, rho0,
        dt), the inputs of the correction."""
        import torch
        outs = [torch.empty(self.shape, dtype=torch.float64, device=phi.device) for _ in range(5)]
        p = self._ptrs((phi, u, v, w, p1, p2), ("phi", "u", "v", "w", "p1", "p2"))
        ph = self._ptrs(h, ("hphi", "hu", "hv", "hw"))
        po = self._ptrs([phi_out] + outs, ("phi_out", "u_star", "v_star", "w_star", "rho", "p_star"))
        rho0, dt = C.c_double(), C.c_double()
        _check(lib().pcx_flow_predict(self._h, int(s), float(Dt), *p, float(r), *ph, *po, C.byref(rho0), C.byref(dt),
                                      _stream_handle(stream)), "pcx_flow_predict")
        return (*outs, rho0.value, dt.value)


class VarCoef:
    """pcx_varcoef: the variable-coefficient projection D((1/rho_f) G p) =
    D u* / dt by preconditioned conjugate gradients, the comparator for the
    splitting.  Fields are torch float64 CUDA tensors of shape (nz, ny, nx)."""

    def __init__(self, grid, autotune=False):
        L = lib()
        self.gs = grid
        self._g = make_grid(grid)
        self._o = make_options("fp64", autotune=autotune)
        h = C.c_void_p()
        _check(L.pcx_varcoef_create(C.byref(self._g), C.byref(self._o), C.byref(h)), "pcx_varcoef_create")
        self._L = L
        self._h = h
        self.shape = (grid.nz, grid.ny, grid.nx)

    def close(self):
        if getattr(self, "_h", None):
            self._L.pcx_varcoef_destroy(self._h)  # the library handle outlives module teardown
            self._h = None

    __del__ = close

    def apply(self, rho, p, out=None, stream=None):
        import torch
        out = out if out is not None else torch.empty(self.shape, dtype=torch.float64, device=p.device)
        _check(lib().pcx_varcoef_apply(self._h, _ptr(rho, self.shape, "rho"), _ptr(p, self.shape, "p"),
                                       _ptr(out, self.shape, "out"), _stream_handle(stream)), "pcx_varcoef_apply")
        return out

    def project(self, dt, rho0, rho, u, v, w, tol=1e-12, maxit=1000, outs=None, stream=None, check=True):
        """Returns (u_out, v_out, w_out, p_out, iterations, relative residual,
        status); raises on an error status other than NOT_CONVERGED unless
        check is False."""
        import torch
        if outs is None:
            outs = [torch.empty(self.shape, dtype=torch.float64, device=u.device) for _ in range(4)]
        ins = [_ptr(t, self.shape, n) for t, n in zip((rho, u, v, w), ("rho", "u", "v", "w"))]
        po = [_ptr(t, self.shape, n) for t, n in zip(outs, ("u_out", "v_out", "w_out", "p_out"))]
        it = C.c_int32()
        rr = C.c_double()
        st = lib().pcx_varcoef_project(self._h, float(dt), float(rho0), *ins, float(tol), int(maxit), *po,
                                       _stream_handle(stream), C.byref(it), C.byref(rr))
        if check and st not in (PCX_OK, PCX_ERR_NOT_CONVERGED):
            _check(st, "pcx_varcoef_project")
        return (*outs, it.value, rr.value, st)
