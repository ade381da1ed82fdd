"""Plain FP64 CPU oracle for the pressure-correction step (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product package
``paper_2502_04189_amd`` never imports it, and the two share no code.

The numerical work is in ``oracle.c`` (single-threaded C, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Each function states the passage of the CaNS-Fizzy paper it follows
("Methods and Implementation strategy": staggered second-order finite
differences, pressure-correction projection, constant-coefficient splitting,
FFT-based direct Poisson solver).  Arrays are C-contiguous ``[k][j][i]`` FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_DP = C.POINTER(C.c_double)


class OrGrid(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double),
        ("zf", _DP),
        ("bcx", C.c_int), ("bcy", C.c_int), ("bcz", C.c_int),
    ]


class OrDiag(C.Structure):
    _fields_ = [
        ("f_inf", C.c_double), ("rel_residual", C.c_double),
        ("max_div_abs", C.c_double), ("max_div_rel", C.c_double),
        ("mean_p", C.c_double),
    ]


SOURCES = ("oracle.c", "flow.c", "dirichlet.c", "varcoef.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    stale = not os.path.exists(_LIB_PATH) or any(os.path.getmtime(_LIB_PATH) < os.path.getmtime(s) for s in srcs)
    if force or stale:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    """The compiled oracle; PCX_ORACLE_LIB names another build of the same
    source (the mutation tests load deliberately broken copies that way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PCX_ORACLE_LIB") or _LIB_PATH
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(path)
        G = C.POINTER(OrGrid)
        L.oracle_check_grid.argtypes = [G]
        L.oracle_step.argtypes = [G, C.c_double, C.c_double] + [_DP] * 9 + [C.POINTER(OrDiag)]
        L.oracle_rhs.argtypes = [G, C.c_double, C.c_double] + [_DP] * 6
        L.oracle_poisson.argtypes = [G, _DP, _DP]
        L.oracle_rhs_at.argtypes = [G, C.c_double, C.c_double] + [_DP] * 5 + [C.c_int64, C.c_void_p, _DP]
        L.oracle_correct_at.argtypes = ([G, C.c_double, C.c_double] + [_DP] * 6 +
                                        [C.c_int64, C.c_void_p, C.c_void_p, _DP])
        L.oracle_correct.argtypes = [G, C.c_double, C.c_double] + [_DP] * 9
        L.oracle_grad.argtypes = [G, _DP, _DP, _DP, _DP]
        L.oracle_div.argtypes = [G, _DP, _DP, _DP, _DP]
        L.oracle_apply_L.argtypes = [G, _DP, _DP]
        L.oracle_volume_mean.argtypes = [G, _DP]
        L.oracle_volume_mean.restype = C.c_double
        L.oracle_dense_poisson.argtypes = [G, _DP, _DP]
        L.oracle_fft.argtypes = [C.c_int, _DP, _DP, C.c_int]
        L.oracle_dct2.argtypes = [C.c_int, _DP, _DP]
        L.oracle_dct3.argtypes = [C.c_int, _DP, _DP]
        L.oracle_thomas.argtypes = [C.c_int, _DP, _DP, _DP, _DP]
        L.oracle_cyclic.argtypes = [C.c_int, _DP, _DP, _DP, _DP]
        L.oracle_eig.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int]
        L.oracle_eig.restype = C.c_double
        if hasattr(L, "oracle_varcoef_solve"):  # varcoef.c
            I = C.POINTER(C.c_int)
            L.oracle_varcoef_apply.argtypes = [G, _DP, _DP, _DP]
            L.oracle_varcoef_solve.argtypes = [G, _DP, C.c_double, _DP, _DP, C.c_double, C.c_int, I, _DP]
            L.oracle_varcoef_project.argtypes = ([G, C.c_double, _DP, C.c_double] + [_DP] * 7 +
                                                 [C.c_double, C.c_int, I, _DP])
        if hasattr(L, "oracle_poisson_bc"):  # dirichlet.c
            L.oracle_poisson_bc.argtypes = [G, _DP, _DP]
            L.oracle_apply_L_bc.argtypes = [G, _DP, _DP]
            L.oracle_eig_bc.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int]
            L.oracle_eig_bc.restype = C.c_double
            L.oracle_has_dirichlet.argtypes = [G]
        if hasattr(L, "oracle_acdi_rhs"):  # flow.c (a mutant build of oracle.c alone lacks it)
            A, F = C.POINTER(OrAcdi), C.POINTER(OrFlow)
            L.oracle_acdi_normals.argtypes = [G, A] + [_DP] * 5
            L.oracle_acdi_flux.argtypes = [G, A] + [_DP] * 4
            L.oracle_acdi_rhs.argtypes = [G, A] + [_DP] * 5
            L.oracle_curvature.argtypes = [G, A, _DP, _DP]
            L.oracle_momentum_rhs.argtypes = [G, F] + [_DP] * 7
            L.oracle_rk3_coeffs.argtypes = [C.c_int, _DP, _DP, _DP]
            L.oracle_flow_substep.argtypes = ([G, F, C.c_int, C.c_double] + [_DP] * 6 + [C.c_double] +
                                              [_DP] * 9 + [C.POINTER(OrDiag)])
        _lib = L
    return _lib


class OrAcdi(C.Structure):
    _fields_ = [("gamma", C.c_double), ("eps", C.c_double), ("eps_s", C.c_double)]


class OrFlow(C.Structure):
    _fields_ = [("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double),
                ("sigma", C.c_double), ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
                ("acdi", OrAcdi)]


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


class Grid:
    """Grid/BC descriptor (bc: 0 periodic, 1 wall, 2 Dirichlet -- the last
    only for the *_bc Poisson functions); zf holds nz+1 z faces."""

    def __init__(self, nx, ny, nz, lx, ly, zf, bcx=0, bcy=0, bcz=1):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly = float(lx), float(ly)
        self.zf = np.ascontiguousarray(zf, dtype=np.float64)
        self.bcx, self.bcy, self.bcz = int(bcx), int(bcy), int(bcz)
        self._c = OrGrid(self.nx, self.ny, self.nz, self.lx, self.ly, _p(self.zf),
                         self.bcx, self.bcy, self.bcz)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def cref(self):
        return C.byref(self._c)

    @classmethod
    def from_workload(cls, g):
        return cls(g.nx, g.ny, g.nz, g.lx, g.ly, g.zf, g.bcx, g.bcy, g.bcz)


def _chk(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed (rc={rc})")


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def step(g: Grid, dt, rho0, rho, pstar, u, v, w):
    """Whole pressure-correction step (projection with the constant-coefficient
    splitting).  Returns (u_out, v_out, w_out, p, diag dict)."""
    ins = [_arr(a) for a in (rho, pstar, u, v, w)]
    outs = [np.empty(g.shape) for _ in range(4)]
    d = OrDiag()
    rc = lib().oracle_step(g.cref, float(dt), float(rho0), *[_p(a) for a in ins],
                           *[_p(a) for a in outs], C.byref(d))
    _chk(rc, "step")
    diag = {k: getattr(d, k) for k, _ in OrDiag._fields_}
    return outs[0], outs[1], outs[2], outs[3], diag


def rhs(g, dt, rho0, rho, pstar, u, v, w):
    ins = [_arr(a) for a in (rho, pstar, u, v, w)]
    f = np.empty(g.shape)
    _chk(lib().oracle_rhs(g.cref, float(dt), float(rho0), *[_p(a) for a in ins], _p(f)), "rhs")
    return f


def rhs_at(g, dt, rho0, rho, pstar, u, v, w, cells):
    """f at the given flat cell indices (k ny + j) nx + i."""
    ins = [_arr(a) for a in (rho, pstar, u, v, w)]
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty(len(cells))
    _chk(lib().oracle_rhs_at(g.cref, float(dt), float(rho0), *[_p(a) for a in ins], len(cells), cells.ctypes.data,
                             _p(out)), "rhs_at")
    return out


def correct_at(g, dt, rho0, rho, pstar, u, v, w, p, dirs, cells):
    """Corrected velocity on the +dir face (0 u, 1 v, 2 w) of the given flat
    cell indices, from the pressure p."""
    ins = [_arr(a) for a in (rho, pstar, u, v, w, p)]
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    dirs = np.ascontiguousarray(dirs, dtype=np.int32)
    out = np.empty(len(cells))
    _chk(lib().oracle_correct_at(g.cref, float(dt), float(rho0), *[_p(a) for a in ins], len(cells),
                                 dirs.ctypes.data, cells.ctypes.data, _p(out)), "correct_at")
    return out


def poisson(g, f):
    f = _arr(f)
    p = np.empty(g.shape)
    _chk(lib().oracle_poisson(g.cref, _p(f), _p(p)), "poisson")
    return p


def correct(g, dt, rho0, rho, pstar, u, v, w, p):
    ins = [_arr(a) for a in (rho, pstar, u, v, w, p)]
    outs = [np.empty(g.shape) for _ in range(3)]
    _chk(lib().oracle_correct(g.cref, float(dt), float(rho0), *[_p(a) for a in ins],
                              *[_p(a) for a in outs]), "correct")
    return tuple(outs)


def grad(g, q):
    q = _arr(q)
    outs = [np.empty(g.shape) for _ in range(3)]
    _chk(lib().oracle_grad(g.cref, _p(q), *[_p(a) for a in outs]), "grad")
    return tuple(outs)


def div(g, u, v, w):
    ins = [_arr(a) for a in (u, v, w)]
    out = np.empty(g.shape)
    _chk(lib().oracle_div(g.cref, *[_p(a) for a in ins], _p(out)), "div")
    return out


def apply_L(g, p):
    p = _arr(p)
    out = np.empty(g.shape)
    _chk(lib().oracle_apply_L(g.cref, _p(p), _p(out)), "apply_L")
    return out


def volume_mean(g, q):
    q = _arr(q)
    return lib().oracle_volume_mean(g.cref, _p(q))


def dense_poisson(g, f):
    f = _arr(f)
    p = np.empty(g.shape)
    _chk(lib().oracle_dense_poisson(g.cref, _p(f), _p(p)), "dense_poisson")
    return p


def fft(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    _chk(lib().oracle_fft(len(re), _p(re), _p(im), int(sign)), "fft")
    return re + 1j * im


def dct2(x):
    x = _arr(x)
    X = np.empty_like(x)
    _chk(lib().oracle_dct2(len(x), _p(x), _p(X)), "dct2")
    return X


def dct3(X):
    X = _arr(X)
    x = np.empty_like(X)
    _chk(lib().oracle_dct3(len(X), _p(X), _p(x)), "dct3")
    return x


def thomas(a, b, c, d):
    a, b, c = _arr(a), _arr(b), _arr(c)
    x = _arr(d).copy()
    _chk(lib().oracle_thomas(len(x), _p(a), _p(b), _p(c), _p(x)), "thomas")
    return x


def cyclic(a, b, c, d):
    a, b, c = _arr(a), _arr(b), _arr(c)
    x = _arr(d).copy()
    _chk(lib().oracle_cyclic(len(x), _p(a), _p(b), _p(c), _p(x)), "cyclic")
    return x


def eig(n, h, bc, l):
    return lib().oracle_eig(int(n), float(h), int(bc), int(l))


# ----------------------------------------------------------------- flow.c
# Phase-field transport (ACDI), momentum predictor and the Runge-Kutta
# substep around the pressure-correction step ("Mathematical model",
# "Methods and Implementation strategy"); readings in flow.c's header.

def flow_params(rho1=1000.0, rho2=1.0, mu1=1e-2, mu2=1e-4, sigma=0.0, g=(0.0, 0.0, 0.0), gamma=1.0, eps=None,
                eps_s=1e-100, dx=None):
    """OrFlow with the ACDI thickness eps (default: 0.51 dx, dx required then)."""
    if eps is None:
        eps = 0.51 * dx
    return OrFlow(rho1, rho2, mu1, mu2, sigma, g[0], g[1], g[2], OrAcdi(gamma, eps, eps_s))


def acdi_normals(g, fl, phi):
    """(psi, nx, ny, nz) at cell centres."""
    outs = [np.empty(g.shape) for _ in range(4)]
    _chk(lib().oracle_acdi_normals(g.cref, C.byref(fl.acdi), _p(_arr(phi)), *[_p(o) for o in outs]), "acdi_normals")
    return tuple(outs)


def acdi_flux(g, fl, phi):
    """Regularization flux (ax, ay, az) on the +x/+y/+z faces."""
    outs = [np.empty(g.shape) for _ in range(3)]
    _chk(lib().oracle_acdi_flux(g.cref, C.byref(fl.acdi), _p(_arr(phi)), *[_p(o) for o in outs]), "acdi_flux")
    return tuple(outs)


def acdi_rhs(g, fl, phi, u, v, w):
    """Right-hand side of the phase-field transport at cell centres."""
    out = np.empty(g.shape)
    ins = [_arr(a) for a in (phi, u, v, w)]
    _chk(lib().oracle_acdi_rhs(g.cref, C.byref(fl.acdi), *[_p(a) for a in ins], _p(out)), "acdi_rhs")
    return out


def curvature(g, fl, phi):
    out = np.empty(g.shape)
    _chk(lib().oracle_curvature(g.cref, C.byref(fl.acdi), _p(_arr(phi)), _p(out)), "curvature")
    return out


def momentum_rhs(g, fl, phi, u, v, w):
    """Momentum predictor right-hand side per unit mass (ru, rv, rw) on the faces."""
    outs = [np.empty(g.shape) for _ in range(3)]
    ins = [_arr(a) for a in (phi, u, v, w)]
    _chk(lib().oracle_momentum_rhs(g.cref, C.byref(fl), *[_p(a) for a in ins], *[_p(o) for o in outs]),
         "momentum_rhs")
    return tuple(outs)


def rk3_coeffs(s):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _chk(lib().oracle_rk3_coeffs(int(s), C.byref(a), C.byref(b), C.byref(c)), "rk3_coeffs")
    return a.value, b.value, c.value


def flow_substep(g, fl, s, Dt, phi, u, v, w, p1, p2, r, h):
    """One Runge-Kutta substep.  h = [hphi, hu, hv, hw] (previous substep's
    right-hand sides, updated in place).  Returns (phi, u, v, w, p, diag)."""
    ins = [_arr(a) for a in (phi, u, v, w, p1, p2)]
    for a in h:
        assert a.dtype == np.float64 and a.flags.c_contiguous
    outs = [np.empty(g.shape) for _ in range(5)]
    d = OrDiag()
    rc = lib().oracle_flow_substep(g.cref, C.byref(fl), int(s), float(Dt), *[_p(a) for a in ins], float(r),
                                   *[_p(a) for a in h], *[_p(o) for o in outs], C.byref(d))
    _chk(rc, "flow_substep")
    return (*outs, {k: getattr(d, k) for k, _ in OrDiag._fields_})


# ------------------------------------------------------------ dirichlet.c
# Constant-coefficient Poisson solve with periodic, Neumann or homogeneous
# Dirichlet directions (the direct solver of "Methods and Implementation
# strategy" in its sine-transform variants); explicit eigenvector sums.

def apply_L_bc(g, p):
    out = np.empty(g.shape)
    _chk(lib().oracle_apply_L_bc(g.cref, _p(_arr(p)), _p(out)), "apply_L_bc")
    return out


def poisson_bc(g, f):
    """L p = f for a grid with a Dirichlet direction (non-singular)."""
    out = np.empty(g.shape)
    _chk(lib().oracle_poisson_bc(g.cref, _p(_arr(f)), _p(out)), "poisson_bc")
    return out


def eig_bc(n, h, bc, l):
    return lib().oracle_eig_bc(int(n), float(h), int(bc), int(l))


# -------------------------------------------------------------- varcoef.c
# The variable-coefficient projection the splitting replaces ("Methods and
# Implementation strategy"), for the splitting-error comparator.

def varcoef_apply(g, rho, p):
    out = np.empty(g.shape)
    _chk(lib().oracle_varcoef_apply(g.cref, _p(_arr(rho)), _p(_arr(p)), _p(out)), "varcoef_apply")
    return out


def varcoef_project(g, dt, rho, rho0, u, v, w, tol=1e-12, maxit=2000):
    """(u_out, v_out, w_out, p, iterations, relative residual)."""
    ins = [_arr(a) for a in (rho, u, v, w)]
    outs = [np.empty(g.shape) for _ in range(4)]
    it, rr = C.c_int(), C.c_double()
    rc = lib().oracle_varcoef_project(g.cref, float(dt), _p(ins[0]), float(rho0), *[_p(a) for a in ins[1:]],
                                      *[_p(o) for o in outs], float(tol), int(maxit), C.byref(it), C.byref(rr))
    _chk(rc, "varcoef_project")
    return (*outs, it.value, rr.value)
