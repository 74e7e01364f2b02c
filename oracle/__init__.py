"""Serial FP64 oracle for the mixed-precision multigrid / iterative-refinement
method of Oo & Vogel (arXiv 2007.07539).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The GPU library never imports or calls it,
and it shares no code with the GPU library.

The arithmetic lives in ``mg_ref.c`` (plain C, double precision, physical
units); this module only marshals numpy arrays through ctypes.  Arrays are
numpy float64 of shape ``(n, n)`` (2-D, index ``[y, x]``) or ``(n, n, n)``
(3-D, index ``[z, y, x]``), x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_ref.c")
_LIB = os.path.join(_HERE, "libmgref.so")
# the same source built for speed on the host that runs it (timing only)
_LIB_NATIVE = os.path.join(_HERE, "libmgref_native.so")

OK, ERR_ARG, ERR_SHAPE, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_NOMEM = 0, -1, -2, -6, -7, -9

# Discretisations of Section 5: the finite-difference stencil, and the
# bilinear / trilinear Q1 finite elements the paper's measurements use.
DISCS = {"fd": 0, "q1": 1}


def _disc(d) -> int:
    if d not in DISCS:
        raise ValueError(f"unknown discretisation {d!r}")
    return DISCS[d]


def build(force: bool = False, native: bool = False) -> str:
    """Compile the oracle with gcc (serial, no fast-math): -O2 for the tests,
    or with native=True -O3 -march=native into a second library, the copy the
    CPU baseline times (same source, same arithmetic: no contraction of
    products and sums into fused multiply-adds)."""
    lib = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp"
        flags = ["-O3", "-march=native", "-ffp-contract=off"] if native else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _IrOpts(ctypes.Structure):
    _fields_ = [
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double),
        ("residual_scaling", ctypes.c_int), ("recursive_residual", ctypes.c_int),
        ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double), ("use_initial_guess", ctypes.c_int),
        ("cycles", ctypes.c_int), ("base_n", ctypes.c_int), ("base_tol", ctypes.c_double),
        ("base_max_iter", ctypes.c_int), ("disc", ctypes.c_int),
    ]


class _IrResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double)]


_libs = {}


def _load(native: bool = False):
    if native not in _libs:
        lib = ctypes.CDLL(build(native=native))
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.ref_points.argtypes, lib.ref_points.restype = [i, i], ctypes.c_long
        lib.ref_levels.argtypes, lib.ref_levels.restype = [i], i
        lib.ref_apply_A_disc.argtypes = [i, i, i, dp, dp]
        lib.ref_residual_disc.argtypes = [i, i, i, dp, dp, dp]
        lib.ref_jacobi_disc.argtypes = [i, i, i, ctypes.c_double, dp, dp, dp]
        lib.ref_restrict_disc.argtypes = [i, i, i, dp, dp]
        lib.ref_prolong.argtypes = [i, i, dp, dp]
        lib.ref_vcycle.argtypes, lib.ref_vcycle.restype = [i, i, i, i, ctypes.c_double, dp, dp], i
        lib.ref_vcycle_base.argtypes = [i, i, i, i, i, ctypes.c_double, ctypes.c_double, i, dp, dp]
        lib.ref_vcycle_base.restype = i
        lib.ref_vcycle_disc.argtypes = [i, i, i, i, i, i, ctypes.c_double, ctypes.c_double, i, dp, dp]
        lib.ref_vcycle_disc.restype = i
        lib.ref_cg_disc.argtypes, lib.ref_cg_disc.restype = [i, i, i, dp, dp, ctypes.c_double, i], i
        lib.ref_norm2.argtypes, lib.ref_norm2.restype = [dp, ctypes.c_long], ctypes.c_double
        lib.ref_norminf.argtypes, lib.ref_norminf.restype = [dp, ctypes.c_long], ctypes.c_double
        lib.ref_ir_solve.argtypes = [i, i, dp, dp, ctypes.POINTER(_IrOpts), ctypes.POINTER(_IrResult), dp, i]
        lib.ref_ir_solve.restype = i
        for f in ("ref_apply_A_disc", "ref_residual_disc", "ref_jacobi_disc", "ref_restrict_disc", "ref_prolong"):
            getattr(lib, f).restype = None
        _libs[native] = lib
    return _libs[native]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(a: np.ndarray):
    if a.ndim not in (2, 3) or any(s != a.shape[0] for s in a.shape):
        raise ValueError(f"expected an (n,n) or (n,n,n) array, got {a.shape}")
    return a.ndim, a.shape[0]


def apply_A(v, disc="fd"):
    """A v with zero Dirichlet boundary (Section 5): the finite-difference
    Laplacian (disc "fd") or the Q1 finite-element stiffness matrix ("q1")."""
    v = _f64(v)
    dim, n = _shape(v)
    out = np.empty_like(v)
    _load().ref_apply_A_disc(dim, n, _disc(disc), _ptr(v), _ptr(out))
    return out


def residual(b, c, disc="fd"):
    """b - A c."""
    b, c = _f64(b), _f64(c)
    dim, n = _shape(b)
    out = np.empty_like(b)
    _load().ref_residual_disc(dim, n, _disc(disc), _ptr(b), _ptr(c), _ptr(out))
    return out


def jacobi(b, c, omega=0.8, disc="fd"):
    """One damped-Jacobi sweep c + omega (b - A c) / diag(A) (Section 4.2)."""
    b, c = _f64(b), _f64(c)
    dim, n = _shape(b)
    out = np.empty_like(b)
    _load().ref_jacobi_disc(dim, n, _disc(disc), float(omega), _ptr(b), _ptr(c), _ptr(out))
    return out


def restrict(r, disc="fd"):
    """Restriction to the next coarser grid: full weighting (fd), or the
    transpose of linear interpolation (q1)."""
    r = _f64(r)
    dim, n = _shape(r)
    nc = (n - 1) // 2
    out = np.empty((nc,) * dim)
    _load().ref_restrict_disc(dim, n, _disc(disc), _ptr(r), _ptr(out))
    return out


def prolong(e):
    """Linear interpolation to the next finer grid."""
    e = _f64(e)
    dim, nc = _shape(e)
    out = np.empty((2 * nc + 1,) * dim)
    _load().ref_prolong(dim, nc, _ptr(e), _ptr(out))
    return out


def base_max_iter_default(dim: int, n_base: int) -> int:
    """CG steps allowed on the base level when none are given: its unknowns
    (where exact-arithmetic CG terminates), at most 10000."""
    return min(10000, n_base**dim)


def cg(b, tol, max_iter=None, disc="fd"):
    """Conjugate gradients for A x = b from x = 0 (the base solver of Section
    4.2), until ||r||_2 <= tol ||b||_2; returns (x, steps)."""
    b = _f64(b)
    dim, n = _shape(b)
    x = np.empty_like(b)
    k = _load().ref_cg_disc(dim, n, _disc(disc), _ptr(b), _ptr(x), float(tol),
                            int(base_max_iter_default(dim, n) if max_iter is None else max_iter))
    if k < 0:
        raise ValueError(f"ref_cg failed with status {k}")
    return x, k


def hierarchy(n: int, nlevels: int = 0) -> list:
    """Level sizes n, (n-1)/2, ...: down to one point for n = 2^m - 1, else to
    the first even size (the paper's grids c 2^k - 1 end on c - 1); nlevels > 0
    keeps the finest nlevels of them."""
    out = [n]
    while out[-1] > 1 and out[-1] % 2 == 1:
        out.append((out[-1] - 1) // 2)
    return out[:nlevels] if nlevels else out


def vcycle(b, nu1=2, nu2=2, omega=0.8, base_n=1, base_tol=1e-4, base_max_iter=None, disc="fd"):
    """One V-cycle from a zero initial guess (Algorithm 1, recursive), physical
    units, down to the base level of base_n points per dimension (one point:
    exact; more: CG to base_tol)."""
    b = _f64(b)
    dim, n = _shape(b)
    c = np.empty_like(b)
    mi = base_max_iter_default(dim, base_n) if base_max_iter is None else base_max_iter
    st = _load().ref_vcycle_disc(dim, n, _disc(disc), int(base_n), int(nu1), int(nu2), float(omega),
                                 float(base_tol), int(mi), _ptr(b), _ptr(c))
    if st != OK:
        raise ValueError(f"ref_vcycle failed with status {st}")
    return c


def norm2(v) -> float:
    v = _f64(v).ravel()
    return _load().ref_norm2(_ptr(v), v.size)


def norminf(v) -> float:
    v = _f64(v).ravel()
    return _load().ref_norminf(_ptr(v), v.size)


def levels(n: int) -> int:
    return _load().ref_levels(int(n))


@dataclass
class IrResult:
    status: int
    u: np.ndarray
    iterations: int
    rel_residual: float
    true_rel_residual: float
    history: np.ndarray


def ir_solve(b, u0=None, *, nu1=2, nu2=2, omega=0.8, residual_scaling=True,
             recursive_residual=False, max_iter=100, rtol=1e-10, cycles=1, base_n=1, base_tol=1e-4,
             base_max_iter=None, disc="fd", native=False) -> IrResult:
    """Iterative refinement with residuum scaling and one V-cycle per step
    (Algorithm 2), all in FP64.  Stops when ||r||_2 <= rtol ||b||_2.  With
    cycles > 1 each step applies that many V-cycles to the scaled residual
    equation, each continuing from the correction so far.  native=True runs
    the -O3 -march=native build of the same source (for timing)."""
    b = _f64(b)
    dim, n = _shape(b)
    u = np.zeros_like(b) if u0 is None else _f64(u0).copy()
    opts = _IrOpts(int(nu1), int(nu2), float(omega), int(bool(residual_scaling)),
                   int(bool(recursive_residual)), int(max_iter), float(rtol), int(u0 is not None), int(cycles),
                   int(base_n), float(base_tol),
                   int(base_max_iter_default(dim, base_n) if base_max_iter is None else base_max_iter),
                   _disc(disc))
    res = _IrResult()
    hist = np.zeros(max_iter + 2)
    st = _load(native).ref_ir_solve(dim, n, _ptr(b), _ptr(u), ctypes.byref(opts), ctypes.byref(res),
                                    _ptr(hist), hist.size)
    k = res.iterations
    return IrResult(st, u, k, res.rel_residual, res.true_rel_residual, hist[: k + 1].copy())
