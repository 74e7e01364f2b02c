"""Python binding of the C ABI in include/mgir.h (ctypes; argument marshalling only).

Every step of the solver runs in the gfx950 kernels of ``libmgir.so``.  torch
provides device memory (the workspace and the caller's vectors) and the
current HIP stream.  There is no CPU fallback: if the library is missing the
import of this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgir.so")

MG_OK, MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_PREC, MG_ERR_WORKSPACE, MG_ERR_HIP, MG_ERR_NOT_CONVERGED, \
    MG_ERR_NONFINITE, MG_ERR_STATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
# Discretisations: finite differences (n = 2^m - 1) or Q1 finite elements
# (n = c 2^k - 1 for odd c as well, the paper's grids).
DISC = {"fd": 0, "q1": 1}


def full_levels(n: int) -> int:
    """Levels of the full hierarchy n, (n-1)/2, ... (down to one point, or to
    the first even size)."""
    m = 1
    while n > 1 and n % 2 == 1:
        n = (n - 1) // 2
        m += 1
    return m
TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
BUF_RHS, BUF_COR, BUF_RES, BUF_SOL = 0, 1, 2, 3
STAGE_SMOOTH_FIRST, STAGE_SWEEP, STAGE_RESTRICT, STAGE_PROLONG_SWEEP, STAGE_COARSE = 0, 1, 2, 3, 4
EXPORTS = ("mg_default_options", "mg_setup", "mg_workspace_size", "mg_bind_workspace", "mg_vcycle", "ir_solve",
           "mg_destroy", "mg_status_string", "mg_last_error", "mg_level_write", "mg_level_read", "mg_stage",
           "mg_levels", "mg_level_n", "mg_profile_step", "mg_set_shape", "mg_get_shape", "mg_bandwidth_probe",
           "mg_setup_batched", "ir_solve_batched", "mg_instances", "mg_setup_multi", "ir_solve_multi",
           "mg_rhs_count", "mg_alpha_shift", "mg_vcycle_noalloc", "mg_get_instance_shape")
SHAPE_STENCIL, SHAPE_RESTRICT, SHAPE_UPDATE, SHAPE_SMOOTH, SHAPE_SWEEP, SHAPE_PROLONG, SHAPE_TAIL, SHAPE_FUSE, \
    SHAPE_FUSE_SR = 0, 1, 2, 3, 4, 5, 6, 7, 8


class MgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double),
                ("residual_scaling", ctypes.c_int), ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("use_initial_guess", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("rescale_half", ctypes.c_int), ("cycles_per_step", ctypes.c_int), ("base_tol", ctypes.c_double),
                ("base_max_iter", ctypes.c_int), ("discretization", ctypes.c_int), ("defer_update", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libmgir.so (built by paper_2007_07539_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_07539_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    H = ctypes.c_void_p
    lib.mg_default_options.argtypes, lib.mg_default_options.restype = [ctypes.POINTER(Options)], None
    lib.mg_setup.argtypes = [ctypes.POINTER(H), i, i, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Options)]
    lib.mg_workspace_size.argtypes = [H, ctypes.POINTER(ctypes.c_size_t)]
    lib.mg_bind_workspace.argtypes = [H, vp, ctypes.c_size_t, vp]
    lib.mg_vcycle.argtypes = [H, vp, vp, vp]
    lib.mg_vcycle_noalloc.argtypes = [H, vp, vp, vp]
    lib.ir_solve.argtypes = [H, vp, vp, ctypes.POINTER(Stats), vp]
    lib.mg_destroy.argtypes = [H]
    lib.mg_status_string.argtypes, lib.mg_status_string.restype = [i], ctypes.c_char_p
    lib.mg_last_error.argtypes, lib.mg_last_error.restype = [], ctypes.c_char_p
    lib.mg_level_write.argtypes = [H, i, i, vp, i, vp]
    lib.mg_level_read.argtypes = [H, i, i, vp, i, vp]
    lib.mg_stage.argtypes = [H, i, i, vp]
    lib.mg_levels.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.mg_level_n.argtypes = [H, i, ctypes.POINTER(ctypes.c_int)]
    lib.mg_profile_step.argtypes = [H, vp, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_char_p),
                                    ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int)]
    lib.mg_set_shape.argtypes = [H, i, i, ctypes.POINTER(ctypes.c_int), i]
    lib.mg_get_shape.argtypes = [H, i, i, ctypes.POINTER(ctypes.c_int), i]
    lib.mg_get_instance_shape.argtypes = [H, i, i, i, ctypes.POINTER(ctypes.c_int), i]
    lib.mg_bandwidth_probe.argtypes = [vp, vp, ctypes.c_size_t, i, i, vp]
    lib.mg_setup_batched.argtypes = [ctypes.POINTER(H), i, i, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Options)]
    lib.ir_solve_batched.argtypes = [H, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(Stats), vp]
    lib.mg_instances.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.mg_setup_multi.argtypes = [ctypes.POINTER(H), i, i, i, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Options)]
    lib.ir_solve_multi.argtypes = [H, vp, vp, ctypes.POINTER(Stats), vp]
    lib.mg_rhs_count.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    lib.mg_alpha_shift.argtypes = [H, i, ctypes.POINTER(ctypes.c_int)]
    for f in EXPORTS:
        if f not in ("mg_default_options", "mg_status_string", "mg_last_error"):
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != MG_OK:
        lib = load()
        msg = lib.mg_last_error().decode(errors="replace")
        raise MgError(status, f"{what}: {lib.mg_status_string(status).decode()}: {msg}")


def default_options() -> Options:
    o = Options()
    load().mg_default_options(ctypes.byref(o))
    return o


def _stream_ptr(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t: torch.Tensor) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveResult:
    status: int
    iterations: int
    rel_residual: float
    seconds: float
    history: list = field(default_factory=list)


class Solver:
    """One grid: ``mg_setup`` + a torch-allocated workspace bound with ``mg_bind_workspace``.

    level_prec: list of 'f64' | 'f32' | 'f16' | 'bf16', finest level first
    (None = all FP64).  Vectors are torch tensors of shape (n,)*dim on the GPU.
    """

    def __init__(self, dim: int, n: int, level_prec=None, *, nu1=2, nu2=2, omega=0.8, residual_scaling=True,
                 max_iter=100, rtol=1e-10, use_initial_guess=False, use_graph=True, autotune=False,
                 rescale_half=False, cycles_per_step=1, nlevels=0, base_tol=1e-4, base_max_iter=0,
                 disc="fd", defer_update=0, device=None, stream=None):
        self.lib = load()
        self.dim, self.n = dim, n
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        o = default_options()
        o.nu1, o.nu2, o.omega = nu1, nu2, omega
        o.residual_scaling, o.max_iter, o.rtol = int(bool(residual_scaling)), max_iter, rtol
        o.use_initial_guess, o.use_graph, o.autotune = int(bool(use_initial_guess)), int(bool(use_graph)), \
            int(bool(autotune))
        o.rescale_half = int(bool(rescale_half))
        o.cycles_per_step = int(cycles_per_step)
        o.base_tol, o.base_max_iter = float(base_tol), int(base_max_iter)
        o.defer_update = int(defer_update)
        if disc not in DISC:
            raise ValueError(f"disc must be one of {sorted(DISC)}, got {disc!r}")
        o.discretization = DISC[disc]
        self.disc = disc
        self.options = o
        self._h = ctypes.c_void_p()
        m = full_levels(n)
        if nlevels:
            m = int(nlevels)
        if level_prec is None:
            level_prec = ["f64"] * m
        self.level_prec = list(level_prec)
        if len(self.level_prec) != m:
            raise ValueError(f"level_prec needs {m} entries (finest first), got {len(self.level_prec)}")
        arr = (ctypes.c_int * m)(*[PREC[p] for p in self.level_prec])
        _check(self.lib.mg_setup(ctypes.byref(self._h), dim, n, int(nlevels), arr, ctypes.byref(o)), "mg_setup")
        nb = ctypes.c_size_t()
        _check(self.lib.mg_workspace_size(self._h, ctypes.byref(nb)), "mg_workspace_size")
        self.workspace_bytes = nb.value
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            _check(self.lib.mg_bind_workspace(self._h, ctypes.c_void_p(base + off), nb.value,
                                              _stream_ptr(stream)), "mg_bind_workspace")
        nl = ctypes.c_int()
        _check(self.lib.mg_levels(self._h, ctypes.byref(nl)), "mg_levels")
        self.nlevels = nl.value

    # -- helpers ---------------------------------------------------------------
    def alpha_shift(self, instance: int = 0) -> int:
        """j of alpha = 2^j ||r||_inf (-1 with residual scaling off)."""
        v = ctypes.c_int()
        _check(self.lib.mg_alpha_shift(self._h, int(instance), ctypes.byref(v)), "mg_alpha_shift")
        return v.value

    def level_n(self, level: int) -> int:
        v = ctypes.c_int()
        _check(self.lib.mg_level_n(self._h, level, ctypes.byref(v)), "mg_level_n")
        return v.value

    def level_shape(self, level: int):
        return (self.level_n(level),) * self.dim

    def close(self):
        if self._h:
            self.lib.mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the three operations of the method ----------------------------------------
    def vcycle(self, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """One V-cycle for A e = b from e = 0; returns c = e / h^2 in level_prec[0]."""
        dt = TORCH_DTYPE[self.level_prec[0]]
        if b.dtype != dt or tuple(b.shape) != (self.n,) * self.dim:
            raise ValueError(f"b must be {dt} of shape {(self.n,) * self.dim}")
        c = torch.empty_like(b) if out is None else out
        _check(self.lib.mg_vcycle(self._h, _dptr(b), _dptr(c), _stream_ptr(stream)), "mg_vcycle")
        return c

    def vcycle_noalloc(self, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The same V-cycle through mg_vcycle_noalloc (the library's own
        device array, no workspace, no allocation inside the call)."""
        dt = TORCH_DTYPE[self.level_prec[0]]
        if b.dtype != dt or tuple(b.shape) != (self.n,) * self.dim:
            raise ValueError(f"b must be {dt} of shape {(self.n,) * self.dim}")
        c = torch.empty_like(b) if out is None else out
        _check(self.lib.mg_vcycle_noalloc(self._h, _dptr(b), _dptr(c), _stream_ptr(stream)), "mg_vcycle_noalloc")
        return c

    def solve(self, b: torch.Tensor, u: torch.Tensor | None = None, stream=None, history_cap: int = 256,
              check: bool = True) -> tuple[torch.Tensor, SolveResult]:
        """Iterative refinement to ||r||_2 <= rtol ||b||_2 (Algorithm 2)."""
        if b.dtype != torch.float64 or tuple(b.shape) != (self.n,) * self.dim:
            raise ValueError(f"b must be float64 of shape {(self.n,) * self.dim}")
        if u is None:
            u = torch.zeros_like(b)
        hist = (ctypes.c_double * history_cap)()
        st = Stats(0, 0.0, 0.0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), history_cap)
        status = self.lib.ir_solve(self._h, _dptr(b), _dptr(u), ctypes.byref(st), _stream_ptr(stream))
        res = SolveResult(status, st.iterations, st.rel_residual, st.seconds,
                          [hist[i] for i in range(min(st.iterations + 1, history_cap))])
        if check and status not in (MG_OK,):
            _check(status, "ir_solve")
        return u, res

    # -- stage-level access ---------------------------------------------------------
    def write(self, level: int, buf: int, src: torch.Tensor, stream=None):
        rev = {v: k for k, v in TORCH_DTYPE.items()}
        _check(self.lib.mg_level_write(self._h, level, buf, _dptr(src), PREC[rev[src.dtype]], _stream_ptr(stream)),
               "mg_level_write")

    def read(self, level: int, buf: int, dtype=torch.float64, stream=None) -> torch.Tensor:
        rev = {v: k for k, v in TORCH_DTYPE.items()}
        out = torch.empty(self.level_shape(level), dtype=dtype, device=self.device)
        _check(self.lib.mg_level_read(self._h, level, buf, _dptr(out), PREC[rev[dtype]], _stream_ptr(stream)),
               "mg_level_read")
        return out

    def stage(self, stage: int, level: int, stream=None):
        _check(self.lib.mg_stage(self._h, stage, level, _stream_ptr(stream)), "mg_stage")

    def set_shape(self, level: int, kind: int, params):
        arr = (ctypes.c_int * len(params))(*params)
        _check(self.lib.mg_set_shape(self._h, level, kind, arr, len(params)), "mg_set_shape")

    def get_shape(self, level: int, kind: int, count: int | None = None):
        """The shape's values (count of them; default: the set a caller passes
        to set_shape, e.g. three for SHAPE_FUSE_SR, four to include lds16, two
        ({ty, zc}) on a Q1 handle)."""
        arr = (ctypes.c_int * 7)()
        _check(self.lib.mg_get_shape(self._h, level, kind, arr, 7), "mg_get_shape")
        if count is None and getattr(self, "disc", "fd") == "q1":
            count = 2
        n = {SHAPE_RESTRICT: 4, SHAPE_TAIL: 1, SHAPE_FUSE: 5, SHAPE_FUSE_SR: 3}.get(kind, 6) if count is None else count
        return list(arr[:n])

    def profile_step(self, stream=None, cap: int = 512):
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        by = (ctypes.c_double * cap)()
        lv = (ctypes.c_int * cap)()
        cnt = ctypes.c_int()
        _check(self.lib.mg_profile_step(self._h, _stream_ptr(stream), cap, ctypes.byref(cnt), names, ms, by, lv),
               "mg_profile_step")
        return [(names[i].decode(), lv[i], ms[i], by[i]) for i in range(min(cnt.value, cap))]


def _bind(lib, h, device, stream):
    nb = ctypes.c_size_t()
    _check(lib.mg_workspace_size(h, ctypes.byref(nb)), "mg_workspace_size")
    with torch.cuda.device(device):
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
        base = ws.data_ptr()
        off = (-base) % 256
        _check(lib.mg_bind_workspace(h, ctypes.c_void_p(base + off), nb.value, _stream_ptr(stream)),
               "mg_bind_workspace")
    return ws, nb.value


class BatchedSolver:
    """Many 3-D grids of different sizes: ``mg_setup_batched`` + ``ir_solve_batched``.

    sizes: list of n_i = 2^m_i - 1.  level_prec: Lmax formats (finest first,
    the last one for every instance's base level), None = all FP64.
    """

    def __init__(self, sizes, level_prec=None, *, nu1=2, nu2=2, omega=0.8, residual_scaling=True, max_iter=100,
                 rtol=1e-10, use_initial_guess=False, use_graph=True, autotune=False, device=None, stream=None):
        self.lib = load()
        self.sizes = [int(n) for n in sizes]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        o = default_options()
        o.nu1, o.nu2, o.omega = nu1, nu2, omega
        o.residual_scaling, o.max_iter, o.rtol = int(bool(residual_scaling)), max_iter, rtol
        o.use_initial_guess, o.use_graph, o.autotune = int(bool(use_initial_guess)), int(bool(use_graph)), \
            int(bool(autotune))
        self.options = o
        lmax = max(int(n + 1).bit_length() - 1 for n in self.sizes)
        if level_prec is None:
            level_prec = ["f64"] * lmax
        self.level_prec = list(level_prec)
        if len(self.level_prec) != lmax:
            raise ValueError(f"level_prec needs {lmax} entries (finest first), got {len(self.level_prec)}")
        self._h = ctypes.c_void_p()
        ns = (ctypes.c_int * len(self.sizes))(*self.sizes)
        arr = (ctypes.c_int * lmax)(*[PREC[p] for p in self.level_prec])
        _check(self.lib.mg_setup_batched(ctypes.byref(self._h), 3, len(self.sizes), ns, arr, ctypes.byref(o)),
               "mg_setup_batched")
        self.workspace, self.workspace_bytes = _bind(self.lib, self._h, self.device, stream)

    def instance_prec(self, i: int):
        """The single-grid level map that instance i follows."""
        m = int(self.sizes[i] + 1).bit_length() - 1
        return self.level_prec[: m - 1] + [self.level_prec[-1]]

    def close(self):
        if self._h:
            self.lib.mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, us=None, stream=None, history_cap: int = 256, check: bool = True):
        """Algorithm 2 for every instance; returns (us, [SolveResult per instance], status)."""
        k = len(self.sizes)
        if len(bs) != k:
            raise ValueError(f"expected {k} right-hand sides")
        for b, n in zip(bs, self.sizes):
            if b.dtype != torch.float64 or tuple(b.shape) != (n, n, n):
                raise ValueError(f"b must be float64 of shape {(n, n, n)}")
        if us is None:
            us = [torch.zeros_like(b) for b in bs]
        bp = (ctypes.c_void_p * k)(*[_dptr(b).value for b in bs])
        up = (ctypes.c_void_p * k)(*[_dptr(u).value for u in us])
        hists = [(ctypes.c_double * history_cap)() for _ in range(k)]
        stats = (Stats * k)()
        for i in range(k):
            stats[i].history = ctypes.cast(hists[i], ctypes.POINTER(ctypes.c_double))
            stats[i].history_cap = history_cap
        status = self.lib.ir_solve_batched(self._h, bp, up, stats, _stream_ptr(stream))
        res = [SolveResult(status, stats[i].iterations, stats[i].rel_residual, stats[i].seconds,
                           [hists[i][j] for j in range(min(stats[i].iterations + 1, history_cap))])
               for i in range(k)]
        if check and status != MG_OK:
            _check(status, "ir_solve_batched")
        return us, res, status

    def profile_step(self, stream=None, cap: int = 1024):
        return Solver.profile_step(self, stream, cap)

    def get_shape(self, inst: int, level: int, kind: int, count: int | None = None):
        """Instance inst's shape of level and kind (see Solver.get_shape)."""
        arr = (ctypes.c_int * 7)()
        _check(self.lib.mg_get_instance_shape(self._h, inst, level, kind, arr, 7), "mg_get_instance_shape")
        n = (4 if kind == SHAPE_RESTRICT else 6) if count is None else count
        return list(arr[:n])


class MultiSolver:
    """Many right-hand sides on one 3-D grid: ``mg_setup_multi`` + ``ir_solve_multi``.

    Vectors are FP64 device tensors of shape (n, n, n, nrhs), index [z, y, x, k]
    (right-hand sides interleaved).
    """

    def __init__(self, n: int, nrhs: int, level_prec=None, *, nu1=2, nu2=2, omega=0.8, residual_scaling=True,
                 max_iter=100, rtol=1e-10, use_initial_guess=False, use_graph=True, autotune=False, device=None,
                 stream=None):
        self.lib = load()
        self.n, self.nrhs = int(n), int(nrhs)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        o = default_options()
        o.nu1, o.nu2, o.omega = nu1, nu2, omega
        o.residual_scaling, o.max_iter, o.rtol = int(bool(residual_scaling)), max_iter, rtol
        o.use_initial_guess, o.use_graph, o.autotune = int(bool(use_initial_guess)), int(bool(use_graph)), \
            int(bool(autotune))
        self.options = o
        m = int(n + 1).bit_length() - 1
        if level_prec is None:
            level_prec = ["f64"] * m
        self.level_prec = list(level_prec)
        if len(self.level_prec) != m:
            raise ValueError(f"level_prec needs {m} entries (finest first), got {len(self.level_prec)}")
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_int * m)(*[PREC[p] for p in self.level_prec])
        _check(self.lib.mg_setup_multi(ctypes.byref(self._h), 3, self.n, self.nrhs, arr, ctypes.byref(o)),
               "mg_setup_multi")
        self.workspace, self.workspace_bytes = _bind(self.lib, self._h, self.device, stream)

    def close(self):
        if self._h:
            self.lib.mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b: torch.Tensor, u: torch.Tensor | None = None, stream=None, history_cap: int = 256,
              check: bool = True):
        """Algorithm 2 per right-hand side; returns (u, [SolveResult per column], status)."""
        shape = (self.n,) * 3 + (self.nrhs,)
        if b.dtype != torch.float64 or tuple(b.shape) != shape:
            raise ValueError(f"b must be float64 of shape {shape}")
        if u is None:
            u = torch.zeros_like(b)
        k = self.nrhs
        hists = [(ctypes.c_double * history_cap)() for _ in range(k)]
        stats = (Stats * k)()
        for i in range(k):
            stats[i].history = ctypes.cast(hists[i], ctypes.POINTER(ctypes.c_double))
            stats[i].history_cap = history_cap
        status = self.lib.ir_solve_multi(self._h, _dptr(b), _dptr(u), stats, _stream_ptr(stream))
        res = [SolveResult(status, stats[i].iterations, stats[i].rel_residual, stats[i].seconds,
                           [hists[i][j] for j in range(min(stats[i].iterations + 1, history_cap))])
               for i in range(k)]
        if check and status != MG_OK:
            _check(status, "ir_solve_multi")
        return u, res, status

    def profile_step(self, stream=None, cap: int = 1024):
        return Solver.profile_step(self, stream, cap)

    def get_shape(self, level: int, kind: int, count: int | None = None):
        """Level's shape (see Solver.get_shape; zc, and zcc of the restriction,
        are the values that shape these kernels)."""
        return Solver.get_shape(self, level, kind, count)


def bandwidth_probe(dst: torch.Tensor, src: torch.Tensor, kind: int, blocks: int = 4096, stream=None):
    """One copy (0) / read (1) / write (2) pass over src.numel() bytes' worth of
    16-byte lanes; kind 3: the update's access mix, dst = two FP64 arrays of N
    elements back to back, src = two FP16 arrays of N elements."""
    nbytes = src.numel() * src.element_size()
    if kind in (3, 6, 7):
        nbytes = dst.numel() * dst.element_size() // 2
    _check(load().mg_bandwidth_probe(_dptr(dst), _dptr(src), nbytes, kind, blocks, _stream_ptr(stream)),
           "mg_bandwidth_probe")
