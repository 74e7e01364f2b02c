"""C-ABI boundary on the CPU: the library loads, exports every function the
header declares, and its validation paths answer without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2007_07539_amd import mgir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return mgir.load()


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "mgir.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_functions_are_exported(lib):
    names = _declared_functions()
    assert "ir_solve" in names and "mg_vcycle" in names and "mg_setup" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/mgir.h but not exported"
    assert set(mgir.EXPORTS) <= set(names)


def test_default_options(lib):
    o = mgir.default_options()
    assert (o.nu1, o.nu2, o.omega, o.residual_scaling, o.max_iter, o.rtol, o.use_initial_guess) == \
        (2, 2, 0.8, 1, 100, 1e-10, 0)


@pytest.mark.parametrize("dim,n,status", [(3, 0, mgir.MG_ERR_SHAPE), (3, 1, mgir.MG_ERR_SHAPE),
                                          (3, 100, mgir.MG_ERR_SHAPE), (4, 127, mgir.MG_ERR_SHAPE),
                                          (1, 127, mgir.MG_ERR_SHAPE), (3, 8191, mgir.MG_ERR_SHAPE),
                                          (3, 2047, mgir.MG_ERR_SHAPE)])
def test_setup_rejects_bad_shapes(lib, dim, n, status):
    h = ctypes.c_void_p()
    assert lib.mg_setup(ctypes.byref(h), dim, n, 0, None, None) == status
    assert not h.value
    assert lib.mg_last_error()


def test_setup_rejects_bad_options_and_maps(lib):
    h = ctypes.c_void_p()
    o = mgir.default_options()
    o.nu1 = 0
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, None, ctypes.byref(o)) == mgir.MG_ERR_ARG
    o = mgir.default_options()
    o.omega = 2.5
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, None, ctypes.byref(o)) == mgir.MG_ERR_ARG
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 1, None, None) == mgir.MG_ERR_ARG   # no coarse level
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 6, None, None) == mgir.MG_ERR_ARG   # deeper than 31 -> 1
    bad = (ctypes.c_int * 5)(0, 2, 7, 1, 0)
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, bad, None) == mgir.MG_ERR_PREC
    assert lib.mg_setup(None, 3, 31, 0, None, None) == mgir.MG_ERR_ARG


def test_workspace_size_and_unbound_errors(lib):
    h = ctypes.c_void_p()
    prec = (ctypes.c_int * 7)(2, 2, 2, 2, 2, 2, 0)
    assert lib.mg_setup(ctypes.byref(h), 3, 127, 0, prec, None) == mgir.MG_OK
    try:
        nb = ctypes.c_size_t()
        assert lib.mg_workspace_size(h, ctypes.byref(nb)) == mgir.MG_OK
        P = 128
        finest16 = (P + 2) * P * P * 2
        fp64 = (P + 2) * P * P * 8
        assert nb.value >= 3 * finest16 + 2 * fp64
        nl = ctypes.c_int()
        assert lib.mg_levels(h, ctypes.byref(nl)) == 0 and nl.value == 7
        n = ctypes.c_int()
        assert lib.mg_level_n(h, 6, ctypes.byref(n)) == 0 and n.value == 1
        assert lib.mg_level_n(h, 7, ctypes.byref(n)) == mgir.MG_ERR_ARG
        # nothing bound yet: every device operation refuses
        assert lib.ir_solve(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None) == mgir.MG_ERR_WORKSPACE
        assert lib.mg_vcycle(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == mgir.MG_ERR_WORKSPACE
        assert lib.mg_stage(h, 1, 0, None) == mgir.MG_ERR_WORKSPACE
        assert b"workspace" in lib.mg_last_error()
        assert lib.mg_bind_workspace(h, ctypes.c_void_p(256), 16, None) == mgir.MG_ERR_WORKSPACE
        assert lib.mg_bind_workspace(h, ctypes.c_void_p(255), nb.value, None) == mgir.MG_ERR_WORKSPACE
    finally:
        assert lib.mg_destroy(h) == mgir.MG_OK
    assert lib.mg_destroy(None) == mgir.MG_OK


def test_status_strings(lib):
    for s in range(-8, 1):
        assert lib.mg_status_string(s)
    assert lib.mg_status_string(-99) == b"unknown status"


def _setup_batched(lib, sizes, prec=None, opt=None, dim=3):
    h = ctypes.c_void_p()
    ns = (ctypes.c_int * max(1, len(sizes)))(*sizes)
    pa = None if prec is None else (ctypes.c_int * len(prec))(*prec)
    st = lib.mg_setup_batched(ctypes.byref(h), dim, len(sizes), ns, pa, None if opt is None else ctypes.byref(opt))
    return st, h


def test_batched_setup_validation(lib):
    for sizes in ([], [15, 16], [15, 1], [15, 2047]):
        st, h = _setup_batched(lib, sizes)
        assert st in (mgir.MG_ERR_ARG, mgir.MG_ERR_SHAPE) and not h.value
    assert _setup_batched(lib, [15, 7], dim=2)[0] == mgir.MG_ERR_SHAPE
    assert _setup_batched(lib, [15, 7], prec=[0, 2, 9, 0])[0] == mgir.MG_ERR_PREC
    o = mgir.default_options()
    o.nu1 = 1
    assert _setup_batched(lib, [15, 7], opt=o)[0] == mgir.MG_ERR_ARG


def test_batched_workspace_and_refusals(lib):
    sizes = [63, 7, 127, 15]
    st, h = _setup_batched(lib, sizes, prec=[2] * 6 + [0])
    assert st == mgir.MG_OK
    try:
        nb = ctypes.c_size_t()
        assert lib.mg_workspace_size(h, ctypes.byref(nb)) == mgir.MG_OK
        # every instance's finest level: three FP16 arrays plus FP64 u and r
        need = sum((n + 3) * (n + 1) ** 2 * (3 * 2 + 2 * 8) for n in sizes)
        assert nb.value >= need
        k = ctypes.c_int()
        assert lib.mg_instances(h, ctypes.byref(k)) == 0 and k.value == 4
        nl = ctypes.c_int()
        assert lib.mg_levels(h, ctypes.byref(nl)) == 0 and nl.value == 7
        ptrs = (ctypes.c_void_p * 4)(*([16] * 4))
        assert lib.ir_solve_batched(h, ptrs, ptrs, None, None) == mgir.MG_ERR_WORKSPACE
        assert lib.mg_level_n(h, 0, ctypes.byref(k)) == mgir.MG_ERR_STATE
        assert lib.mg_get_shape(h, 0, 0, (ctypes.c_int * 5)(), 5) == mgir.MG_ERR_STATE
        # shapes are read per instance: instance 2 (n = 127) has six levels below its base
        arr = (ctypes.c_int * 7)()
        for kind in (mgir.SHAPE_STENCIL, mgir.SHAPE_SMOOTH, mgir.SHAPE_SWEEP, mgir.SHAPE_PROLONG):
            assert lib.mg_get_instance_shape(h, 2, 5, kind, arr, 7) == mgir.MG_OK
            assert arr[0] in (4, 8) and 1 <= arr[1] <= 127
        assert lib.mg_get_instance_shape(h, 2, 0, mgir.SHAPE_UPDATE, arr, 7) == mgir.MG_OK and arr[0] == 4
        assert lib.mg_get_instance_shape(h, 2, 0, mgir.SHAPE_RESTRICT, arr, 4) == mgir.MG_OK
        assert arr[0] in (4, 8) and arr[1] >= 1 and arr[2] >= 1
        assert lib.mg_get_instance_shape(h, 2, 6, mgir.SHAPE_STENCIL, arr, 7) == mgir.MG_ERR_ARG  # the base
        assert lib.mg_get_instance_shape(h, 1, 2, mgir.SHAPE_STENCIL, arr, 7) == mgir.MG_ERR_ARG  # n = 7: 2 levels
        assert lib.mg_get_instance_shape(h, 4, 0, mgir.SHAPE_STENCIL, arr, 7) == mgir.MG_ERR_ARG
        assert lib.mg_get_instance_shape(h, -1, 0, mgir.SHAPE_STENCIL, arr, 7) == mgir.MG_ERR_ARG
        assert lib.mg_get_instance_shape(h, 2, 1, mgir.SHAPE_UPDATE, arr, 7) == mgir.MG_ERR_ARG
        assert lib.mg_get_instance_shape(h, 2, 0, mgir.SHAPE_TAIL, arr, 7) == mgir.MG_ERR_ARG
    finally:
        assert lib.mg_destroy(h) == mgir.MG_OK
    # a single-grid handle refuses the batched solve
    h = ctypes.c_void_p()
    assert lib.mg_setup(ctypes.byref(h), 3, 15, 0, None, None) == mgir.MG_OK
    try:
        k = ctypes.c_int()
        assert lib.mg_instances(h, ctypes.byref(k)) == 0 and k.value == 1
        ptrs = (ctypes.c_void_p * 1)(16)
        assert lib.ir_solve_batched(h, ptrs, ptrs, None, None) == mgir.MG_ERR_STATE
    finally:
        lib.mg_destroy(h)


def test_multi_setup_validation_and_workspace(lib):
    h = ctypes.c_void_p()
    for n, k in ((15, 3), (15, 12), (15, 128), (16, 8), (1023, 8)):
        st = lib.mg_setup_multi(ctypes.byref(h), 3, n, k, None, None)
        assert st in (mgir.MG_ERR_ARG, mgir.MG_ERR_SHAPE) and not h.value
    assert lib.mg_setup_multi(ctypes.byref(h), 2, 15, 8, None, None) == mgir.MG_ERR_SHAPE
    f16 = (ctypes.c_int * 4)(2, 2, 2, 0)
    # FP16 levels need at least 8 columns (one thread's chunk)
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 15, 4, f16, None) == mgir.MG_ERR_ARG
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 15, 4, None, None) == mgir.MG_OK  # FP64: 4 columns
    lib.mg_destroy(h)
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 127, 32, (ctypes.c_int * 7)(2, 2, 2, 2, 2, 2, 0), None) == 0
    try:
        nb = ctypes.c_size_t()
        assert lib.mg_workspace_size(h, ctypes.byref(nb)) == mgir.MG_OK
        P = 128
        assert nb.value >= (P + 2) * P * P * 32 * (3 * 2 + 2 * 8)
        k = ctypes.c_int()
        assert lib.mg_rhs_count(h, ctypes.byref(k)) == 0 and k.value == 32
        assert lib.mg_level_n(h, 1, ctypes.byref(k)) == 0 and k.value == 63
        assert lib.ir_solve_multi(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None) == mgir.MG_ERR_WORKSPACE
        assert lib.mg_vcycle(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == mgir.MG_ERR_WORKSPACE
        # the stencil and restriction shapes of the levels below the base can be read
        arr = (ctypes.c_int * 7)()
        for lvl in range(6):
            assert lib.mg_get_shape(h, lvl, mgir.SHAPE_SWEEP, arr, 7) == mgir.MG_OK and arr[1] >= 1
            assert lib.mg_get_shape(h, lvl, mgir.SHAPE_RESTRICT, arr, 4) == mgir.MG_OK and arr[2] >= 1
        assert lib.mg_get_shape(h, 6, mgir.SHAPE_SWEEP, arr, 7) == mgir.MG_ERR_ARG
        assert lib.mg_get_shape(h, 0, mgir.SHAPE_TAIL, arr, 1) == mgir.MG_ERR_ARG
        assert lib.mg_get_instance_shape(h, 0, 0, mgir.SHAPE_SWEEP, arr, 7) == mgir.MG_ERR_STATE
    finally:
        lib.mg_destroy(h)
    assert lib.mg_setup(ctypes.byref(h), 3, 15, 0, None, None) == mgir.MG_OK
    try:
        assert lib.ir_solve_multi(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None) == mgir.MG_ERR_STATE
    finally:
        lib.mg_destroy(h)


def test_rescale_half_option(lib):
    """Per-level rescaling: off by default, adds the scaled-residual buffers of
    the half-precision levels to the workspace, single-grid handles only."""
    assert mgir.default_options().rescale_half == 0
    dsh = (ctypes.c_int * 5)(0, 0, 1, 2, 2)  # 31^3: FP64, FP64, FP32, FP16, FP16
    sizes = []
    for flag in (0, 1):
        o = mgir.default_options()
        o.rescale_half = flag
        h = ctypes.c_void_p()
        assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, dsh, ctypes.byref(o)) == mgir.MG_OK
        nb = ctypes.c_size_t()
        assert lib.mg_workspace_size(h, ctypes.byref(nb)) == mgir.MG_OK
        sizes.append(nb.value)
        assert lib.mg_destroy(h) == mgir.MG_OK
    # levels 3^3 and 1 in FP16: their FP32 / FP16 accumulator copies (padded,
    # 256-byte aligned) plus {s, 1/s} per level and the partial maxima
    assert sizes[1] > sizes[0]
    o = mgir.default_options()
    o.rescale_half = 1
    h = ctypes.c_void_p()
    ns = (ctypes.c_int * 2)(15, 31)
    assert lib.mg_setup_batched(ctypes.byref(h), 3, 2, ns, dsh, ctypes.byref(o)) == mgir.MG_ERR_ARG
    assert b"rescale_half" in lib.mg_last_error()
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 31, 8, None, ctypes.byref(o)) == mgir.MG_ERR_ARG


def test_cycles_per_step_option(lib):
    assert mgir.default_options().cycles_per_step == 1
    h = ctypes.c_void_p()
    for bad in (0, 17, -1):
        o = mgir.default_options()
        o.cycles_per_step = bad
        assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, None, ctypes.byref(o)) == mgir.MG_ERR_ARG
        assert b"cycles_per_step" in lib.mg_last_error()
    o = mgir.default_options()
    o.cycles_per_step = 3
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, None, ctypes.byref(o)) == mgir.MG_OK
    assert lib.mg_destroy(h) == mgir.MG_OK
    ns = (ctypes.c_int * 2)(15, 31)
    assert lib.mg_setup_batched(ctypes.byref(h), 3, 2, ns, None, ctypes.byref(o)) == mgir.MG_ERR_ARG
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 31, 8, None, ctypes.byref(o)) == mgir.MG_ERR_ARG


def test_partial_hierarchy_setup(lib):
    """nlevels < m stops at a multi-point base level solved by CG; the level map
    then has nlevels entries and the workspace holds the CG vectors."""
    o = mgir.default_options()
    assert (o.base_tol, o.base_max_iter) == (1e-4, 0)
    h = ctypes.c_void_p()
    prec = (ctypes.c_int * 3)(2, 2, 0)  # 31^3 FP16, 15^3 FP16, 7^3 FP64 base
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 3, prec, None) == mgir.MG_OK
    try:
        nl, nb = ctypes.c_int(), ctypes.c_int()
        assert lib.mg_levels(h, ctypes.byref(nl)) == 0 and nl.value == 3
        assert lib.mg_level_n(h, 2, ctypes.byref(nb)) == 0 and nb.value == 7
        ws = ctypes.c_size_t()
        assert lib.mg_workspace_size(h, ctypes.byref(ws)) == mgir.MG_OK
        assert ws.value >= 4 * 10 * 8 * 8 * 8  # x, r, p, q of the padded 7^3 base in FP64
    finally:
        assert lib.mg_destroy(h) == mgir.MG_OK
    o.base_tol = -1.0
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 3, prec, ctypes.byref(o)) == mgir.MG_ERR_ARG


def test_q1_discretisation_option(lib):
    """Q1 finite elements: any odd n (the paper's c 2^k - 1 grids), hierarchy to
    the first even size, one-workgroup CG base bounded, single-grid only."""
    assert mgir.default_options().discretization == mgir.DISC["fd"]
    h = ctypes.c_void_p()
    o = mgir.default_options()
    o.discretization = 2
    assert lib.mg_setup(ctypes.byref(h), 3, 31, 0, None, ctypes.byref(o)) == mgir.MG_ERR_ARG
    o.discretization = mgir.DISC["q1"]
    for dim, n in [(3, 96), (3, 1), (2, 4096), (3, 1025), (2, 8193)]:
        assert lib.mg_setup(ctypes.byref(h), dim, n, 0, None, ctypes.byref(o)) == mgir.MG_ERR_SHAPE
    # finite differences keep n = 2^m - 1
    assert lib.mg_setup(ctypes.byref(h), 3, 191, 0, None, None) == mgir.MG_ERR_SHAPE
    # 191 -> 95 -> 47 -> 23 -> 11 -> 5 -> 2: seven levels, base of 2^3 points
    assert lib.mg_setup(ctypes.byref(h), 3, 191, 0, None, ctypes.byref(o)) == mgir.MG_OK
    nl, nb = ctypes.c_int(), ctypes.c_int()
    assert lib.mg_levels(h, ctypes.byref(nl)) == mgir.MG_OK and nl.value == 7
    assert lib.mg_level_n(h, 6, ctypes.byref(nb)) == mgir.MG_OK and nb.value == 2
    q1_bytes = ctypes.c_size_t()
    assert lib.mg_workspace_size(h, ctypes.byref(q1_bytes)) == mgir.MG_OK and q1_bytes.value > 0
    one = (ctypes.c_int * 1)(1)
    assert lib.mg_set_shape(h, 0, mgir.SHAPE_TAIL, one, 1) == mgir.MG_ERR_STATE
    assert lib.mg_destroy(h) == mgir.MG_OK
    assert mgir.full_levels(191) == 7 and mgir.full_levels(511) == 9 and mgir.full_levels(6143) == 12
    # 2^m - 1 grids coarsen to one point as with finite differences
    h = ctypes.c_void_p()
    assert lib.mg_setup(ctypes.byref(h), 2, 255, 0, None, ctypes.byref(o)) == mgir.MG_OK
    assert lib.mg_levels(h, ctypes.byref(nl)) == mgir.MG_OK and nl.value == 8
    assert lib.mg_destroy(h) == mgir.MG_OK
    # a base level above 64^3 points is refused (one workgroup runs the CG)
    assert lib.mg_setup(ctypes.byref(h), 3, 1023, 2, None, None) == mgir.MG_ERR_SHAPE
    assert lib.mg_setup(ctypes.byref(h), 3, 287, 2, None, ctypes.byref(o)) == mgir.MG_ERR_SHAPE
    assert lib.mg_setup(ctypes.byref(h), 3, 287, 3, None, ctypes.byref(o)) == mgir.MG_ERR_SHAPE  # 71^3
    assert lib.mg_setup(ctypes.byref(h), 3, 287, 4, None, ctypes.byref(o)) == mgir.MG_OK  # 35^3
    assert lib.mg_destroy(h) == mgir.MG_OK
    # single-grid handles only
    assert _setup_batched(lib, [15, 7], opt=o)[0] == mgir.MG_ERR_ARG
    h = ctypes.c_void_p()
    assert lib.mg_setup_multi(ctypes.byref(h), 3, 15, 4, None, ctypes.byref(o)) == mgir.MG_ERR_ARG


def test_noalloc_vcycle_refusals_without_a_gpu(lib):
    """mg_vcycle_noalloc checks the handle and the scratch size before any
    device work: a 511^3 hierarchy needs more than the library's array."""
    h = ctypes.c_void_p()
    prec = (ctypes.c_int * 9)(*([mgir.PREC["f16"]] * 8 + [mgir.PREC["f64"]]))
    assert lib.mg_setup(ctypes.byref(h), 3, 511, 0, prec, None) == mgir.MG_OK
    dummy = ctypes.c_void_p(256)
    assert lib.mg_vcycle_noalloc(h, dummy, dummy, None) == mgir.MG_ERR_WORKSPACE
    assert b"mg_vcycle_noalloc holds" in lib.mg_last_error()
    lib.mg_destroy(h)
    assert lib.mg_vcycle_noalloc(None, dummy, dummy, None) == mgir.MG_ERR_ARG
