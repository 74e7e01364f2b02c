"""Range of the FP16 levels under residual scaling (CPU).

With alpha = ||r||_inf the correction equation's right-hand side has max-norm
one (Algorithm 2, Section 4.3).  Its solution in grid-scaled units is bounded
by max(L^-1 1), which grows like K_D (n+1)^2 with K_D the centre value of the
torsion function (-Laplace w = 1, w = 0 on the boundary) of the unit square or
cube.  The library scales by 2^j ||r||_inf on grids where that bound would
bring FP16 values near 65504.  These tests pin K_D by its Fourier series, pin
that the oracle's discrete values stay below it in both discretisations, and
check the exponent the library picks against those facts."""
import ctypes

import numpy as np
import pytest

from paper_2007_07539_amd import mgir
from paper_2007_07539_amd import workloads as W

LIMIT = 2.0**14


def torsion_centre(dim, terms=799):
    """w at the centre from the eigen-expansion: the coefficient of
    prod sin(k_d pi x_d) for odd k is 4^D / (pi^(D+2) prod k_d sum k_d^2),
    and each sine is (-1)^((k-1)/2) at x = 1/2."""
    k = np.arange(1, terms + 1, 2, dtype=np.float64)
    sgn = (-1.0) ** ((k - 1) // 2)
    if dim == 2:
        K1, K2 = np.meshgrid(k, k, indexing="ij")
        S = np.outer(sgn, sgn)
        return float(np.sum(16.0 * S / (np.pi**4 * K1 * K2 * (K1**2 + K2**2))))
    tot = 0.0
    for i, kz in enumerate(k):
        K1, K2 = np.meshgrid(k, k, indexing="ij")
        S = np.outer(sgn, sgn) * sgn[i]
        tot += float(np.sum(64.0 * S / (np.pi**5 * K1 * K2 * kz * (K1**2 + K2**2 + kz**2))))
    return tot


K2 = 0.0736713532
KLIB = {2: 0.074, 3: 0.058}   # the library's bound constants


def test_torsion_constants():
    assert torsion_centre(2) == pytest.approx(K2, abs=2e-9)
    k3 = torsion_centre(3, terms=399)
    assert k3 == pytest.approx(0.05621, abs=5e-5)
    assert K2 < KLIB[2] and k3 < KLIB[3]


@pytest.mark.parametrize("dim,sizes", [(2, (15, 31, 63, 127)), (3, (7, 15, 31))])
def test_discrete_bound_against_torsion_limit(ref, dim, sizes):
    """max(A^-1 1) in physical units, i.e. max(L^-1 1) h^2 in grid-scaled
    units, tends to the torsion-function centre value: from below for the
    finite differences, from above for Q1 with the lumped unit load; on every
    grid both stay under the library's constant."""
    kd = K2 if dim == 2 else torsion_centre(3, terms=399)
    for disc, sign in (("fd", -1), ("q1", 1)):
        gaps = []
        for n in sizes:
            h = 1.0 / (n + 1)
            b = np.ones((n,) * dim) * (h**dim if disc == "q1" else 1.0)
            top = ref.ir_solve(b, rtol=1e-12, disc=disc).u.max()
            assert sign * (top - kd) > 0 and top < KLIB[dim], (disc, n, top)
            gaps.append(abs(top - kd))
        assert all(b < a for a, b in zip(gaps, gaps[1:])), (disc, gaps)
        assert gaps[-1] < 0.02 * kd


def _shift(dim, n, prec, disc=0, scaling=1, rescale=0):
    lib = mgir.load()
    o = mgir.default_options()
    o.residual_scaling, o.discretization, o.rescale_half = scaling, disc, rescale
    m = mgir.full_levels(n)
    arr = (ctypes.c_int * m)(*([mgir.PREC[prec]] * (m - 1) + [0]))
    h = ctypes.c_void_p()
    st = lib.mg_setup(ctypes.byref(h), dim, n, 0, arr, ctypes.byref(o))
    if st != mgir.MG_OK:
        return st, None
    try:
        j = ctypes.c_int()
        assert lib.mg_alpha_shift(h, 0, ctypes.byref(j)) == mgir.MG_OK
        return st, j.value
    finally:
        lib.mg_destroy(h)


@pytest.mark.parametrize("dim,n,disc", [(2, 255, 0), (2, 511, 0), (2, 2047, 0), (2, 4095, 0), (3, 511, 0),
                                        (3, 1023, 0), (2, 6143, 1), (3, 287, 1), (2, 8191, 1)])
def test_alpha_exponent_keeps_fp16_in_range(dim, n, disc):
    """The exponent j keeps K_D (n+1)^2 / 2^j <= 2^14 (a factor four below
    FP16's 65504) and is the least such j up to the rounding of K_D."""
    kd = K2 if dim == 2 else 0.05621
    st, j = _shift(dim, n, "f16", disc)
    assert st == mgir.MG_OK
    bound = kd * (n + 1) ** 2
    assert bound / 2.0**j <= LIMIT
    assert j == 0 or bound / 2.0 ** (j - 1) > 0.95 * LIMIT
    # other formats need no shift; no scaling reports -1
    assert _shift(dim, n, "bf16", disc)[1] == 0 and _shift(dim, n, "f32", disc)[1] == 0
    assert _shift(dim, n, "f16", disc, scaling=0)[1] == -1


def test_headline_grid_needs_no_shift():
    assert _shift(3, 511, "f16")[1] == 0
    assert _shift(3, 255, "f16")[1] == 0


def test_rescaled_fp16_level_beyond_range_is_rejected():
    """With rescale_half an FP16 level gets its own right-hand side of max-norm
    one, so alpha cannot help: a level of 2047^2 points is refused, 127^2 is fine."""
    lib = mgir.load()
    o = mgir.default_options()
    o.rescale_half = 1
    for n, want in ((4095, mgir.MG_ERR_PREC), (255, mgir.MG_OK)):
        m = mgir.full_levels(n)
        arr = (ctypes.c_int * m)(*([0] + [mgir.PREC["f16"]] * (m - 2) + [0]))
        h = ctypes.c_void_p()
        assert lib.mg_setup(ctypes.byref(h), 2, n, 0, arr, ctypes.byref(o)) == want
        if h.value:
            lib.mg_destroy(h)


def test_batched_instances_get_their_own_exponent():
    lib = mgir.load()
    ns = (ctypes.c_int * 3)(1023, 255, 511)
    arr = (ctypes.c_int * 10)(*([mgir.PREC["f16"]] * 9 + [0]))
    h = ctypes.c_void_p()
    assert lib.mg_setup_batched(ctypes.byref(h), 3, 3, ns, arr, None) == mgir.MG_OK
    try:
        got = []
        for i in range(3):
            j = ctypes.c_int()
            assert lib.mg_alpha_shift(h, i, ctypes.byref(j)) == mgir.MG_OK
            got.append(j.value)
        assert got == [2, 0, 0]
        assert lib.mg_alpha_shift(h, 3, ctypes.byref(ctypes.c_int())) == mgir.MG_ERR_ARG
    finally:
        lib.mg_destroy(h)
