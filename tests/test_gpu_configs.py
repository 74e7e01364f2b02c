"""The benchmark configurations at their stated sizes (GPU), each solve's
final iterate re-evaluated by the oracle's FP64 residual, plus the 511^3
launch shapes of the fused finest-level kernels compared bitwise with the
unfused kernels, the residuum scaling's reason to exist (Section 4.3), and
FP16 levels on 2-D grids large enough to need the range-safe scale.

Host memory: a few FP64 arrays of 511^3 (1.07 GB each) at a time."""
import gc

import numpy as np
import pytest
import torch

from paper_2007_07539_amd import mgir
from paper_2007_07539_amd import workloads as W
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _oracle_rel(ref, b, u, disc="fd"):
    return ref.norm2(ref.residual(b, u, disc)) / ref.norm2(b)


def test_poisson3d_255_uniform_fp16_vs_fp64(dev, ref):
    """255^3, f uniform[-1, 1] (seed 2), 8 levels: FP16 levels with an FP64
    base and residual scaling against the FP64 map without scaling.  Both reach
    1e-10 by the oracle's residual; the FP64 count equals the oracle's +-1 and
    the FP16 count is within two of it."""
    n = 255
    print("255^3 uniform RHS, f16 vs f64", flush=True)
    b = W.uniform_rhs(3, n, seed=2)
    bt = torch.from_numpy(b).to(dev)
    L = W.levels_for(n)
    u16, r16 = mgir.Solver(3, n, W.precision_map("f16", L), autotune=True).solve(bt)
    u64, r64 = mgir.Solver(3, n, W.precision_map("f64", L), residual_scaling=False, autotune=True).solve(bt)
    u16, u64 = u16.cpu().numpy(), u64.cpu().numpy()
    rel16, rel64 = _oracle_rel(ref, b, u16), _oracle_rel(ref, b, u64)
    print(f"  f16 {r16.iterations} it rel {rel16:.3e}; f64 {r64.iterations} it rel {rel64:.3e}", flush=True)
    assert rel16 <= 1e-10 and rel64 <= 1e-10
    assert r16.iterations <= r64.iterations + 2
    o = ref.ir_solve(b, residual_scaling=False, recursive_residual=True)
    assert o.status == 0 and abs(o.iterations - r64.iterations) <= 1
    assert rel_err(u64, o.u) <= 1e-8 and rel_err(u16, o.u) <= 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("name", ["f32", "bf16", "hsd"])
def test_poisson3d_511_maps(dev, ref, name):
    """511^3, the manufactured sine plus noise (seed 3), 9 levels: the FP32,
    BF16 and FP16/FP32/FP64 maps reach 1e-10 by the oracle's residual within
    two iterations of the FP64 map, and agree with its solution."""
    n = 511
    print(f"511^3 sine + noise, map {name}", flush=True)
    b = W.poisson3d_sine_noise_rhs(n, seed=3)
    bt = torch.from_numpy(b).to(dev)
    L = W.levels_for(n)
    u64, r64 = mgir.Solver(3, n, W.precision_map("f64", L), residual_scaling=False, autotune=True).solve(bt)
    s = mgir.Solver(3, n, W.precision_map(name, L), autotune=True)
    u, r = s.solve(bt)
    del s
    u = u.cpu().numpy()
    rel = _oracle_rel(ref, b, u)
    print(f"  {name}: {r.iterations} it (f64 {r64.iterations}), oracle rel {rel:.3e}", flush=True)
    assert r.status == 0 and rel <= 1e-10
    assert r.iterations <= r64.iterations + 2
    assert rel_err(u, u64.cpu().numpy()) <= 1e-8
    del u, u64, bt
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_fused_kernels_in_their_511_shapes_bitwise(dev):
    """At 511^3 the fused first smoothing + restriction runs with 3 coarse rows
    per tile (102 KB of LDS) and the fused last sweep + update with 1024-thread
    blocks: shapes no smaller grid reaches.  One refinement step and a whole
    solve with these shapes equal the unfused kernels' bit for bit."""
    n = 511
    print("511^3 fused shapes vs unfused", flush=True)
    prec = W.precision_map("f16", W.levels_for(n))
    bt = torch.from_numpy(W.poisson3d_sine_noise_rhs(n, seed=3)).to(dev)

    def run(fused, max_iter):
        s = mgir.Solver(3, n, prec, max_iter=max_iter)
        if fused:
            s.set_shape(0, mgir.SHAPE_FUSE_SR, [1, 3, 85])
            s.set_shape(0, mgir.SHAPE_FUSE, [1, 4, 64, 1, 4])
            assert s.get_shape(0, mgir.SHAPE_FUSE_SR) == [1, 3, 85]
            assert s.get_shape(0, mgir.SHAPE_FUSE) == [1, 4, 64, 1, 4]
        else:
            s.set_shape(0, mgir.SHAPE_FUSE_SR, [0])
            s.set_shape(0, mgir.SHAPE_FUSE, [0])
        u, r = s.solve(bt, check=False)
        out = {"u": u}
        if max_iter == 1:
            assert r.status == mgir.MG_ERR_NOT_CONVERGED and r.iterations == 1
            out.update(bhat=s.read(0, mgir.BUF_RHS, torch.float16), bc=s.read(1, mgir.BUF_RHS, torch.float16),
                       r=s.read(0, mgir.BUF_RES))
        del s
        torch.cuda.empty_cache()
        return out, r

    for max_iter in (1, 100):
        print(f"  max_iter {max_iter}", flush=True)
        a, ra = run(True, max_iter)
        b_, rb = run(False, max_iter)
        for key in a:
            assert torch.equal(a[key], b_[key]), (max_iter, key)
        assert ra.iterations == rb.iterations
        assert np.allclose(ra.history, rb.history, rtol=1e-13, atol=0)
        del a, b_
        torch.cuda.empty_cache()


@pytest.mark.parametrize("scale", [1e-6, 1e-9])
def test_fp16_without_residual_scaling_stalls(dev, scale):
    """Section 4.3: without scaling, residual entries below FP16's range flush
    to zero in the low-precision correction equation, so refinement stalls;
    with alpha = ||r||_inf the same FP16 V-cycles converge.  (A normal status
    return, MG_ERR_NOT_CONVERGED.)"""
    n = 127
    print(f"FP16 without scaling, RHS scale {scale:g}", flush=True)
    b = scale * W.uniform_rhs(3, n, seed=5)
    bt = torch.from_numpy(b).to(dev)
    prec = W.precision_map("f16", W.levels_for(n))
    _, on = mgir.Solver(3, n, prec, residual_scaling=True).solve(bt)
    _, off = mgir.Solver(3, n, prec, residual_scaling=False, max_iter=40).solve(bt, check=False)
    print(f"  scaled: {on.iterations} it; unscaled: status {off.status}, rel {off.rel_residual:.2e}", flush=True)
    assert on.status == mgir.MG_OK and on.rel_residual <= 1e-10
    assert off.status == mgir.MG_ERR_NOT_CONVERGED
    assert off.rel_residual > 1e3 * on.rel_residual


@pytest.mark.parametrize("disc,n", [("fd", 2047), ("q1", 6143)])
def test_fp16_on_large_2d_grids_stays_in_range(dev, ref, disc, n):
    """2-D grids whose correction bound exceeds FP16's range for a right-hand
    side of max-norm one (the paper's k = 1 sine from u0 = 0; 6143^2 is its
    largest Q1 mesh): the range-safe alpha keeps the FP16 levels finite and the
    solve reaches 1e-10 within two iterations of FP64."""
    print(f"2-D {disc} n={n}, k=1 sine, FP16 levels", flush=True)
    b = W.manufactured_rhs(2, n, 1)
    if disc == "q1":
        b = b / float(n + 1) ** 2   # lumped load vector h^2 f
    bt = torch.from_numpy(b).to(dev)
    L = mgir.full_levels(n)
    s16 = mgir.Solver(2, n, W.precision_map("f16", L), disc=disc)
    assert s16.alpha_shift() >= 1
    u16, r16 = s16.solve(bt)
    _, r64 = mgir.Solver(2, n, W.precision_map("f64", L), disc=disc, residual_scaling=False).solve(bt)
    rel = _oracle_rel(ref, b, u16.cpu().numpy(), disc)
    print(f"  shift {s16.alpha_shift()}: f16 {r16.iterations} it rel {rel:.3e}; f64 {r64.iterations} it", flush=True)
    assert r16.status == mgir.MG_OK and rel <= 1e-10
    assert r16.iterations <= r64.iterations + 2
