"""GPU parity at the full 511^3 size of the benchmark, in the launch
configuration bench.py times (autotuned shapes, fused coarse end, fused last
sweep + update).  The oracle evaluates each compared output over the whole
grid (one serial C pass, a few seconds); the solve is checked through its
true residual, a property that holds at any size.

Host memory: about ten FP64 arrays of 511^3 (1.07 GB each)."""
import gc

import numpy as np
import pytest
import torch

from paper_2007_07539_amd import mgir
from paper_2007_07539_amd import workloads as W
from tests.helpers import TOL, rel_err, round_to

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 511


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _put(s, level, buf, x, dev):
    s.write(level, buf, torch.from_numpy(x).to(dev))
    return s.read(level, buf).cpu().numpy()


def test_fullsize_fp16_kernels(dev, ref):
    """One sweep, one residual + restriction and one prolongation + sweep of
    the finest FP16 level at 511^3 against the oracle on the same inputs."""
    print("full-size kernels, f16, n=511", flush=True)
    prec = W.precision_map("f16", W.levels_for(N))
    s = mgir.Solver(3, N, prec, autotune=True)
    rng = np.random.default_rng(900)
    h2 = (1.0 / (N + 1)) ** 2
    bq = _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (N,) * 3), dev)
    cq = _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (N,) * 3), dev)
    # residual + restriction first (it leaves b and c in place)
    s.stage(mgir.STAGE_RESTRICT, 0)
    torch.cuda.synchronize()
    out = s.read(1, mgir.BUF_RHS).cpu().numpy()
    r = ref.residual(bq, cq * h2)
    assert rel_err(out, ref.restrict(r)) <= TOL["f16"]
    del out, r
    gc.collect()
    s.stage(mgir.STAGE_SWEEP, 0)
    torch.cuda.synchronize()
    out = s.read(0, mgir.BUF_COR).cpu().numpy()
    assert rel_err(out, ref.jacobi(bq, cq * h2, 0.8) / h2) <= TOL["f16"]
    del out
    gc.collect()
    nc = (N - 1) // 2
    hc2 = (1.0 / (nc + 1)) ** 2
    cq = _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (N,) * 3), dev)
    ecq = _put(s, 1, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (nc,) * 3), dev)
    s.stage(mgir.STAGE_PROLONG_SWEEP, 0)
    torch.cuda.synchronize()
    out = s.read(0, mgir.BUF_COR).cpu().numpy()
    corrected = round_to((cq * h2 + ref.prolong(ecq * hc2)) / h2, "f16")
    assert rel_err(out, ref.jacobi(bq, corrected * h2, 0.8) / h2) <= TOL["f16"]
    del s
    gc.collect()
    torch.cuda.empty_cache()


def test_fullsize_fp64_vcycle(dev, ref):
    """A whole FP64 V-cycle at 511^3 (nine levels, fused coarse end) against
    the oracle's recursive V-cycle."""
    print("full-size V-cycle, f64, n=511", flush=True)
    s = mgir.Solver(3, N, W.precision_map("f64", W.levels_for(N)), residual_scaling=False, autotune=True)
    b = W.uniform_rhs(3, N, seed=901)
    c = s.vcycle(torch.from_numpy(b).to(dev)).cpu().numpy()
    assert rel_err(c * (1.0 / (N + 1)) ** 2, ref.vcycle(b)) <= 1e-12
    del s
    torch.cuda.empty_cache()


def test_fullsize_solves(dev, ref):
    """The benchmark solve: FP16 V-cycles reach 1e-10 by the oracle's own
    residual within the FP64 solve's iteration count + 2."""
    print("full-size IR solves, n=511", flush=True)
    b = W.poisson3d_sine_noise_rhs(N, seed=3)
    bt = torch.from_numpy(b).to(dev)
    u16, r16 = mgir.Solver(3, N, W.precision_map("f16", W.levels_for(N)), autotune=True).solve(bt)
    u64, r64 = mgir.Solver(3, N, W.precision_map("f64", W.levels_for(N)), residual_scaling=False,
                           autotune=True).solve(bt)
    assert r16.iterations <= r64.iterations + 2
    u = u16.cpu().numpy()
    rel = ref.norm2(ref.residual(b, u)) / ref.norm2(b)
    print(f"oracle relative residual of the FP16 solve: {rel:.3e}", flush=True)
    assert rel <= 1e-10
    assert r16.rel_residual == pytest.approx(rel, rel=1e-6)
    # both solves approximate the same discrete solution to the tolerance
    assert rel_err(u, u64.cpu().numpy()) <= 1e-8
