"""Several V-cycles per refinement step (cycles_per_step): each further cycle
continues from the correction so far on the same scaled residual before u and
r are updated once.  Pinned against the oracle's IR with the same number of
cycles per step (whose own pin is that a step of m cycles equals m one-cycle
steps), and checked to compose bitwise with the fused kernels and the graphs."""
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


@pytest.mark.parametrize("dim,n", [(3, 63), (2, 255)])
@pytest.mark.parametrize("m", [2, 3])
def test_cycles_fp64_matches_oracle(dev, ref, dim, n, m):
    print(f"cycles f64 dim={dim} n={n} m={m}", flush=True)
    b = W.uniform_rhs(dim, n, seed=110 + m)
    s = mgir.Solver(dim, n, W.precision_map("f64", W.levels_for(n)), residual_scaling=False, cycles_per_step=m)
    u, res = s.solve(torch.from_numpy(b).to(dev))
    u = u.cpu().numpy()
    o = ref.ir_solve(b, residual_scaling=False, recursive_residual=True, cycles=m)
    assert res.status == 0 and o.status == 0
    assert abs(res.iterations - o.iterations) <= 1
    if res.iterations == o.iterations:
        assert rel_err(u, o.u) <= 1e-12
    assert ref.norm2(ref.residual(b, u)) / ref.norm2(b) <= 1e-10


@pytest.mark.parametrize("name", ["f16", "bf16", "hsd", "f32"])
@pytest.mark.parametrize("m", [2, 3])
def test_cycles_mixed_reach_tolerance(dev, ref, name, m):
    n = 127
    print(f"cycles {name} n={n} m={m}", flush=True)
    b = W.uniform_rhs(3, n, seed=120)
    bt = torch.from_numpy(b).to(dev)
    _, r64 = mgir.Solver(3, n, W.precision_map("f64", W.levels_for(n)), residual_scaling=False,
                         cycles_per_step=m).solve(bt)
    u, res = mgir.Solver(3, n, W.precision_map(name, W.levels_for(n)), cycles_per_step=m).solve(bt)
    assert res.status == 0
    assert ref.norm2(ref.residual(b, u.cpu().numpy())) / ref.norm2(b) <= 1e-10
    assert res.iterations <= r64.iterations + 2


@pytest.mark.parametrize("name,n", [("f16", 63), ("bf16", 31), ("f32", 127)])
def test_cycles_compose_with_fusions_and_graphs(dev, name, n):
    """Fused first smoothing + restriction, fused last sweep + update, graph or
    eager: the iterates of a two-cycle solve do not change."""
    print(f"cycles composition {name} n={n}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    b = torch.from_numpy(W.uniform_rhs(3, n, seed=121)).to(dev)
    ref_u, ref_r = mgir.Solver(3, n, prec, cycles_per_step=2).solve(b)
    ref_u = ref_u.clone()
    s = mgir.Solver(3, n, prec, cycles_per_step=2)
    s.set_shape(0, mgir.SHAPE_FUSE, [0])
    s.set_shape(0, mgir.SHAPE_FUSE_SR, [0])
    s.set_shape(0, mgir.SHAPE_TAIL, [0])
    u, r = s.solve(b)
    assert r.iterations == ref_r.iterations and torch.equal(u, ref_u)
    assert np.allclose(r.history, ref_r.history, rtol=1e-13, atol=0)
    u2, r2 = mgir.Solver(3, n, prec, cycles_per_step=2, use_graph=False).solve(b)
    assert r2.iterations == ref_r.iterations and torch.equal(u2, ref_u)
    assert r2.history == ref_r.history
