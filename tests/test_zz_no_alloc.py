"""mg_vcycle_noalloc (GPU): the V-cycle on the library's own device array
equals mg_vcycle on a bound workspace bit for bit, on consecutive calls of
different sizes and formats (the second smaller than the first, so the array
holds the first call's values where the second has its ghost cells), and
leaves the handle's bound workspace as it was.  Sizes beyond the array are
refused before any device work."""
import pytest
import torch

from paper_2007_07539_amd import mgir
from paper_2007_07539_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(dev, name, n, seed):
    prec = W.precision_map(name, W.levels_for(n))
    s = mgir.Solver(3, n, prec, device=dev)
    b = torch.from_numpy(W.uniform_rhs(3, n, seed=seed)).to(dev).to(mgir.TORCH_DTYPE[prec[0]])
    return s, b


def test_noalloc_vcycle_matches_bound_workspace(dev):
    # largest first, then smaller ones, then the first again
    cases = [("f16", 255, 21), ("f64", 127, 22), ("f16", 63, 23), ("bf16", 31, 24), ("h_mg", 15, 25),
             ("f16", 255, 21)]
    for name, n, seed in cases:
        print(f"no-alloc V-cycle {name} n={n}", flush=True)
        s, b = _case(dev, name, n, seed)
        ref = s.vcycle(b).clone()
        cor = s.read(0, mgir.BUF_COR, torch.float64)
        got = s.vcycle_noalloc(b)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (name, n)
        # the bound workspace still holds what mg_vcycle left there
        assert torch.equal(s.read(0, mgir.BUF_COR, torch.float64), cor), (name, n)
        # and a second call in a row gives the same again
        assert torch.equal(s.vcycle_noalloc(b), ref), (name, n)
        del s


def test_noalloc_vcycle_refuses_large_hierarchies(dev):
    s = mgir.Solver(3, 511, W.precision_map("f16", W.levels_for(511)), device=dev)
    b = torch.zeros((511,) * 3, dtype=torch.float16, device=dev)
    with pytest.raises(mgir.MgError) as e:
        s.vcycle_noalloc(b)
    assert e.value.status == mgir.MG_ERR_WORKSPACE
