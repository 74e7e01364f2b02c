"""The bandwidth probes that calibrate the traffic counters and measure the
streaming ceilings do the work they claim (so their bytes are real)."""
import pytest
import torch

from paper_2007_07539_amd import mgir

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_copy_and_write_probes(dev):
    src = torch.arange(4096, dtype=torch.float64, device=dev)
    dst = torch.zeros_like(src)
    mgir.bandwidth_probe(dst, src, 0, blocks=7)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_update_mix_probe(dev):
    n = 4096
    g = torch.Generator(device="cpu").manual_seed(5)
    ru = torch.rand(2 * n, dtype=torch.float64, generator=g).to(dev)
    cb = torch.rand(2 * n, generator=g).to(torch.float16).to(dev)
    r0, u0 = ru[:n].clone(), ru[n:].clone()
    c, b = cb[:n].double(), cb[n:].double()
    mgir.bandwidth_probe(ru, cb, 3, blocks=5)
    torch.cuda.synchronize()
    assert torch.allclose(ru[:n], r0 - c * b, rtol=0, atol=1e-15)
    assert torch.equal(ru[n:], u0 + c)
