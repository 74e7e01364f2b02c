"""Partial hierarchies with the CG base solver on a multi-point base level
(Section 4.2; the paper's grids coarsen to such a base).  Pinned against the
oracle's CG (itself pinned to dense solves): in grid-scaled units the base
system has the residual of the physical one and CG is invariant under scaling
of the operator, so both stop after the same steps and agree to rounding."""
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


@pytest.mark.parametrize("dim,n,nl,prec,tol", [(3, 31, 3, "f64", 1e-10), (2, 63, 3, "f64", 1e-10),
                                               (3, 63, 3, "f32", 1e-3), (2, 127, 4, "f32", 1e-3)])
def test_cg_base_stage_matches_oracle(dev, ref, dim, n, nl, prec, tol):
    print(f"cg base stage dim={dim} n={n} nl={nl} {prec}", flush=True)
    s = mgir.Solver(dim, n, ["f64"] * (nl - 1) + [prec], nlevels=nl,
                    base_tol=1e-12 if prec == "f64" else 1e-5, base_max_iter=5000)
    base = nl - 1
    nb = s.level_n(base)
    b = W.uniform_rhs(dim, nb, seed=130 + nb)
    s.write(base, mgir.BUF_RHS, torch.from_numpy(b).to(dev))
    s.stage(mgir.STAGE_COARSE, base)
    torch.cuda.synchronize()
    x = s.read(base, mgir.BUF_COR).cpu().numpy()
    hb2 = (1.0 / (nb + 1)) ** 2
    xo, _ = ref.cg(b, 1e-12 if prec == "f64" else 1e-5)
    # the GPU solves L x = b with L = h^2 A, the oracle A e = b: x = e / h^2
    assert rel_err(x * hb2, xo) <= tol


@pytest.mark.parametrize("dim,n,nl", [(3, 31, 3), (3, 63, 4), (2, 255, 5)])
def test_vcycle_with_cg_base_matches_oracle(dev, ref, dim, n, nl):
    print(f"vcycle cg base dim={dim} n={n} nl={nl}", flush=True)
    s = mgir.Solver(dim, n, ["f64"] * nl, nlevels=nl, base_tol=1e-13, base_max_iter=5000)
    b = W.uniform_rhs(dim, n, seed=140 + n)
    c = s.vcycle(torch.from_numpy(b).to(dev)).cpu().numpy()
    nb = s.level_n(nl - 1)
    e = ref.vcycle(b, base_n=nb, base_tol=1e-13, base_max_iter=5000)
    assert rel_err(c * (1.0 / (n + 1)) ** 2, e) <= 1e-10


@pytest.mark.parametrize("name", ["f64", "f16", "h_mg", "hsd"])
def test_solves_with_cg_base_reach_tolerance(dev, ref, name):
    n, nl = 127, 4  # base 15^3
    print(f"ir cg base {name} n={n} nl={nl}", flush=True)
    b = W.uniform_rhs(3, n, seed=150)
    bt = torch.from_numpy(b).to(dev)
    _, r64 = mgir.Solver(3, n, ["f64"] * nl, nlevels=nl, residual_scaling=False).solve(bt)
    o = ref.ir_solve(b, residual_scaling=False, recursive_residual=True, base_n=15)
    assert abs(r64.iterations - o.iterations) <= 1
    s = mgir.Solver(3, n, W.precision_map(name, nl), nlevels=nl, residual_scaling=name != "f64")
    u, res = s.solve(bt)
    assert res.status == 0
    assert ref.norm2(ref.residual(b, u.cpu().numpy())) / ref.norm2(b) <= 1e-10
    assert res.iterations <= r64.iterations + 2


@pytest.mark.parametrize("dim,n,nl", [(3, 63, 4), (2, 255, 5)])
def test_options_compose(dev, ref, dim, n, nl):
    """A CG base in FP16 reached through rescaled restrictions (DSH-type map),
    with two V-cycles per step: every option on at once still solves to the
    tolerance, within two steps of the FP64 solve of the same hierarchy."""
    print(f"composed options dim={dim} n={n} nl={nl}", flush=True)
    b = W.uniform_rhs(dim, n, seed=160)
    bt = torch.from_numpy(b).to(dev)
    _, r64 = mgir.Solver(dim, n, ["f64"] * nl, nlevels=nl, residual_scaling=False, cycles_per_step=2).solve(bt)
    s = mgir.Solver(dim, n, W.precision_map("dsh", nl), nlevels=nl, rescale_half=True, cycles_per_step=2)
    u, res = s.solve(bt)
    assert res.status == 0
    assert ref.norm2(ref.residual(b, u.cpu().numpy())) / ref.norm2(b) <= 1e-10
    assert res.iterations <= r64.iterations + 2
