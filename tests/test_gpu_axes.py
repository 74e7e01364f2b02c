"""The paper's test axes (Section 6): oscillatory manufactured solutions
k = 1, 20, 400 and a random initial guess in [0, 1].

Pins: the FP64 solve against the oracle's IR from the same initial guess, and
the closed form of the discrete solution (a sine mode is an eigenvector of the
discrete Laplacian, so u = f / lambda_k exactly); the FP16 solve reaches the
tolerance within two iterations of the FP64 one."""
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


def _discrete_solution(dim, n, k):
    """The sine mode is an eigenvector of the discrete Laplacian with
    eigenvalue dim (4/h^2) sin^2(k pi h/2), so A u = f is solved by f / lambda;
    also returns lambda_k / lambda_min, which bounds the relative error of u by
    that many times the relative residual (||e|| <= ||r|| / lambda_min and
    ||u|| = ||f|| / lambda_k)."""
    h = 1.0 / (n + 1)
    lam = dim * 4.0 / h**2 * np.sin(k * np.pi * h / 2) ** 2
    lam_min = dim * 4.0 / h**2 * np.sin(np.pi * h / 2) ** 2
    return dim * (k * np.pi) ** 2 / lam * W.sine_mode(dim, n, (k, k, k)), lam / lam_min


@pytest.mark.parametrize("dim,n", [(3, 63), (2, 255)])
@pytest.mark.parametrize("k", [1, 20, 400])
def test_axes_fp64_matches_oracle_and_closed_form(dev, ref, dim, n, k):
    print(f"axes f64 dim={dim} n={n} k={k}", flush=True)
    b = W.manufactured_rhs(dim, n, k)
    u0 = W.random_initial_guess(dim, n, seed=100 + k)
    s = mgir.Solver(dim, n, W.precision_map("f64", W.levels_for(n)), residual_scaling=False,
                    use_initial_guess=True)
    u, res = s.solve(torch.from_numpy(b).to(dev), torch.from_numpy(u0).to(dev))
    u = u.cpu().numpy()
    o = ref.ir_solve(b, u0, residual_scaling=False, recursive_residual=True)
    assert res.status == 0 and o.status == 0
    assert abs(res.iterations - o.iterations) <= 1
    if res.iterations == o.iterations:
        assert rel_err(u, o.u) <= 1e-12
    rel = ref.norm2(ref.residual(b, u)) / ref.norm2(b)
    assert rel <= 1e-10
    exact, ratio = _discrete_solution(dim, n, k)
    assert np.linalg.norm(u - exact) / np.linalg.norm(exact) <= 1.01 * ratio * rel


@pytest.mark.parametrize("name", ["f16", "h_mg", "bf16"])
@pytest.mark.parametrize("k", [1, 20, 400])
def test_axes_mixed_reach_tolerance(dev, ref, name, k):
    n = 63
    print(f"axes {name} n={n} k={k}", flush=True)
    b = W.manufactured_rhs(3, n, k)
    u0 = W.random_initial_guess(3, n, seed=200 + k)
    bt, u0t = torch.from_numpy(b).to(dev), torch.from_numpy(u0).to(dev)
    _, r64 = mgir.Solver(3, n, W.precision_map("f64", W.levels_for(n)), residual_scaling=False,
                         use_initial_guess=True).solve(bt, u0t.clone())
    u, res = mgir.Solver(3, n, W.precision_map(name, W.levels_for(n)), use_initial_guess=True).solve(bt, u0t.clone())
    assert res.status == 0
    rel = ref.norm2(ref.residual(b, u.cpu().numpy())) / ref.norm2(b)
    assert rel <= 1e-10
    assert res.iterations <= r64.iterations + 2
