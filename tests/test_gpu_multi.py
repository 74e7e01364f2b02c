"""GPU: many right-hand sides on one grid, stored interleaved [z, y, x, k],
through mg_setup_multi / ir_solve_multi.

Column k runs the arithmetic of a single-grid solve of right-hand side k
(same sums, same roundings, its own alpha_k), so where the iteration counts
agree its solution must equal the single-grid solution bit for bit (the norms
behind the stop test are reduced in another order, so a count could differ
only when a residual lands within rounding of the tolerance).  The
single-grid path is held to the oracle in test_gpu_parity; one FP64 case is
also checked against the oracle directly.
"""
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


def _true_rel(ref, b, u):
    return ref.norm2(ref.residual(b, u)) / ref.norm2(b)


def _rhs(n, k, seed, emax=0.0):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-emax, emax, k)
    return np.stack([(10.0 ** e[j]) * rng.uniform(-1, 1, (n,) * 3) for j in range(k)], axis=-1)


def _compare_columns(dev, n, prec, b, u, res, cols, **kw):
    for j in cols:
        bj = torch.from_numpy(np.ascontiguousarray(b[..., j])).to(dev)
        u1, r1 = mgir.Solver(3, n, prec, **kw).solve(bj, check=False)
        assert r1.status == 0, j
        if res[j].iterations == r1.iterations:
            assert torch.equal(u[..., j].contiguous(), u1), j
        else:  # a stop decision within rounding of the tolerance
            assert abs(res[j].iterations - r1.iterations) == 1, j


@pytest.mark.parametrize("name", ["f64", "f32", "f16", "bf16", "hsd", "h_mg"])
@pytest.mark.parametrize("n,k", [(15, 8), (31, 16)])
def test_multi_matches_single(dev, name, n, k):
    print(f"multi {name} n={n} k={k}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    scaling = name != "f64"
    b = _rhs(n, k, 300 + n, emax=3.0)
    ms = mgir.MultiSolver(n, k, prec, residual_scaling=scaling)
    u, res, status = ms.solve(torch.from_numpy(b).to(dev))
    assert status == 0
    assert max(r.rel_residual for r in res) <= 1e-10
    _compare_columns(dev, n, prec, b, u, res, range(k), residual_scaling=scaling)


def test_multi_fp64_against_oracle(dev, ref):
    n, k = 15, 4
    b = _rhs(n, k, 310)
    u, res, status = mgir.MultiSolver(n, k, ["f64"] * 4, residual_scaling=False).solve(torch.from_numpy(b).to(dev))
    assert status == 0
    u = u.cpu().numpy()
    for j in range(k):
        o = ref.ir_solve(np.ascontiguousarray(b[..., j]), residual_scaling=False, recursive_residual=True)
        assert abs(res[j].iterations - o.iterations) <= 1
        uj = np.ascontiguousarray(u[..., j])
        assert _true_rel(ref, b[..., j], uj) <= 1e-10
        if res[j].iterations == o.iterations:
            assert rel_err(uj, o.u) <= 1e-12


def test_multi_graph_eager_and_repeat(dev):
    n, k = 31, 8
    prec = W.precision_map("f16", W.levels_for(n))
    b = torch.from_numpy(_rhs(n, k, 320, emax=2.0)).to(dev)
    g = mgir.MultiSolver(n, k, prec, use_graph=True)
    ug, rg, _ = g.solve(b)
    ue, re_, _ = mgir.MultiSolver(n, k, prec, use_graph=False).solve(b)
    ug2, rg2, _ = g.solve(b)
    assert torch.equal(ug, ue) and torch.equal(ug, ug2)
    for j in range(k):
        assert rg[j].history == re_[j].history == rg2[j].history


def test_multi_edge_cases(dev):
    """A zero column, a non-finite column, an iteration cap and a resumed solve."""
    n, k = 15, 8
    prec = W.precision_map("f16", W.levels_for(n))
    b = _rhs(n, k, 330, emax=4.0)
    b[..., 2] = 0.0
    bt = torch.from_numpy(b).to(dev)
    ms = mgir.MultiSolver(n, k, prec)
    u, res, status = ms.solve(bt)
    assert status == 0
    assert res[2].iterations == 0 and res[2].rel_residual == 0.0 and not u[..., 2].any()
    _compare_columns(dev, n, prec, b, u, res, [0, 1, 3, 7])
    bad = bt.clone()
    bad[1, 2, 3, 5] = float("nan")
    u, res, status = ms.solve(bad, check=False)
    assert status == mgir.MG_ERR_NONFINITE
    assert not u[..., 5].any()
    assert all(res[j].rel_residual <= 1e-10 for j in range(k) if j not in (5,))
    capped = mgir.MultiSolver(n, k, prec, max_iter=2)
    uc, rc, status = capped.solve(bt, check=False)
    assert status == mgir.MG_ERR_NOT_CONVERGED
    assert all(rc[j].iterations == 2 for j in range(k) if j != 2)
    resumed = mgir.MultiSolver(n, k, prec, use_initial_guess=True)
    ur, rr, status = resumed.solve(bt, uc.clone())
    assert status == 0
    for j in (0, 4):
        u1, r1 = mgir.Solver(3, n, prec, use_initial_guess=True).solve(
            bt[..., j].contiguous(), uc[..., j].contiguous())
        if rr[j].iterations == r1.iterations:
            assert torch.equal(ur[..., j].contiguous(), u1)


def test_multi_64_columns(dev):
    n, k = 7, 64
    prec = W.precision_map("f16", W.levels_for(n))
    b = _rhs(n, k, 340, emax=6.0)
    u, res, status = mgir.MultiSolver(n, k, prec).solve(torch.from_numpy(b).to(dev))
    assert status == 0
    _compare_columns(dev, n, prec, b, u, res, [0, 17, 63])


@pytest.mark.slow
def test_multi_workload_127_32(dev, ref):
    """127^3 with 32 right-hand sides scaled by 10^e, e uniform in [-6, 6],
    FP16 V-cycles: every column reaches 1e-10 within the FP64 count + 2, and
    sampled columns equal their single-grid solves."""
    n, k = 127, 32
    b = W.multi_rhs(n, k, seed=5)
    bt = torch.from_numpy(b).to(dev)
    prec = W.precision_map("f16", W.levels_for(n))
    u, res, status = mgir.MultiSolver(n, k, prec).solve(bt)
    assert status == 0
    _, r64, st64 = mgir.MultiSolver(n, k, ["f64"] * 7, residual_scaling=False).solve(bt)
    assert st64 == 0
    for j in range(k):
        assert res[j].rel_residual <= 1e-10
        assert res[j].iterations <= r64[j].iterations + 2
    _compare_columns(dev, n, prec, b, u, res, [0, 13, 31])
    uj = u[..., 0].contiguous().cpu().numpy()
    assert _true_rel(ref, np.ascontiguousarray(b[..., 0]), uj) <= 1e-10


@pytest.mark.parametrize("name", ["f16", "f64"])
def test_multi_autotuned_bitwise_and_cached(dev, tmp_path, monkeypatch, name):
    """The many-right-hand-side autotuner times each level's planes per thread
    over whole steps; the choice only cuts the work differently, so the tuned
    handle's solution equals the untuned one bit for bit.  With MGIR_TUNE_CACHE
    set the choice is stored once and read back by a second handle."""
    n, k = 31, 16
    print(f"multi autotune {name} n={n} k={k}", flush=True)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MGIR_TUNE_CACHE", str(path))
    prec = W.precision_map(name, W.levels_for(n))
    scaling = name != "f64"
    b = torch.from_numpy(_rhs(n, k, 320, emax=2.0)).to(dev)
    tuned = mgir.MultiSolver(n, k, prec, residual_scaling=scaling, autotune=True)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "|multi|" in lines[0]
    kinds = (mgir.SHAPE_SMOOTH, mgir.SHAPE_SWEEP, mgir.SHAPE_PROLONG, mgir.SHAPE_RESTRICT)

    def shapes(s):
        return [s.get_shape(l, kk) for l in range(W.levels_for(n) - 1) for kk in kinds]

    again = mgir.MultiSolver(n, k, prec, residual_scaling=scaling, autotune=True)
    assert path.read_text().splitlines() == lines
    assert shapes(again) == shapes(tuned)
    ut, rt, st = tuned.solve(b)
    up, rp, sp = mgir.MultiSolver(n, k, prec, residual_scaling=scaling).solve(b)
    ua, ra, sa = again.solve(b)
    assert st == sp == sa == 0
    for j in range(k):
        assert rt[j].history == rp[j].history == ra[j].history, j
    assert torch.equal(ut, up) and torch.equal(ut, ua)
    assert max(r.rel_residual for r in rt) <= 1e-10
