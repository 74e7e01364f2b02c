"""GPU: batched instances of uneven sizes (one launch per V-cycle stage over
all instances) through mg_setup_batched / ir_solve_batched.

Each instance must compute bit for bit what a single-grid solver of its size
and level map computes (the batched launches run the same per-tile device
code), so the comparison is exact equality of u and of the iteration count;
the single-grid path itself is held to the oracle in test_gpu_parity.  One
FP64 case is also compared with the oracle directly.
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


def _single(n, prec, b, **kw):
    return mgir.Solver(3, n, prec, **kw).solve(b, check=False)


SIZES = [15, 3, 63, 7, 31, 15, 127, 7]


@pytest.mark.parametrize("name", ["f64", "f32", "f16", "bf16", "hsd", "h_mg"])
def test_batched_matches_single_bitwise(dev, name):
    print(f"batched {name} sizes={SIZES}", flush=True)
    lmax = max(W.levels_for(n) for n in SIZES)
    prec = W.precision_map(name, lmax)
    scaling = name != "f64"
    rng = np.random.default_rng(200)
    bs = [torch.from_numpy(rng.uniform(-1, 1, (n,) * 3)).to(dev) for n in SIZES]
    bsv = mgir.BatchedSolver(SIZES, prec, residual_scaling=scaling)
    us, res, status = bsv.solve(bs)
    assert status == 0
    for i, n in enumerate(SIZES):
        u1, r1 = _single(n, bsv.instance_prec(i), bs[i], residual_scaling=scaling)
        assert r1.status == 0
        assert res[i].iterations == r1.iterations, (i, n)
        assert torch.equal(us[i], u1), (i, n)
        assert res[i].rel_residual == r1.rel_residual
        assert res[i].rel_residual <= 1e-10


def test_batched_fp64_against_oracle(dev, ref):
    sizes = [7, 15, 31]
    rng = np.random.default_rng(201)
    bs = [rng.uniform(-1, 1, (n,) * 3) for n in sizes]
    bsv = mgir.BatchedSolver(sizes, ["f64"] * 5, residual_scaling=False)
    us, res, status = bsv.solve([torch.from_numpy(b).to(dev) for b in bs])
    assert status == 0
    for b, u, r in zip(bs, us, res):
        o = ref.ir_solve(b, residual_scaling=False, recursive_residual=True)
        u = u.cpu().numpy()
        assert abs(r.iterations - o.iterations) <= 1
        assert _true_rel(ref, b, u) <= 1e-10
        if r.iterations == o.iterations:
            assert rel_err(u, o.u) <= 1e-12


def test_batched_graph_eager_and_repeat(dev):
    sizes = [31, 7, 63, 15]
    prec = W.precision_map("f16", 6)
    rng = np.random.default_rng(202)
    bs = [torch.from_numpy(rng.uniform(-1, 1, (n,) * 3)).to(dev) for n in sizes]
    g = mgir.BatchedSolver(sizes, prec, use_graph=True)
    ug, rg, _ = g.solve(bs)
    ue, re_, _ = mgir.BatchedSolver(sizes, prec, use_graph=False).solve(bs)
    ug2, rg2, _ = g.solve(bs)  # the captured graph replayed on a second solve
    for i in range(len(sizes)):
        assert torch.equal(ug[i], ue[i]) and torch.equal(ug[i], ug2[i])
        assert rg[i].history == re_[i].history == rg2[i].history


def test_batched_edge_cases(dev):
    """Zero right-hand side, a non-finite one, an iteration cap and an initial
    guess, mixed in one batch with ordinary instances."""
    sizes = [15, 7, 15, 31]
    prec = W.precision_map("f16", 5)
    rng = np.random.default_rng(203)
    bs = [torch.from_numpy(rng.uniform(-1, 1, (n,) * 3)).to(dev) for n in sizes]
    bs[1].zero_()
    us = [torch.full_like(b, 2.0) for b in bs]
    bsv = mgir.BatchedSolver(sizes, prec)
    us, res, status = bsv.solve(bs, us)
    assert status == 0
    assert res[1].iterations == 0 and res[1].rel_residual == 0.0 and not us[1].any()
    for i in (0, 2, 3):
        u1, r1 = _single(sizes[i], bsv.instance_prec(i), bs[i])
        assert torch.equal(us[i], u1) and res[i].iterations == r1.iterations
    bad = [b.clone() for b in bs]
    bad[2][1, 2, 3] = float("nan")
    _, res, status = bsv.solve(bad, check=False)
    assert status == mgir.MG_ERR_NONFINITE
    assert res[0].rel_residual <= 1e-10 and res[3].rel_residual <= 1e-10
    capped = mgir.BatchedSolver(sizes, prec, max_iter=2)
    us, res, status = capped.solve(bs, check=False)
    assert status == mgir.MG_ERR_NOT_CONVERGED
    assert all(r.iterations == 2 for i, r in enumerate(res) if i != 1)
    assert all(torch.isfinite(u).all() for u in us)
    # resume every instance from its capped iterate
    resumed = mgir.BatchedSolver(sizes, prec, use_initial_guess=True)
    us2, res2, status = resumed.solve(bs, [u.clone() for u in us])
    assert status == 0
    for i in (0, 2, 3):
        u1, r1 = mgir.Solver(3, sizes[i], bsv.instance_prec(i), use_initial_guess=True).solve(bs[i], us[i].clone())
        assert torch.equal(us2[i], u1) and res2[i].iterations == r1.iterations
        assert res2[i].rel_residual <= 1e-10


@pytest.mark.slow
def test_batched_workload_64_instances(dev, ref):
    """64 instances drawn from {63, 127, 255}^3 with FP16 corrections: all
    converge within the FP64 count + 2, and one instance of each size is
    identical to its single-grid solve."""
    ns, rhs = W.batched_instances()
    print(f"batched 64 instances, sizes {sorted(set(ns))}", flush=True)
    prec = W.precision_map("f16", 8)
    bs = [torch.from_numpy(r).to(dev) for r in rhs]
    bsv = mgir.BatchedSolver(ns, prec)
    us, res, status = bsv.solve(bs)
    assert status == 0
    assert max(r.rel_residual for r in res) <= 1e-10
    for n in sorted(set(ns)):
        i = ns.index(n)
        u1, r1 = _single(n, bsv.instance_prec(i), bs[i])
        assert torch.equal(us[i], u1) and res[i].iterations == r1.iterations
        _, r64 = _single(n, ["f64"] * W.levels_for(n), bs[i], residual_scaling=False)
        assert res[i].iterations <= r64.iterations + 2
        # sampled true residual from the oracle on the smallest instance
        if n == 63:
            assert _true_rel(ref, rhs[i], us[i].cpu().numpy()) <= 1e-10
    del us, bsv
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["f16", "f64"])
def test_batched_autotuned_bitwise_and_cached(dev, tmp_path, monkeypatch, name):
    """The batched autotuner picks launch shapes per class of levels (pitch and
    format) by timing whole batched steps; every shape forms the same
    roundings, so the tuned handle's solutions equal the untuned handle's and
    each instance's single-grid solve bit for bit.  With MGIR_TUNE_CACHE set the
    choice is stored once and a second handle reads it back."""
    sizes = [63, 7, 127, 15, 63]
    print(f"batched autotune {name} sizes={sizes}", flush=True)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MGIR_TUNE_CACHE", str(path))
    lmax = max(W.levels_for(n) for n in sizes)
    prec = W.precision_map(name, lmax)
    scaling = name != "f64"
    rng = np.random.default_rng(205)
    bs = [torch.from_numpy(rng.uniform(-1, 1, (n,) * 3)).to(dev) for n in sizes]
    tuned = mgir.BatchedSolver(sizes, prec, residual_scaling=scaling, autotune=True)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "|batched|" in lines[0]
    kinds = (mgir.SHAPE_SMOOTH, mgir.SHAPE_SWEEP, mgir.SHAPE_PROLONG, mgir.SHAPE_RESTRICT)

    def shapes(s):
        return [s.get_shape(i, l, k) for i, n in enumerate(sizes) for l in range(W.levels_for(n) - 1) for k in kinds]

    # one shape per tuned class (pitch >= 16): every level of the class takes it
    sh = shapes(tuned)
    per = {}
    for i, n in enumerate(sizes):
        for l in range(W.levels_for(n) - 1):
            if (n + 1) >> l < 16:
                continue
            key = ((n + 1) >> l, tuned.instance_prec(i)[l])
            val = [tuned.get_shape(i, l, k) for k in kinds]
            assert per.setdefault(key, val) == val, (i, l)
    again = mgir.BatchedSolver(sizes, prec, residual_scaling=scaling, autotune=True)
    assert path.read_text().splitlines() == lines  # read back, not tuned again
    assert shapes(again) == sh
    plain = mgir.BatchedSolver(sizes, prec, residual_scaling=scaling)
    ut, rt, st = tuned.solve(bs)
    up, rp, sp = plain.solve(bs)
    ua, ra, sa = again.solve(bs)
    assert st == sp == sa == 0
    for i, n in enumerate(sizes):
        assert rt[i].history == rp[i].history == ra[i].history, (i, n)
        assert torch.equal(ut[i], up[i]) and torch.equal(ut[i], ua[i]), (i, n)
        u1, r1 = _single(n, tuned.instance_prec(i), bs[i], residual_scaling=scaling)
        assert r1.iterations == rt[i].iterations and torch.equal(ut[i], u1), (i, n)
        assert rt[i].rel_residual <= 1e-10
