"""GPU parity of the Q1 finite-element path (the paper's discretisation,
Section 5) and of the paper's grid family n = c 2^k - 1 (Section 6) against
the oracle, whose Q1 operator, restriction and V-cycle are pinned to
quadrature assembly, Kronecker definitions and dense solves.

Units: on level l the GPU holds c_l = h_l^(D-2) e_l / 2^(D l) (the grid-scaled
correction of the FE system, with full weighting in place of P^T); on the
finest level c = g e with g = h^(D-2), and b is the physical load vector."""
import numpy as np
import pytest
import torch

from paper_2007_07539_amd import mgir
from paper_2007_07539_amd import workloads as W
from tests.helpers import TOL, rel_err, round_to

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "f16", "bf16"]
ACC_TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 1e-6, "bf16": 1e-6}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _g(dim, n):
    return (1.0 / (n + 1)) ** (dim - 2)


def _solver(dim, n, fine, coarse=None, **kw):
    m = mgir.full_levels(n)
    prec = [fine] * m
    if coarse is not None:
        prec[1:] = [coarse] * (m - 1)
    return mgir.Solver(dim, n, prec, disc="q1", **kw)


def _put(s, level, buf, x, dev):
    s.write(level, buf, torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev))
    return s.read(level, buf).cpu().numpy()


def _get(s, level, buf):
    torch.cuda.synchronize()
    return s.read(level, buf).cpu().numpy()


def _true_rel(ref, b, u):
    return ref.norm2(ref.residual(b, u, "q1")) / ref.norm2(b)


# pitches that are multiples of 4 take the four-point and marching kernels,
# the others (n = 9, 21) the one-point-per-thread kernels
CASES = [(3, 7), (3, 15), (3, 63), (3, 95), (2, 15), (2, 255), (2, 383), (3, 9), (3, 21), (2, 9)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,n", CASES)
def test_q1_sweep(dev, ref, prec, dim, n):
    print(f"q1 sweep prec={prec} dim={dim} n={n}", flush=True)
    s = _solver(dim, n, prec)
    rng = np.random.default_rng(10 * n + dim)
    g = _g(dim, n)
    bq = _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (n,) * dim), dev)
    cq = _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (n,) * dim), dev)
    s.stage(mgir.STAGE_SWEEP, 0)
    out = _get(s, 0, mgir.BUF_COR)
    expect = ref.jacobi(bq, cq / g, 0.8, "q1") * g
    assert rel_err(out, expect) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,n", CASES)
def test_q1_smooth_first(dev, ref, prec, dim, n):
    print(f"q1 smooth_first prec={prec} dim={dim} n={n}", flush=True)
    s = _solver(dim, n, prec)
    rng = np.random.default_rng(20 * n + dim)
    g = _g(dim, n)
    bq = _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (n,) * dim), dev)
    s.stage(mgir.STAGE_SMOOTH_FIRST, 0)
    out = _get(s, 0, mgir.BUF_COR)
    c1 = round_to(ref.jacobi(bq, np.zeros_like(bq), 0.8, "q1") * g, prec)
    c2 = ref.jacobi(bq, c1 / g, 0.8, "q1") * g
    assert rel_err(out, c2) <= TOL[prec]


@pytest.mark.parametrize("pf,pc", [(a, b) for a in PRECS for b in PRECS])
@pytest.mark.parametrize("dim,n", [(3, 15), (3, 47), (2, 63), (2, 95), (3, 9), (3, 21), (2, 9)])
def test_q1_resid_restrict(dev, ref, pf, pc, dim, n):
    print(f"q1 restrict {pf}->{pc} dim={dim} n={n}", flush=True)
    s = _solver(dim, n, pf, pc)
    rng = np.random.default_rng(30 * n + dim)
    g = _g(dim, n)
    bq = _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (n,) * dim), dev)
    cq = _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (n,) * dim), dev)
    s.stage(mgir.STAGE_RESTRICT, 0)
    out = _get(s, 1, mgir.BUF_RHS)
    # full weighting = P^T / 2^D
    expect = ref.restrict(ref.residual(bq, cq / g, "q1"), "q1") / 2**dim
    assert rel_err(out, expect) <= max(TOL[pc], ACC_TOL[pf])


@pytest.mark.parametrize("pf,pc", [("f16", "f16"), ("f16", "f32"), ("bf16", "f64"), ("bf16", "bf16")])
@pytest.mark.parametrize("n", [31, 47, 63, 95, 127])
def test_q1_fused_restrict_bitwise(dev, pf, pc, n):
    """On 3-D levels in a 2-byte format the residual and its restriction run
    as one kernel (the fine residual kept in LDS); for several tile shapes,
    ragged last tiles and chunks included, the restricted b equals that of the
    two kernels bit for bit."""
    print(f"q1 fused restrict {pf}->{pc} n={n}", flush=True)
    s = _solver(3, n, pf, pc)
    assert s.get_shape(0, mgir.SHAPE_SWEEP) != [0, 0]  # a level with the LDS-staged kernels
    assert s.get_shape(0, mgir.SHAPE_RESTRICT, 3)[2] == 0  # fused by default
    rng = np.random.default_rng(31 * n)
    _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (n,) * 3), dev)
    _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (n,) * 3), dev)
    s.set_shape(0, mgir.SHAPE_RESTRICT, [0, 0, 1])
    assert s.get_shape(0, mgir.SHAPE_RESTRICT, 3)[2] == 1
    s.stage(mgir.STAGE_RESTRICT, 0)
    ref = s.read(1, mgir.BUF_RHS).clone()
    tried = 0
    for shape in ([0, 0], [2, 2], [4, 4], [2, 16], [6, 8], [4, 32], [8, 6]):
        try:
            s.set_shape(0, mgir.SHAPE_RESTRICT, shape)
        except mgir.MgError:
            continue
        tried += 1
        s.write(1, mgir.BUF_RHS, torch.full_like(ref, 7.0))
        s.stage(mgir.STAGE_RESTRICT, 0)
        assert torch.equal(s.read(1, mgir.BUF_RHS), ref), shape
    assert tried >= 3
    for bad in ([3, 4], [2, 3], [2, 4, 2]):
        with pytest.raises(mgir.MgError):
            s.set_shape(0, mgir.SHAPE_RESTRICT, bad)


@pytest.mark.parametrize("pf,pc", [(a, b) for a in PRECS for b in PRECS])
@pytest.mark.parametrize("dim,n", [(3, 15), (3, 47), (2, 63), (2, 95), (3, 9), (3, 21), (2, 9)])
def test_q1_prolong_sweep(dev, ref, pf, pc, dim, n):
    print(f"q1 prolong {pc}->{pf} dim={dim} n={n}", flush=True)
    s = _solver(dim, n, pf, pc)
    nc = (n - 1) // 2
    rng = np.random.default_rng(40 * n + dim)
    gf, gc = _g(dim, n), _g(dim, nc) / 2**dim
    bq = _put(s, 0, mgir.BUF_RHS, rng.uniform(-1, 1, (n,) * dim), dev)
    cq = _put(s, 0, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (n,) * dim), dev)
    ecq = _put(s, 1, mgir.BUF_COR, 0.3 * rng.uniform(-1, 1, (nc,) * dim), dev)
    s.stage(mgir.STAGE_PROLONG_SWEEP, 0)
    out = _get(s, 0, mgir.BUF_COR)
    corrected = round_to((cq / gf + ref.prolong(ecq / gc)) * gf, pf)
    expect = ref.jacobi(bq, corrected / gf, 0.8, "q1") * gf
    assert rel_err(out, expect) <= TOL[pf]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim", [2, 3])
def test_q1_coarse_solve(dev, prec, dim):
    s = _solver(dim, 7, "f64", prec)
    base = s.nlevels - 1
    bq = _put(s, base, mgir.BUF_RHS, np.full((1,) * dim, 0.7071), dev)
    s.stage(mgir.STAGE_COARSE, base)
    out = _get(s, base, mgir.BUF_COR)
    # S = 8/3 on one point
    assert rel_err(out, round_to(bq * 0.375, prec)) <= TOL[prec]


@pytest.mark.parametrize("dim,n", [(3, 7), (3, 31), (3, 63), (3, 47), (2, 63), (2, 255), (2, 191)])
def test_q1_vcycle_fp64(dev, ref, dim, n):
    print(f"q1 vcycle f64 dim={dim} n={n}", flush=True)
    s = _solver(dim, n, "f64", base_tol=1e-14, base_max_iter=5000)
    b = W.uniform_rhs(dim, n, seed=50 + n) / (n + 1) ** dim
    c = s.vcycle(torch.from_numpy(b).to(dev)).cpu().numpy()
    base = s.level_n(s.nlevels - 1)
    e = ref.vcycle(b, disc="q1", base_n=base, base_tol=1e-14, base_max_iter=5000)
    assert rel_err(c / _g(dim, n), e) <= 1e-11


@pytest.mark.parametrize("name,tol", [("f32", 1e-5), ("f16", 2e-2), ("bf16", 1e-1), ("hsd", 2e-2)])
@pytest.mark.parametrize("dim,n", [(3, 63), (2, 255)])
def test_q1_vcycle_mixed(dev, ref, name, tol, dim, n):
    print(f"q1 vcycle {name} dim={dim} n={n}", flush=True)
    m = mgir.full_levels(n)
    s = mgir.Solver(dim, n, W.precision_map(name, m), disc="q1")
    prec = W.precision_map(name, m)
    bq = round_to(W.uniform_rhs(dim, n, seed=60 + n), prec[0])
    bt = torch.from_numpy(bq).to(dev).to(mgir.TORCH_DTYPE[prec[0]])
    c = s.vcycle(bt).to(torch.float64).cpu().numpy()
    e = ref.vcycle(bq, disc="q1")
    assert rel_err(c / _g(dim, n), e) <= tol


@pytest.mark.parametrize("dim,n", [(3, 63), (2, 255), (3, 95), (2, 383)])
def test_q1_ir_fp64_matches_oracle(dev, ref, dim, n):
    print(f"q1 ir f64 dim={dim} n={n}", flush=True)
    m = mgir.full_levels(n)
    base = ref.hierarchy(n)[-1]
    b = W.uniform_rhs(dim, n, seed=70 + n) / (n + 1) ** dim
    s = mgir.Solver(dim, n, ["f64"] * m, disc="q1", residual_scaling=False, base_tol=1e-12, base_max_iter=5000)
    u, res = s.solve(torch.from_numpy(b).to(dev))
    u = u.cpu().numpy()
    o = ref.ir_solve(b, disc="q1", residual_scaling=False, recursive_residual=True, base_n=base, base_tol=1e-12,
                     base_max_iter=5000)
    assert res.status == 0 and o.status == 0
    assert abs(res.iterations - o.iterations) <= 1
    assert _true_rel(ref, b, u) <= 1e-10
    assert rel_err(u, o.u) <= 1e-8


@pytest.mark.parametrize("name", ["f32", "f16", "bf16", "h_mg", "hsd"])
@pytest.mark.parametrize("dim,n", [(3, 63), (2, 255), (3, 95)])
def test_q1_ir_mixed_reaches_tolerance(dev, ref, name, dim, n):
    print(f"q1 ir {name} dim={dim} n={n}", flush=True)
    m = mgir.full_levels(n)
    b = W.uniform_rhs(dim, n, seed=80 + n) / (n + 1) ** dim
    bt = torch.from_numpy(b).to(dev)
    _, r64 = mgir.Solver(dim, n, ["f64"] * m, disc="q1", residual_scaling=False).solve(bt)
    s = mgir.Solver(dim, n, W.precision_map(name, m), disc="q1")
    u, res = s.solve(bt)
    assert res.status == 0
    assert _true_rel(ref, b, u.cpu().numpy()) <= 1e-10
    assert res.iterations <= r64.iterations + 2


def test_q1_options_compose(dev, ref):
    """Q1 with rescaled restrictions into half-precision levels, two V-cycles per
    step and a partial hierarchy on a paper grid: still to the tolerance."""
    dim, n, nl = 3, 95, 4  # base 11^3 by CG
    print(f"q1 composed dim={dim} n={n} nl={nl}", flush=True)
    b = W.uniform_rhs(dim, n, seed=90) / (n + 1) ** dim
    s = mgir.Solver(dim, n, W.precision_map("dsh", nl), disc="q1", nlevels=nl, rescale_half=True,
                    cycles_per_step=2)
    u, res = s.solve(torch.from_numpy(b).to(dev))
    assert res.status == 0
    assert _true_rel(ref, b, u.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("dim,n", [(3, 191), (3, 287), (2, 6143)])
def test_q1_paper_grids_full_size(dev, ref, dim, n):
    """The paper's smallest and largest meshes (193^3 and 289^3 vertices, and
    6145^2), FP16 cycle, base level c - 1 solved by CG: the FP64 residual
    recomputed by the oracle meets the tolerance, in no more steps than the
    FP64 cycle needs plus two."""
    print(f"q1 paper grid dim={dim} n={n}", flush=True)
    m = mgir.full_levels(n)
    b = W.uniform_rhs(dim, n, seed=100 + n) / (n + 1) ** dim
    bt = torch.from_numpy(b).to(dev)
    _, r64 = mgir.Solver(dim, n, ["f64"] * m, disc="q1", residual_scaling=False).solve(bt)
    s = mgir.Solver(dim, n, W.precision_map("f16", m), disc="q1")
    u, res = s.solve(bt)
    assert res.status == 0 and r64.status == 0
    assert _true_rel(ref, b, u.cpu().numpy()) <= 1e-10
    assert res.iterations <= r64.iterations + 2


@pytest.mark.parametrize("dim,n,nl", [(3, 95, 0), (2, 383, 5)])
def test_q1_initial_guess_and_partial_hierarchy(dev, ref, dim, n, nl):
    """Q1 from the paper's random initial guess in [0, 1] (Section 6), on a full
    hierarchy and on a 2-D partial one (base 23^2 by CG), without graphs in the
    second case: the FP64 residual meets the tolerance, within two steps of the
    FP64 cycle."""
    print(f"q1 u0 dim={dim} n={n} nl={nl}", flush=True)
    m = nl or mgir.full_levels(n)
    b = W.q1_load_vector(dim, n, seed=110)
    u0 = W.random_initial_guess(dim, n, seed=111)
    bt = torch.from_numpy(b).to(dev)
    kw = dict(disc="q1", nlevels=nl, use_initial_guess=True, use_graph=nl == 0)
    u64 = torch.from_numpy(u0).to(dev)
    _, r64 = mgir.Solver(dim, n, ["f64"] * m, residual_scaling=False, **kw).solve(bt, u64)
    u = torch.from_numpy(u0).to(dev)
    s = mgir.Solver(dim, n, W.precision_map("f16", m), **kw)
    u, res = s.solve(bt, u)
    assert res.status == 0 and r64.status == 0
    assert _true_rel(ref, b, u.cpu().numpy()) <= 1e-10
    assert res.iterations <= r64.iterations + 2


@pytest.mark.parametrize("name,dim,n", [("f16", 3, 95), ("f16", 3, 21), ("f16", 2, 255), ("f64", 3, 63)])
def test_q1_deferred_update_bitwise(dev, name, dim, n):
    """Postponed solution updates on the Q1 path (the marching update at n = 95
    and 63, the one-point update at n = 21 and in 2-D): the stored corrections,
    added to u in step order when the ring is full and before u is read, give u
    bit for bit and the same residual history as the update in every step."""
    print(f"q1 defer {name} dim={dim} n={n}", flush=True)
    m = mgir.full_levels(n)
    b = torch.from_numpy(W.q1_load_vector(dim, n, seed=120)).to(dev)
    kw = dict(disc="q1", residual_scaling=name != "f64")
    u0, r0 = mgir.Solver(dim, n, W.precision_map(name, m), **kw).solve(b)
    for k in (3, 64):
        u1, r1 = mgir.Solver(dim, n, W.precision_map(name, m), defer_update=k, **kw).solve(b)
        assert r1.status == 0 and r1.iterations == r0.iterations, k
        assert r1.history == r0.history, k
        assert torch.equal(u1, u0), k


Q1_KINDS = (mgir.SHAPE_SWEEP, mgir.SHAPE_RESTRICT, mgir.SHAPE_UPDATE)


def _q1_lds_levels(s):
    return [l for l in range(s.nlevels - 1) if s.get_shape(l, mgir.SHAPE_SWEEP) != [0, 0]]


@pytest.mark.parametrize("name,n,defer", [("f16", 63, 4), ("bf16", 95, 0), ("f16", 127, 0), ("hsd", 63, 0)])
def test_q1_lds_shapes_bitwise(dev, name, n, defer):
    """The LDS-staged Q1 sweep, residual and update in other launch shapes
    (rows and planes per block, ragged last tiles and chunks) give u bit for bit
    and the same iteration count as the built-in shapes; the norms are summed
    over other blocks, so the history may differ in the last bits."""
    print(f"q1 shapes {name} n={n} defer={defer}", flush=True)
    prec = W.precision_map(name, mgir.full_levels(n))
    b = torch.from_numpy(W.q1_load_vector(3, n, seed=121)).to(dev)
    s = mgir.Solver(3, n, prec, disc="q1", defer_update=defer, residual_scaling=True)
    levels = _q1_lds_levels(s)
    assert levels and levels[0] == 0
    for l in levels:
        for k in Q1_KINDS[: 3 if l == 0 else 2]:
            ty, zc = s.get_shape(l, k)
            assert ty >= 1 and zc >= 1
    u0, r0 = s.solve(b)
    u0 = u0.clone()
    tried = 0
    for ty, zc, split in ((1, 2, 1), (3, 5, 1), (5, 16, 1), (2, 32, 0), (4, 7, 1), (6, 1, 1), (2, 2, 0), (4, 8, 0),
                          (6, 16, 0)):
        set_any = False
        for l in levels:
            for k in Q1_KINDS[: 3 if l == 0 else 2]:
                shape = [ty, zc, split] if k == mgir.SHAPE_RESTRICT else [ty, zc]
                try:
                    s.set_shape(l, k, shape)
                    set_any = True
                    assert s.get_shape(l, k, len(shape)) == shape
                except mgir.MgError:
                    s.set_shape(l, k, [0, 0])
        if not set_any:
            continue
        tried += 1
        print(f"  shape ty={ty} zc={zc}", flush=True)
        u, r = s.solve(b)
        assert r.status == 0 and r.iterations == r0.iterations, (ty, zc)
        assert np.allclose(r.history, r0.history, rtol=1e-12, atol=0), (ty, zc)
        assert torch.equal(u, u0), (ty, zc)
    assert tried >= 4


def test_q1_shapes_refused(dev):
    """Q1 shapes exist only for the LDS-staged kernels: other kinds, levels
    without such kernels, the update below level 0 and shapes that do not fit
    are refused; {0, 0} restores the built-in shape."""
    n = 63
    m = mgir.full_levels(n)
    s = mgir.Solver(3, n, W.precision_map("hsd", m), disc="q1")
    builtin = s.get_shape(0, mgir.SHAPE_SWEEP)
    for kind in (mgir.SHAPE_FUSE, mgir.SHAPE_SMOOTH, mgir.SHAPE_PROLONG, mgir.SHAPE_TAIL):
        with pytest.raises(mgir.MgError):
            s.set_shape(0, kind, [1])
    with pytest.raises(mgir.MgError):
        s.set_shape(1, mgir.SHAPE_UPDATE, [2, 4])
    for bad in ([300, 2], [2, 0], [0, 4], [-1, 2], [2, n + 1]):
        with pytest.raises(mgir.MgError):
            s.set_shape(0, mgir.SHAPE_SWEEP, bad)
    with pytest.raises(mgir.MgError):
        s.set_shape(0, mgir.SHAPE_SWEEP, [2, 4, 1])
    s.set_shape(0, mgir.SHAPE_SWEEP, [2, 4])
    assert s.get_shape(0, mgir.SHAPE_SWEEP) == [2, 4]
    s.set_shape(0, mgir.SHAPE_SWEEP, [0, 0])
    assert s.get_shape(0, mgir.SHAPE_SWEEP) == builtin
    f64 = mgir.Solver(3, n, W.precision_map("f64", m), disc="q1", residual_scaling=False)
    assert f64.get_shape(0, mgir.SHAPE_SWEEP) == [0, 0]
    with pytest.raises(mgir.MgError):
        f64.set_shape(0, mgir.SHAPE_SWEEP, [2, 4])
    f64.set_shape(0, mgir.SHAPE_SWEEP, [0, 0])
    s2 = mgir.Solver(2, 255, W.precision_map("f16", mgir.full_levels(255)), disc="q1")
    assert s2.get_shape(0, mgir.SHAPE_SWEEP) == [0, 0]
    with pytest.raises(mgir.MgError):
        s2.set_shape(0, mgir.SHAPE_SWEEP, [2, 4])


def test_q1_autotuned_bitwise_and_cached(dev, tmp_path, monkeypatch):
    """The Q1 autotuner picks shapes that fit, the solve matches the built-in
    shapes bit for bit, and a second handle of the same configuration reads
    the shapes back from the cache instead of timing."""
    n = 95
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MGIR_TUNE_CACHE", str(path))
    prec = W.precision_map("f16", mgir.full_levels(n))
    b = torch.from_numpy(W.q1_load_vector(3, n, seed=122)).to(dev)
    u0, r0 = mgir.Solver(3, n, prec, disc="q1", defer_update=8).solve(b)
    a = mgir.Solver(3, n, prec, disc="q1", defer_update=8, autotune=True)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "|q1\t" in lines[0]
    c = mgir.Solver(3, n, prec, disc="q1", defer_update=8, autotune=True)
    assert path.read_text().splitlines() == lines

    def shapes(s):
        return [s.get_shape(l, k, 3) for l in _q1_lds_levels(s) for k in Q1_KINDS[: 3 if l == 0 else 2]]

    assert shapes(a) == shapes(c) and all(t >= 1 and z >= 1 for t, z, _ in shapes(a))
    for s in (a, c):
        u, r = s.solve(b)
        assert r.iterations == r0.iterations and torch.equal(u, u0)
