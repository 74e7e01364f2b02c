"""Launch-shape invariance (GPU): every launch shape of every kernel forms the
same roundings, so V-cycles and refinement iterates must agree bitwise across
shapes.  A race in an LDS-staged kernel or a tiling error shows up here."""
import itertools

import numpy as np
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


STENCIL = [[V, zc, bs, xcd, ty] for V, zc, bs, xcd, ty in
           [(8, 1, 256, 0, 0), (4, 3, 64, 1, 0), (8, 7, 128, 1, 0), (8, 64, 256, 1, 0),
            (8, 1, 256, 0, 1), (4, 5, 256, 1, 2), (8, 8, 256, 1, 6), (8, 3, 256, 0, 14), (4, 16, 256, 1, 3)]] + \
    [[8, 2, 256, 1, 2, 2], [4, 7, 256, 0, 5, 2], [8, 16, 256, 1, 14, 2]]
RESTRICT = [[4, 1, 1, 0], [8, 2, 3, 0], [8, 7, 5, 0], [4, 3, 64, 0], [8, 1, 1, 1], [4, 2, 7, 1], [8, 4, 16, 1],
            [8, 6, 3, 1], [8, 1, 2, 2], [4, 3, 5, 2], [8, 5, 9, 2], [8, 6, 1, 2], [8, 2, 7, 3], [4, 1, 3, 3],
            [8, 3, 16, 4], [8, 1, 1, 4]]


def _apply(s, kind, shape):
    applied = 0
    for lvl in range(s.nlevels - 1):
        if kind == mgir.SHAPE_UPDATE and lvl != 0:
            continue
        try:
            s.set_shape(lvl, kind, shape)
            applied += 1
        except mgir.MgError:
            pass
    return applied


@pytest.mark.parametrize("name,n", [("f16", 63), ("f64", 63), ("bf16", 31), ("f32", 31), ("hsd", 127)])
def test_shapes_bitwise(dev, name, n):
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=5)).to(dev)
    bl = b64.to(mgir.TORCH_DTYPE[prec[0]])
    s = mgir.Solver(3, n, prec)
    s.set_shape(0, mgir.SHAPE_TAIL, [0])  # every level through its own kernels
    defaults = {k: [s.get_shape(l, k) for l in range(s.nlevels - 1) if k != mgir.SHAPE_UPDATE or l == 0]
                for k in (mgir.SHAPE_STENCIL, mgir.SHAPE_RESTRICT, mgir.SHAPE_UPDATE)}
    c_ref = s.vcycle(bl).clone()
    u_ref, r_ref = s.solve(b64)
    u_ref = u_ref.clone()
    for kind, shapes in ((mgir.SHAPE_STENCIL, STENCIL), (mgir.SHAPE_RESTRICT, RESTRICT),
                         (mgir.SHAPE_UPDATE, STENCIL)):
        for shape in shapes:
            print(f"{name} n={n} kind={kind} shape={shape}", flush=True)
            if not _apply(s, kind, shape):
                continue
            if kind != mgir.SHAPE_UPDATE:
                c = s.vcycle(bl)
                assert torch.equal(c, c_ref), (kind, shape)
            u, r = s.solve(b64)
            assert r.iterations == r_ref.iterations, (kind, shape)
            assert torch.equal(u, u_ref), (kind, shape)
        for lvl, sh in enumerate(defaults[kind]):
            s.set_shape(lvl, kind, sh)


def test_autotuned_solver_matches_default(dev):
    n = 127
    prec = W.precision_map("f16", W.levels_for(n))
    b = torch.from_numpy(W.uniform_rhs(3, n, seed=6)).to(dev)
    u0, r0 = mgir.Solver(3, n, prec).solve(b)
    st = mgir.Solver(3, n, prec, autotune=True)
    u1, r1 = st.solve(b)
    assert r0.iterations == r1.iterations and torch.equal(u0, u1)


@pytest.mark.parametrize("name,scaling,defer", [("f16", True, 0), ("f64", False, 0), ("f16", True, 4)])
def test_tuning_cache_round_trip(dev, tmp_path, monkeypatch, name, scaling, defer):
    """With MGIR_TUNE_CACHE set, the first autotuned handle records its shapes
    and a second one of the same configuration reads them back instead of
    timing: same shapes, same fused forms, bitwise the same solve; a handle
    of another configuration gets a line of its own."""
    n = 63
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MGIR_TUNE_CACHE", str(path))
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=15)).to(dev)
    kinds = (mgir.SHAPE_SMOOTH, mgir.SHAPE_SWEEP, mgir.SHAPE_PROLONG, mgir.SHAPE_RESTRICT, mgir.SHAPE_FUSE,
             mgir.SHAPE_FUSE_SR)

    def shapes(s):
        return [s.get_shape(l, k) for l in range(s.nlevels - 1) for k in kinds if k in kinds[:4] or l == 0] + \
            [s.get_shape(0, mgir.SHAPE_UPDATE), s.get_shape(0, mgir.SHAPE_FUSE, 6)]

    a = mgir.Solver(3, n, prec, residual_scaling=scaling, autotune=True, defer_update=defer)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    b = mgir.Solver(3, n, prec, residual_scaling=scaling, autotune=True, defer_update=defer)
    assert path.read_text().splitlines() == lines  # read back, not tuned again
    assert shapes(a) == shapes(b)
    ua, ra = a.solve(b64)
    ub, rb = b.solve(b64)
    assert ra.iterations == rb.iterations and torch.equal(ua, ub)
    mgir.Solver(3, 31, W.precision_map(name, W.levels_for(31)), residual_scaling=scaling, autotune=True)
    assert len(path.read_text().splitlines()) == 2


@pytest.mark.parametrize("name,n", [("f16", 7), ("f16", 63), ("f64", 31), ("f32", 15), ("bf16", 127), ("hsd", 255),
                                    ("h_mg", 63), ("f64", 127)])
def test_fused_tail_bitwise(dev, name, n):
    """The single-workgroup coarse end computes exactly the per-level kernels."""
    print(f"tail {name} n={n}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=7)).to(dev)
    bl = b64.to(mgir.TORCH_DTYPE[prec[0]])
    s = mgir.Solver(3, n, prec)
    assert s.get_shape(0, mgir.SHAPE_TAIL) == [1]
    c_on = s.vcycle(bl).clone()
    u_on, r_on = s.solve(b64)
    u_on = u_on.clone()
    s.set_shape(0, mgir.SHAPE_TAIL, [0])
    c_off = s.vcycle(bl)
    u_off, r_off = s.solve(b64)
    assert torch.equal(c_on, c_off)
    assert r_on.iterations == r_off.iterations and torch.equal(u_on, u_off)
    assert r_on.history == r_off.history


@pytest.mark.parametrize("name,n,scaling", [("f16", 63, True), ("bf16", 31, True), ("f32", 127, True),
                                            ("hsd", 63, True), ("h_mg", 31, True), ("f64", 31, True),
                                            ("f16", 7, True)])
def test_fused_sweep_update_bitwise(dev, name, n, scaling):
    """The last finest-level sweep fused into the refinement update changes no
    result, for every launch shape of the fused kernel."""
    print(f"fused update {name} n={n}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=8)).to(dev)
    s = mgir.Solver(3, n, prec, residual_scaling=scaling)
    s.set_shape(0, mgir.SHAPE_FUSE, [0])
    assert s.get_shape(0, mgir.SHAPE_FUSE)[0] == 0
    u_ref, r_ref = s.solve(b64)
    u_ref = u_ref.clone()
    # the sixth value: the right-hand side read back (0) or formed from r (1)
    for shape in ([1, 4, 16, 1, 4], [1, 4, 3, 0, 1], [1, 4, 64, 1, 2], [1, 4, 5, 1, 3], [1, 4, 16, 1, 4, 0],
                  [1, 4, 16, 1, 4, 1], [1, 4, 3, 0, 1, 1], [1, 4, 64, 1, 2, 1], [1, 4, 5, 1, 3, 0]):
        try:
            s.set_shape(0, mgir.SHAPE_FUSE, shape)
        except mgir.MgError:
            continue
        assert s.get_shape(0, mgir.SHAPE_FUSE, len(shape)) == shape
        u, r = s.solve(b64)
        # the norms are summed over the kernel's blocks, so the history may
        # differ in the last bits between shapes; the iterates may not
        assert r.iterations == r_ref.iterations, shape
        assert np.allclose(r.history, r_ref.history, rtol=1e-13, atol=0), shape
        assert torch.equal(u, u_ref), shape


@pytest.mark.parametrize("n,graph", [(31, True), (63, True), (127, True), (63, False)])
def test_fp64_baseline_fused_forms_bitwise(dev, n, graph):
    """The FP64 map without residual scaling (the baseline, whose right-hand
    side is the residual itself) runs the fused first smoothing + restriction
    and the fused last sweep + update; the latter writes the new residual to a
    second array every step.  Both change no iterate, for several shapes of
    each kernel, with and without graphs (the graphs of the two array roles)."""
    print(f"FP64 baseline fused forms n={n} graph={graph}", flush=True)
    prec = W.precision_map("f64", W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=11)).to(dev)
    s = mgir.Solver(3, n, prec, residual_scaling=False, use_graph=graph)
    assert s.get_shape(0, mgir.SHAPE_FUSE)[0] == 1
    assert s.get_shape(0, mgir.SHAPE_FUSE_SR)[0] == 1
    u_on, r_on = s.solve(b64)
    u_on = u_on.clone()
    res_on = s.read(0, mgir.BUF_RES)
    s.set_shape(0, mgir.SHAPE_FUSE, [0])
    s.set_shape(0, mgir.SHAPE_FUSE_SR, [0])
    u_off, r_off = s.solve(b64)
    assert r_off.iterations == r_on.iterations
    assert np.allclose(r_off.history, r_on.history, rtol=1e-13, atol=0)
    assert torch.equal(u_off, u_on)
    # the residual left after the solve is b - A u wherever the arrays ended
    assert torch.equal(s.read(0, mgir.BUF_RES), res_on)
    tried = 0
    for fuse, sr in (([1, 4, 8, 1, 1], [1, 1, 3]), ([1, 4, 3, 0, 2], [1, 1, 7]), ([1, 4, 16, 1, 1], [1, 2, 5]),
                     ([1, 4, 64, 1, 2], [1, 1, 16])):
        try:
            s.set_shape(0, mgir.SHAPE_FUSE, fuse)
            s.set_shape(0, mgir.SHAPE_FUSE_SR, sr)
        except mgir.MgError:
            continue
        tried += 1
        print(f"  shapes {fuse} {sr}", flush=True)
        u, r = s.solve(b64)
        assert r.iterations == r_on.iterations, (fuse, sr)
        assert np.allclose(r.history, r_on.history, rtol=1e-13, atol=0), (fuse, sr)
        assert torch.equal(u, u_on), (fuse, sr)
    assert tried >= 2
    with pytest.raises(mgir.MgError):  # r is the right-hand side: there is no stored b to read
        s.set_shape(0, mgir.SHAPE_FUSE, [1, 4, 8, 1, 1, 0])


@pytest.mark.parametrize("name,n,depth,cycles,from_r", [("f16", 63, 1, 1, None), ("f16", 63, 3, 1, None),
                                                        ("f16", 127, 64, 1, None), ("bf16", 31, 2, 1, None),
                                                        ("f32", 63, 5, 1, None), ("hsd", 127, 3, 1, None),
                                                        ("f64", 63, 4, 1, None), ("f16", 63, 4, 2, None),
                                                        ("f64", 31, 2, 2, None), ("f16", 63, 3, 1, 1),
                                                        ("bf16", 127, 5, 1, 1), ("f32", 31, 2, 2, 0),
                                                        ("f16", 63, 4, 2, 1)])
def test_deferred_update_bitwise(dev, name, n, depth, cycles, from_r):
    """Postponing the solution update (a ring of `depth` stored corrections,
    added to u in step order when full and before u is read) gives the same u
    bit for bit, the same iteration count and the same residual history: from
    zero, from a random guess, when the step limit ends the solve, and on a
    second solve with the same handle."""
    print(f"deferred update {name} n={n} depth={depth} cycles={cycles}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    scaling = name != "f64"
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=12)).to(dev)
    u0 = torch.from_numpy(W.random_initial_guess(3, n, seed=13)).to(dev)
    kw = dict(residual_scaling=scaling, cycles_per_step=cycles)
    for guess, max_iter in ((False, 100), (True, 100), (False, 3)):
        ref = mgir.Solver(3, n, prec, use_initial_guess=guess, max_iter=max_iter, **kw)
        dfr = mgir.Solver(3, n, prec, use_initial_guess=guess, max_iter=max_iter, defer_update=depth, **kw)
        assert dfr.get_shape(0, mgir.SHAPE_FUSE)[0] == 1
        if from_r is not None:  # both take the given way to the right-hand side
            for x in (ref, dfr):
                x.set_shape(0, mgir.SHAPE_FUSE, x.get_shape(0, mgir.SHAPE_FUSE) + [from_r])
                assert x.get_shape(0, mgir.SHAPE_FUSE, 6)[5] == from_r
        for rep in range(2):
            ua, ra = ref.solve(b64, u0.clone() if guess else None, check=False)
            ub, rb = dfr.solve(b64, u0.clone() if guess else None, check=False)
            assert ra.status == rb.status and ra.iterations == rb.iterations, (guess, max_iter, rep)
            assert ra.history == rb.history, (guess, max_iter, rep)
            assert torch.equal(ua, ub), (guess, max_iter, rep)
            assert torch.equal(ref.read(0, mgir.BUF_SOL), dfr.read(0, mgir.BUF_SOL))


def test_deferred_update_profile_step(dev):
    """The profiled step of a handle with postponed updates leaves u updated
    (its flush timed as a launch of its own)."""
    n = 63
    prec = W.precision_map("f16", W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=14)).to(dev)
    ref = mgir.Solver(3, n, prec, max_iter=2)
    dfr = mgir.Solver(3, n, prec, max_iter=2, defer_update=8)
    ref.solve(b64, check=False)
    dfr.solve(b64, check=False)
    pa, pb = ref.profile_step(), dfr.profile_step()
    names = [p[0] for p in pb]
    assert "sweep_update_defer" in names and "defer_flush" in names
    assert torch.equal(ref.read(0, mgir.BUF_SOL), dfr.read(0, mgir.BUF_SOL))
    assert torch.equal(ref.read(0, mgir.BUF_RES), dfr.read(0, mgir.BUF_RES))


@pytest.mark.parametrize("disc,dim,n", [("fd", 3, 31), ("q1", 3, 21), ("q1", 2, 63)])
def test_deferred_update_zero_rhs_clears_u(dev, disc, dim, n):
    """A solve from zero with postponed updates neither fills nor reads u
    before its first flush; with b = 0 it returns at once, and the handle's
    own u is zero too, not the previous solve's."""
    prec = W.precision_map("f16", mgir.full_levels(n))
    s = mgir.Solver(dim, n, prec, disc=disc, defer_update=4)
    b64 = torch.from_numpy(W.q1_load_vector(dim, n, seed=16) if disc == "q1" else W.uniform_rhs(dim, n, seed=16))
    b64 = b64.to(dev)
    s.solve(b64)
    assert s.read(0, mgir.BUF_SOL).abs().max().item() > 0
    u, r = s.solve(torch.zeros_like(b64))
    assert r.status == 0 and r.iterations == 0
    assert not u.any() and not s.read(0, mgir.BUF_SOL).any()
    u2, r2 = s.solve(b64)  # and the next solve from zero again
    ref = mgir.Solver(dim, n, prec, disc=disc)
    u3, r3 = ref.solve(b64)
    assert r2.iterations == r3.iterations and torch.equal(u2, u3)


@pytest.mark.parametrize("name,n", [("f16", 63), ("bf16", 31), ("f32", 127), ("f16", 15), ("h_mg", 31),
                                    ("hsd", 255), ("f64", 63), ("f64", 255)])
def test_fused_smooth_restrict_bitwise(dev, name, n):
    """The first finest-level smoothing fused with the residual + restriction
    of its result changes no result, for every launch shape of the fused
    kernel (several y tiles and plane chunks, ragged last ones)."""
    print(f"fused smooth+restrict {name} n={n}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=9)).to(dev)
    s = mgir.Solver(3, n, prec)
    assert s.get_shape(0, mgir.SHAPE_FUSE_SR)[0] == 1
    s.set_shape(0, mgir.SHAPE_FUSE_SR, [0])
    assert s.get_shape(0, mgir.SHAPE_FUSE_SR)[0] == 0
    u_ref, r_ref = s.solve(b64)
    u_ref = u_ref.clone()
    tried = narrow_tried = 0
    # three values: c1, c2 in FP32 (FP64) LDS; a fourth 1: in the level's 2-byte format
    for shape in ([1, 1, 1], [1, 2, 3], [1, 3, 16], [1, 1, 5], [1, 3, 7], [1, 2, 32], [1, 1, 1, 1], [1, 3, 16, 1],
                  [1, 2, 32, 1], [1, 3, 7, 1]):
        try:
            s.set_shape(0, mgir.SHAPE_FUSE_SR, shape)
        except mgir.MgError:
            continue
        tried += 1
        narrow_tried += len(shape) == 4
        assert s.get_shape(0, mgir.SHAPE_FUSE_SR, len(shape)) == shape
        print(f"  shape {shape}", flush=True)
        u, r = s.solve(b64)
        assert r.iterations == r_ref.iterations, shape
        assert r.history == r_ref.history, shape
        assert torch.equal(u, u_ref), shape
    assert tried >= (2 if prec[0] == "f64" else 3)
    if prec[0] in ("f16", "bf16") and n >= 15:
        assert narrow_tried >= 1


@pytest.mark.parametrize("name,n", [("f16", 127), ("bf16", 63), ("f32", 63), ("hsd", 255), ("h_mg", 127)])
def test_fused_smooth_restrict_coarse_levels_bitwise(dev, name, n):
    """On the coarser levels the fused first smoothing + restriction reads the
    stored right-hand side; turning it off level by level, or changing its
    shape, changes neither the V-cycle nor the solve."""
    print(f"fused smooth+restrict, coarse levels, {name} n={n}", flush=True)
    prec = W.precision_map(name, W.levels_for(n))
    b64 = torch.from_numpy(W.uniform_rhs(3, n, seed=10)).to(dev)
    bl = b64.to(mgir.TORCH_DTYPE[prec[0]])
    s = mgir.Solver(3, n, prec)
    s.set_shape(0, mgir.SHAPE_TAIL, [0])  # every level through its own kernels
    levels = []
    for l in range(1, s.nlevels - 1):
        assert s.get_shape(l, mgir.SHAPE_FUSE_SR)[0] == 0  # off by default on coarser levels
        try:
            s.set_shape(l, mgir.SHAPE_FUSE_SR, [1])
        except mgir.MgError:
            continue
        if s.get_shape(l, mgir.SHAPE_FUSE_SR)[0] == 1:
            levels.append(l)
    assert levels
    c_on = s.vcycle(bl).clone()
    u_on, r_on = s.solve(b64)
    u_on = u_on.clone()
    for shape in ([1, 1, 3], [1, 2, 5], [1, 3, 2], [1, 2, 5, 1], [1, 1, 3, 1]):
        for l in levels:
            try:
                s.set_shape(l, mgir.SHAPE_FUSE_SR, shape)
            except mgir.MgError:
                pass
        assert torch.equal(s.vcycle(bl), c_on), shape
    for l in levels:
        s.set_shape(l, mgir.SHAPE_FUSE_SR, [0])
        assert s.get_shape(l, mgir.SHAPE_FUSE_SR)[0] == 0
    assert torch.equal(s.vcycle(bl), c_on)
    u_off, r_off = s.solve(b64)
    assert r_off.iterations == r_on.iterations and torch.equal(u_off, u_on)
    assert r_off.history == r_on.history
