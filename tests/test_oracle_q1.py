"""Pins of the oracle's Q1 finite-element discretisation (Section 5: bilinear
elements on the unit square, trilinear on the unit cube) and of the paper's
grid family n = c 2^k - 1 (Section 6), against definitions that do not go
through the oracle's code: quadrature assembly, Kronecker products of the
1-D Galerkin matrices, exactness on quadratics, the Galerkin relation and
dense solves."""
import itertools

import numpy as np
import pytest

from tests import dense_ref


def quadrature_stiffness(dim, n):
    """Stiffness matrix of the Q1 elements assembled cell by cell with the
    2-point Gauss rule per axis (exact for the bilinear / trilinear gradient
    products), written from the basis functions themselves."""
    h = 1.0 / (n + 1)
    g = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    verts = list(itertools.product((0, 1), repeat=dim))  # (offset along axis 0, 1, ...)

    def grad(a, xi):
        out = np.empty(dim)
        for d in range(dim):
            t = 1.0 if a[d] else -1.0
            for e in range(dim):
                if e != d:
                    t *= xi[e] if a[e] else 1.0 - xi[e]
            out[d] = t / h
        return out

    Ke = np.zeros((len(verts), len(verts)))
    for xi in itertools.product(g, repeat=dim):
        G = [grad(a, xi) for a in verts]
        for i, j in itertools.product(range(len(verts)), repeat=2):
            Ke[i, j] += (0.5**dim) * G[i] @ G[j] * h**dim
    N = n**dim
    K = np.zeros((N, N))

    def flat(idx):  # idx along axes (x, y, z) -> C order [z, y, x]
        f = 0
        for d in reversed(range(dim)):
            f = f * n + idx[d]
        return f

    for cell in itertools.product(range(n + 1), repeat=dim):
        nodes = [tuple(cell[d] - 1 + a[d] for d in range(dim)) for a in verts]
        for i, ni in enumerate(nodes):
            if min(ni) < 0 or max(ni) >= n:
                continue
            for j, nj in enumerate(nodes):
                if min(nj) < 0 or max(nj) >= n:
                    continue
                K[flat(ni), flat(nj)] += Ke[i, j]
    return K


def dense_of(fn, dim, n):
    N = n**dim
    cols = []
    for p in range(N):
        e = np.zeros(N)
        e[p] = 1.0
        cols.append(fn(e.reshape((n,) * dim)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("dim,n", [(2, 3), (2, 6), (3, 3), (3, 4)])
def test_q1_matches_quadrature_assembly(ref, dim, n):
    K = quadrature_stiffness(dim, n)
    v = np.random.default_rng(11).standard_normal((n,) * dim)
    np.testing.assert_allclose(ref.apply_A(v, "q1").ravel(), K @ v.ravel(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 5)])
def test_q1_matches_kronecker_definition(ref, dim, n):
    v = np.random.default_rng(12).standard_normal((n,) * dim)
    np.testing.assert_allclose(ref.apply_A(v, "q1").ravel(), dense_ref.q1(dim, n) @ v.ravel(), rtol=1e-12,
                               atol=1e-12)


def test_q1_textbook_stencils(ref):
    # bilinear: (1/3) [-1 -1 -1; -1 8 -1; -1 -1 -1], independent of h
    e = np.zeros((5, 5))
    e[2, 2] = 1.0
    np.testing.assert_allclose(ref.apply_A(e, "q1")[1:4, 1:4],
                               np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3.0, rtol=1e-14)
    # trilinear: h/12 [32 centre, 0 faces, -2 edges, -1 corners]
    n = 5
    h = 1.0 / (n + 1)
    e = np.zeros((n,) * 3)
    e[2, 2, 2] = 1.0
    got = ref.apply_A(e, "q1")[1:4, 1:4, 1:4] * 12.0 / h
    for o in itertools.product((-1, 0, 1), repeat=3):
        k = sum(abs(t) for t in o)
        want = {0: 32.0, 1: 0.0, 2: -2.0, 3: -1.0}[k]
        assert got[o[0] + 1, o[1] + 1, o[2] + 1] == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_exact_on_quadratics(ref, dim):
    # the Q1 stiffness matrix applied to the nodal values of a quadratic u gives
    # the load vector of -Laplace(u) (a constant) at nodes whose stencil stays
    # inside: integral of phi_i = h^dim
    n = 9
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]  # [z, y, x] order: grids[0] = x
    coef = [1.0, -2.5, 0.75][:dim]
    u = sum(c * g**2 for c, g in zip(coef, grids)) + 0.5 * grids[0] * grids[1] + 3.0 * grids[-1]
    lap_u = 2.0 * sum(coef)
    au = ref.apply_A(u, "q1")
    inner = (slice(1, n - 1),) * dim
    np.testing.assert_allclose(au[inner], -lap_u * h**dim, rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("dim,nc", [(2, 3), (2, 7), (3, 3)])
def test_q1_galerkin_and_transpose(ref, dim, nc):
    nf = 2 * nc + 1
    P = dense_of(ref.prolong, dim, nc)
    Af = dense_of(lambda v: ref.apply_A(v, "q1"), dim, nf)
    Ac = dense_of(lambda v: ref.apply_A(v, "q1"), dim, nc)
    np.testing.assert_allclose(P.T @ Af @ P, Ac, rtol=1e-11, atol=1e-12)
    R = dense_of(lambda v: ref.restrict(v, "q1"), dim, nf)
    np.testing.assert_allclose(R, P.T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 3)])
def test_q1_jacobi_is_diagonal_scaling(ref, dim, n):
    rng = np.random.default_rng(13)
    b, c = rng.standard_normal((2,) + (n,) * dim)
    A = dense_ref.q1(dim, n)
    want = c.ravel() + 0.8 * (b.ravel() - A @ c.ravel()) / np.diag(A)
    np.testing.assert_allclose(ref.jacobi(b, c, 0.8, "q1").ravel(), want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, 15), (3, 7)])
def test_q1_vcycle_matches_dense(ref, dim, n):
    b = np.random.default_rng(14).uniform(-1, 1, (n,) * dim)
    M = dense_ref.vcycle_matrix(dim, n, disc="q1")
    np.testing.assert_allclose(ref.vcycle(b, disc="q1").ravel(), M @ b.ravel(), rtol=1e-10, atol=1e-12)


def test_hierarchy_of_paper_grids(ref):
    # the paper's meshes of 193^3 .. 289^3 and 4097^2 .. 6145^2 vertices
    # (boundary included): n = c 2^k - 1 interior points per dimension
    assert ref.hierarchy(191) == [191, 95, 47, 23, 11, 5, 2]
    assert ref.hierarchy(287) == [287, 143, 71, 35, 17, 8]
    assert ref.hierarchy(6143)[-1] == 2 and len(ref.hierarchy(6143)) == 12
    assert ref.hierarchy(4095) == [4095 >> k for k in range(12)]
    assert ref.hierarchy(191, 3) == [191, 95, 47]
    assert ref.levels(191) == 7 and ref.levels(511) == 9


@pytest.mark.parametrize("disc", ["fd", "q1"])
@pytest.mark.parametrize("dim,n,base", [(2, 23, 2), (2, 23, 5), (3, 11, 2)])
def test_paper_grid_vcycle_matches_dense(ref, disc, dim, n, base):
    # a CG base solve run to exhaustion is the exact base solve
    b = np.random.default_rng(15).uniform(-1, 1, (n,) * dim)
    M = dense_ref.vcycle_matrix(dim, n, base_n=base, disc=disc)
    got = ref.vcycle(b, base_n=base, base_tol=1e-15, base_max_iter=4 * base**dim, disc=disc)
    np.testing.assert_allclose(got.ravel(), M @ b.ravel(), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("dim,n,base", [(2, 31, 1), (3, 15, 1), (2, 47, 2), (3, 11, 2)])
def test_q1_ir_matches_dense_solve(ref, dim, n, base):
    b = np.random.default_rng(16).uniform(-1, 1, (n,) * dim) / (n + 1) ** dim
    K = quadrature_stiffness(dim, n) if n**dim <= 2000 else dense_ref.q1(dim, n)
    res = ref.ir_solve(b, disc="q1", base_n=base, rtol=1e-12, max_iter=60)
    assert res.status == ref.OK
    u = np.linalg.solve(K, b.ravel())
    np.testing.assert_allclose(res.u.ravel(), u, rtol=0, atol=1e-9 * np.abs(u).max())
    # Section 6: the paper's IR with a half-precision cycle needs 14-15 steps
    # to 1e-10; with the FP64 cycle on these grids it is no more
    assert res.iterations <= 16


def test_q1_fd_differ(ref):
    # the two discretisations are different operators (guards against a
    # dispatch that ignores disc)
    v = np.random.default_rng(17).standard_normal((7, 7, 7))
    assert not np.allclose(ref.apply_A(v, "q1"), ref.apply_A(v, "fd"))
