"""Dense-matrix statements of the multigrid operators for tiny grids.

Independent of the oracle's stencil loops: every operator is assembled here
from its 1-D definition with Kronecker products, so that the oracle can be
checked against plain linear algebra (numpy) on grids of 3^D and 7^D points.
Flattening is numpy C order of an array indexed [z, y, x] (x fastest).
"""
import numpy as np


def lap1d(n):
    """1-D second-difference matrix tridiag(-1, 2, -1) / h^2 with h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    return (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h**2


def stiff1d(n):
    """1-D linear-element stiffness matrix tridiag(-1, 2, -1) / h."""
    h = 1.0 / (n + 1)
    return (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h


def mass1d(n):
    """1-D linear-element mass matrix h tridiag(1/6, 2/3, 1/6)."""
    h = 1.0 / (n + 1)
    return h * (4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)) / 6


def kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def lap(dim, n):
    """Finite-difference -Laplace with zero Dirichlet boundary: sum over axes."""
    I, T = np.eye(n), lap1d(n)
    return sum(kron_all([T if a == b else I for b in range(dim)]) for a in range(dim))


def q1(dim, n):
    """Bilinear / trilinear finite-element stiffness matrix: the tensor-product
    basis makes it sum over axes a of (stiffness along a) x (mass along the
    others)."""
    I, K, M = np.eye(n), stiff1d(n), mass1d(n)
    return sum(kron_all([K if a == b else M for b in range(dim)]) for a in range(dim))


def operator(dim, n, disc="fd"):
    return q1(dim, n) if disc == "q1" else lap(dim, n)


def restrict1d(nf):
    """Full weighting in 1-D: coarse point I averages fine 2I, 2I+1, 2I+2 (0-based)
    with weights 1/4, 1/2, 1/4."""
    nc = (nf - 1) // 2
    R = np.zeros((nc, nf))
    for I in range(nc):
        R[I, 2 * I:2 * I + 3] = [0.25, 0.5, 0.25]
    return R


def restrict(dim, nf):
    return kron_all([restrict1d(nf)] * dim)


def prolong1d(nc):
    """Linear interpolation in 1-D, written from its definition: fine point
    2I+1 copies coarse I; fine point 2I averages coarse I-1 and I (zero outside)."""
    nf = 2 * nc + 1
    P = np.zeros((nf, nc))
    for I in range(nc):
        P[2 * I + 1, I] = 1.0
        P[2 * I, I] += 0.5
        P[2 * I + 2, I] += 0.5
    return P


def prolong(dim, nc):
    return kron_all([prolong1d(nc)] * dim)


def jacobi_iteration_matrix(dim, n, omega, disc="fd"):
    """Error propagation of one damped-Jacobi sweep: S = I - omega D^-1 A."""
    A = operator(dim, n, disc)
    return np.eye(A.shape[0]) - omega * A / np.diag(A)[:, None]


def vcycle_matrix(dim, n, nu1=2, nu2=2, omega=0.8, base_n=1, disc="fd"):
    """Dense V-cycle operator M with c = M b, from the two-grid error propagation
    E = S^nu2 (I - P M_c R A) S^nu1 and M = (I - E) A^-1, recursively down to
    the exact solve on the base level of base_n points per dimension.  The
    restriction R is full weighting (fd) or P^T (q1)."""
    A = operator(dim, n, disc)
    if n == base_n:
        return np.linalg.inv(A)
    nc = (n - 1) // 2
    Mc = vcycle_matrix(dim, nc, nu1, nu2, omega, base_n, disc)
    S = jacobi_iteration_matrix(dim, n, omega, disc)
    P = prolong(dim, nc)
    R = P.T if disc == "q1" else restrict(dim, n)
    I = np.eye(A.shape[0])
    E = np.linalg.matrix_power(S, nu2) @ (I - P @ Mc @ R @ A) @ np.linalg.matrix_power(S, nu1)
    return (I - E) @ np.linalg.inv(A)
