"""Seeded synthetic workloads for the Poisson problems the solver is run on.

This module only generates inputs (grid coordinates, right-hand sides,
instance lists and per-level precision maps).  It holds none of the solver's
arithmetic, and it is the one module shared by the GPU tests and the oracle
tests.  Every random number comes from ``numpy.random.default_rng(seed)``
(PCG64) in the order documented per function.

Right-hand sides are float64 numpy arrays indexed ``[y, x]`` (2-D) or
``[z, y, x]`` (3-D), x fastest, holding f at the interior grid points
x_i = (i+1) h, h = 1/(n+1), of the unit square / cube (the model problem of
Section 5 with homogeneous Dirichlet boundary values).
"""
from __future__ import annotations

import numpy as np

# Storage formats a level of the V-cycle can use.
F64, F32, F16, BF16 = "f64", "f32", "f16", "bf16"


def coords(n: int) -> np.ndarray:
    """Interior node coordinates (i+1)/(n+1), i = 0..n-1."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def levels_for(n: int) -> int:
    """Levels of the full hierarchy n, (n-1)/2, ..., 1 (n = 2^m - 1)."""
    if n < 1 or (n + 1) & n:
        raise ValueError(f"n = {n} is not of the form 2^m - 1")
    return int(n + 1).bit_length() - 1


def sine_mode(dim: int, n: int, k=(1, 1, 1)) -> np.ndarray:
    """prod_d sin(k_d pi x_d) sampled at the interior nodes."""
    x = coords(n)
    s = [np.sin(kd * np.pi * x) for kd in k[:dim]]
    if dim == 2:
        return s[1][:, None] * s[0][None, :]
    return s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]


def poisson2d_sine_rhs(n: int = 255) -> np.ndarray:
    """2-D, f = 2 pi^2 sin(pi x) sin(pi y): exact solution u = sin(pi x) sin(pi y)
    (the paper's test function with k = 1, Section 5)."""
    return 2.0 * np.pi**2 * sine_mode(2, n, (1, 1))


def uniform_rhs(dim: int, n: int, seed: int) -> np.ndarray:
    """f i.i.d. uniform[-1, 1]: one rng.uniform(-1, 1, n^dim) draw, x fastest."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, n**dim).reshape((n,) * dim)


def poisson3d_sine_noise_rhs(n: int = 511, seed: int = 3, noise: float = 1e-3) -> np.ndarray:
    """3-D, f = 14 pi^2 sin(pi x) sin(2 pi y) sin(3 pi z) + noise * uniform[-1, 1].
    Without noise the continuous solution is the sine product itself."""
    f = sine_mode(3, n, (1, 2, 3))
    f *= 14.0 * np.pi**2
    if noise:
        rng = np.random.default_rng(seed)
        f += noise * rng.uniform(-1.0, 1.0, n**3).reshape((n,) * 3)
    return f


def manufactured_rhs(dim: int, n: int, k: int) -> np.ndarray:
    """f = dim (k pi)^2 prod_d sin(k pi x_d): the right-hand side whose
    continuous solution is the paper's test function prod_d sin(k pi x_d)
    (Section 5; the measurements use k = 1, 20 and 400)."""
    return dim * (k * np.pi) ** 2 * sine_mode(dim, n, (k, k, k))


def q1_load_vector(dim: int, n: int, seed: int) -> np.ndarray:
    """Right-hand side of the Q1 finite-element system (Section 5): the lumped
    load vector h^dim f_i of f i.i.d. uniform[-1, 1] (one rng.uniform(-1, 1,
    n^dim) draw, x fastest)."""
    return uniform_rhs(dim, n, seed) / float(n + 1) ** dim


def paper_grid_sizes(dim: int) -> list[int]:
    """Interior points per dimension of the paper's meshes (Section 6): the
    smallest and largest of its ranges, 193^3 .. 289^3 and 4097^2 .. 6145^2
    vertices including the boundary."""
    return [191, 287] if dim == 3 else [4095, 6143]


def random_initial_guess(dim: int, n: int, seed: int) -> np.ndarray:
    """u0 i.i.d. uniform[0, 1], the initial guess of the paper's measurements
    (Section 6): one rng.uniform(0, 1, n^dim) draw, x fastest."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, n**dim).reshape((n,) * dim)


def batched_instances(count: int = 64, sizes=(63, 127, 255), seed: int = 4):
    """Independent 3-D instances: first ``rng.choice(sizes, count)`` draws the
    sizes, then one ``rng.uniform(-1, 1, n_i^3)`` per instance in order."""
    rng = np.random.default_rng(seed)
    ns = [int(v) for v in rng.choice(np.asarray(sizes), count)]
    rhs = [rng.uniform(-1.0, 1.0, n**3).reshape((n,) * 3) for n in ns]
    return ns, rhs


def multi_rhs(n: int = 127, nrhs: int = 32, seed: int = 5, emax: float = 6.0) -> np.ndarray:
    """Many right-hand sides sharing one operator: first e = rng.uniform(-emax,
    emax, nrhs), then for k in order 10**e[k] * rng.uniform(-1, 1, n^3).
    Returned interleaved, shape (n, n, n, nrhs): index [z, y, x, k]."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(-emax, emax, nrhs)
    out = np.empty((n, n, n, nrhs))
    for k in range(nrhs):
        out[..., k] = (10.0 ** e[k]) * rng.uniform(-1.0, 1.0, n**3).reshape((n,) * 3)
    return out


def precision_map(name: str, nlevels: int) -> list[str]:
    """Per-level storage formats, finest level first.

    f64, f32, f16, bf16: that format on every level except the one-point base
    level, which is solved in FP64.  h_mg: FP16 on every level including the
    base (the paper's all-half variant, Table 2).  hsd: FP16 on the finest two
    levels, FP32 on the next three, FP64 below (fine-to-coarse FP16 -> FP32 ->
    FP64, Table 2).  dsh: FP64 down to the third-coarsest level, FP32 on that
    one and FP16 on the last two (fine-to-coarse FP64 -> FP32 -> FP16, Table 2,
    with the level split the paper's Section 6 gives); run it with
    rescale_half.
    """
    if name in (F64, F32, F16, BF16):
        return [name] * (nlevels - 1) + [F64]
    if name == "h_mg":
        return [F16] * nlevels
    if name == "dsh":
        # FP64 fine levels, one FP32 level, FP16 on the last two (the paper's
        # DSH_MG: FP16 base and level 1, FP32 level 2, FP64 above)
        out = [F64] * nlevels
        for i, p in zip(range(nlevels - 1, max(nlevels - 4, -1), -1), (F16, F16, F32)):
            out[i] = p
        return out
    if name == "hsd":
        out = []
        for i in range(nlevels):
            out.append(F16 if i < 2 else F32 if i < 5 else F64)
        out[-1] = F64
        return out
    raise ValueError(f"unknown precision map {name!r}")


# The five workloads, by what they are.
WORKLOADS = {
    "poisson2d_255_sine_f64": dict(dim=2, n=255, maps=["f64"]),
    "poisson3d_255_uniform": dict(dim=3, n=255, maps=["f64", "f16"]),
    "poisson3d_511_sine_noise": dict(dim=3, n=511, maps=["f64", "f32", "f16", "bf16", "hsd"]),
    "batched64_3d_mixed_sizes": dict(dim=3, sizes=(63, 127, 255), count=64, maps=["f16"]),
    "poisson3d_127_32rhs": dict(dim=3, n=127, nrhs=32, maps=["f16"]),
}
