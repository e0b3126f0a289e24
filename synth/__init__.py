"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds random numbers and workload shapes only: point sets, right-hand
sides and Gaussian test matrices drawn with numpy's PCG64, plus the named workload
descriptions. It contains none of the method's arithmetic (no kernel evaluation, no
tree, no factorization), so that the CPU oracle and the GPU path can both consume
the same inputs without sharing any computation.

Seed conventions: points 1000+k, right-hand sides 2000+k, test matrices 3000+k,
where k is the workload number.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "points_uniform",
    "points_grid2d",
    "rhs_normal",
    "test_matrix",
    "Workload",
    "WORKLOADS",
    "batch_gaussian",
    "mlp_init",
    "minibatch_order",
]


def points_uniform(n: int, dim: int, seed: int) -> np.ndarray:
    """n points uniform in the unit hypercube [0,1]^dim, float64, row-major (n, dim)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, dim), dtype=np.float64)


def points_grid2d(n: int) -> np.ndarray:
    """The uniform 2D lattice used for the paper's experiments (Results section):
    sqrt(n) x sqrt(n) points at ((i+1/2)/s, (j+1/2)/s). n must be a perfect square."""
    s = int(round(math.sqrt(n)))
    if s * s != n:
        raise ValueError("grid2d needs a square point count")
    g = (np.arange(s, dtype=np.float64) + 0.5) / s
    xx, yy = np.meshgrid(g, g, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], axis=1)


def rhs_normal(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides ~ N(0,1), shape (n, nrhs), float64, column-major friendly (Fortran order)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


def test_matrix(n: int, s: int, seed: int) -> np.ndarray:
    """Gaussian test matrix Omega ~ N(0,1), shape (n, s), float64, Fortran order.

    The randomized compression draws this matrix once; both the oracle and the GPU
    library receive it as an input instead of drawing their own."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, s)))


@dataclass(frozen=True)
class Workload:
    """A named workload: point set, kernel, tree and compression parameters."""

    name: str
    n: int
    dim: int
    kernel: str  # exponential | matern32 | gaussian | laplace2d | yukawa
    length: float
    nugget: float
    leaf: int
    rank: int  # 0 = adaptive (tol)
    tol: float = 0.0
    nrhs: int = 1
    mode: str = "scaled"  # plain | scaled
    geometry: str = "uniform"  # uniform | grid2d
    oversample: int = 8
    seed_k: int = 0
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        if self.geometry == "grid2d":
            return points_grid2d(self.n)
        return points_uniform(self.n, self.dim, 1000 + self.seed_k)

    def rhs(self) -> np.ndarray:
        return rhs_normal(self.n, self.nrhs, 2000 + self.seed_k)

    def omega(self, s: int) -> np.ndarray:
        return test_matrix(self.n, s, 3000 + self.seed_k)


# Named workloads. Sizes, kernels and parameters are workload descriptions,
# not arithmetic.
WORKLOADS = {
    "exp2d_n2048": Workload("exp2d_n2048", 2048, 2, "exponential", 0.1, 1e-4, 128, 32,
                            mode="plain", seed_k=1),
    "matern32_n65536": Workload("matern32_n65536", 65536, 3, "matern32", 0.2, 1e-6, 256, 64,
                                nrhs=16, seed_k=2),
    "matern32_n262144": Workload("matern32_n262144", 262144, 3, "matern32", 0.2, 1e-6, 256, 96,
                                 seed_k=3),
    "exp3d_n1048576": Workload("exp3d_n1048576", 1048576, 3, "exponential", 0.1, 0.0, 256, 0,
                               tol=1e-8, seed_k=5),
}


LAPLACE_TOLS = (3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 1e-6, 1e-8)


def rank_label_problems():
    """Rank-label problems of the Laplace-2D kernel (Table 3, eps 1e-9) for the
    learned rank model, as (n, geometry, seed, leaf, tol): the paper's grid at
    128^2 and 512^2 points and uniform points in the unit square (seed 1200+k)
    at four sizes, leaf 128 and 256, eight tolerances. Test matrices use seed
    3200+k (k = 0 for the grids). The 256^2 grid is kept out, for held-out
    checks."""
    probs = []
    for n, geo, seed in ((16384, "grid2d", 0), (262144, "grid2d", 0), (16384, "uniform", 20), (32768, "uniform", 21),
                         (65536, "uniform", 22), (131072, "uniform", 23)):
        for leaf in (128, 256):
            for tol in LAPLACE_TOLS:
                probs.append((n, geo, seed, leaf, tol))
    return probs


def random_hss(n_leaves_log2: int, leaf: int, rank: int, seed: int, coupling: float = 0.3,
               margin: float = 1.0):
    """A random HSS matrix with orthonormal bases, for factorization tests that
    must not depend on compression (any N, no kernel evaluation).

    Returns a dict with `levels`, `ranges`, `rank` and per-node lists `D`, `U`,
    `E`, `S` in the layout of the HSS format (root level 0, leaves level L):
    U[i] is leaf x rank, E[l][i] is 2*rank x rank, S[l][i] is rank x rank.
    Orthonormal factors come from QR of Gaussian matrices; couplings are scaled
    so that every S has spectral norm <= `coupling`; each D is G G^T/leaf +
    (margin + 2*L*coupling) I, which keeps the assembled matrix SPD (the
    off-diagonal part has norm at most L*coupling)."""
    rng = np.random.default_rng(seed)
    L = n_leaves_log2
    n = leaf * (2 ** L)
    ranges = [[(i * (n >> l), (i + 1) * (n >> l)) for i in range(2 ** l)] for l in range(L + 1)]
    ranks = [[] for _ in range(L + 1)]
    for l in range(1, L + 1):
        ranks[l] = [rank] * (2 ** l)

    def orth(rows, cols):
        q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
        return np.asfortranarray(q)

    D, U = [], []
    shift = margin + 2.0 * L * coupling
    for _ in range(2 ** L):
        G = rng.standard_normal((leaf, leaf))
        D.append(np.asfortranarray(G @ G.T / leaf + shift * np.eye(leaf)))
        U.append(orth(leaf, rank))
    E = [[] for _ in range(L)]
    for l in range(1, L):
        E[l] = [orth(2 * rank, rank) for _ in range(2 ** l)]
    S = [[] for _ in range(L)]
    for l in range(L):
        for _ in range(2 ** l):
            M = rng.standard_normal((rank, rank))
            M *= coupling / np.linalg.norm(M, 2)
            S[l].append(np.asfortranarray(M))
    return {"n": n, "levels": L, "ranges": ranges, "rank": ranks, "D": D, "U": U, "E": E, "S": S}


def batch_gaussian(count: int = 64, seed: int = 4) -> list:
    """The batched workload: `count` independent systems, N ~ U{4096..32768},
    points uniform in the unit cube, Gaussian kernel exp(-r^2/l^2) with
    l ~ U[0.05, 0.3] plus 1e-5 on the diagonal, leaf 128 below N = 16384 and
    256 above, adaptive truncation at 1e-6 with ranks capped at leaf/2.
    System i draws its points, right-hand side and test matrix from seeds
    1100+i, 2100+i and 3100+i; the sizes and lengths come from seed `seed`."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(4096, 32768, size=count, endpoint=True)
    ls = rng.uniform(0.05, 0.3, size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        leaf = 128 if n < 16384 else 256
        out.append(Workload(f"gaussian_batch{count}_sys{i}", n, 3, "gaussian", float(ls[i]), 1e-5, leaf, 0,
                            tol=1e-6, seed_k=100 + i, extra={"max_rank": leaf // 2}))
    return out


def mlp_init(sizes=(7, 128, 128, 128, 1), seed: int = 5000) -> list:
    """Initial weights of a multilayer perceptron: W (out x in) ~ N(0, 2/in)
    (He initialisation), b = 0; float64 [(W, b), ...]."""
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((o, i)) * math.sqrt(2.0 / i), np.zeros(o)) for i, o in zip(sizes[:-1], sizes[1:])]


def minibatch_order(n: int, epochs: int, seed: int = 5100) -> np.ndarray:
    """Concatenated random permutations of range(n), one per epoch (int64)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(n) for _ in range(epochs)]).astype(np.int64)
