"""CPU FP64 oracle for HSS construction, HSS-ULV factorization, ULV solve,
log-determinant and HSS matrix-vector product.

TEST INFRASTRUCTURE ONLY. This module is the slow, plain reference that the GPU
library is checked against. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does. It
shares no code with the HIP library: it reads the same seeded inputs (points,
right-hand sides, Gaussian test matrices) and nothing else.

Everything is float64, written step by step in the order of the paper
("O(N) distributed direct factorization of structured dense matrices using
runtime systems", Deshmukh, Ma, Yokota, Bosilca, ICPP 2023), with numpy/scipy
primitives (matmul, Cholesky, triangular solve, unpivoted QR) as single steps.

Notation follows the paper: D = dense diagonal blocks A_{l;i,i} at the leaf
level, U = leaf shared bases, E = transfer matrices of the nested basis (the
upper-level U_{l;i} of Sec. 2, Eq. 6), S = skeleton (coupling) blocks between
the two children of a node. Level 0 is the root, level L = max_level holds the
leaves; node i of level l has children 2i and 2i+1 on level l+1.

Parity status per function:
  * ulv_factor / ulv_solve / logdet / matvec / densify: pinned (dense Cholesky of
    the densified matrix, closed-form Schur complement, complement invariance,
    BLR^2-ULV equivalence, full-rank and single-level special cases).
  * construct_plain: pinned by invariants (orthonormality, zero structure of
    Eq. 8, Eckart-Young lower bound on truncation error, exactness at full rank).
  * construct_scaled: pinned by invariants (SPD by construction, exact at full
    rank, Schur complement equals R R^T of the scaled basis QR).
  * qrcp: pinned against brute force (pivot = argmax of residual column norms,
    A P = Q R reconstruction).
  * blr2_factor / blr2_solve / blr2_logdet: pinned (dense solve and slogdet of
    the densified matrix, agreement with the HSS-ULV solve, single-level case
    where the skeleton matrix is the root block).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

# ----------------------------------------------------------------------------
# Kernels (Table 3 of the paper, plus the covariance kernels of the workloads)
# ----------------------------------------------------------------------------

KERNELS = ("exponential", "matern32", "gaussian", "laplace2d", "yukawa")


@dataclass(frozen=True)
class Kernel:
    """A radial kernel f(d) with a diagonal nugget c: A_ij = f(|x_i - x_j|) + c*delta_ij.

    exponential: sigma2*exp(-d/l). The paper's Matern with rho = nu = 1/2,
                 sigma = 1, mu = 0.03 (Table 3) reduces to this with l = mu.
    matern32:    sigma2*(1 + sqrt3 d/l) exp(-sqrt3 d/l) (Matern nu = 3/2).
    gaussian:    sigma2*exp(-d^2/l^2).
    laplace2d:   -ln(eps + d), eps = 1e-9 (Table 3).
    yukawa:      exp(-alpha (theta + d)) / (theta + d), alpha = 1, theta = 1e-9 (Table 3).
    """

    kind: str
    length: float = 1.0
    nugget: float = 0.0
    sigma2: float = 1.0
    alpha: float = 1.0
    eps: float = 1e-9

    def f(self, d: np.ndarray) -> np.ndarray:
        k = self.kind
        if k == "exponential":
            return self.sigma2 * np.exp(-d / self.length)
        if k == "matern32":
            t = math.sqrt(3.0) * d / self.length
            return self.sigma2 * (1.0 + t) * np.exp(-t)
        if k == "gaussian":
            return self.sigma2 * np.exp(-(d * d) / (self.length * self.length))
        if k == "laplace2d":
            return -np.log(self.eps + d)
        if k == "yukawa":
            t = self.eps + d
            return np.exp(-self.alpha * t) / t
        raise ValueError(f"unknown kernel {k}")


def pairwise_dist(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Euclidean distances, computed coordinate by coordinate."""
    acc = np.zeros((X.shape[0], Y.shape[0]))
    for a in range(X.shape[1]):
        diff = X[:, a][:, None] - Y[:, a][None, :]
        acc += diff * diff
    return np.sqrt(acc)


def kernel_block(kern: Kernel, X: np.ndarray, Y: np.ndarray, same: bool = False) -> np.ndarray:
    """K(X, Y); if `same` (the block is a diagonal block), the nugget is added on its diagonal."""
    K = kern.f(pairwise_dist(X, Y))
    if same:
        K = K + kern.nugget * np.eye(X.shape[0])
    return K


def dense_matrix(kern: Kernel, X: np.ndarray) -> np.ndarray:
    """The full dense kernel matrix A = K(X, X) + c I (small N only)."""
    return kernel_block(kern, X, X, same=True)


# ----------------------------------------------------------------------------
# Cluster tree: recursive coordinate bisection
# ----------------------------------------------------------------------------


@dataclass
class Tree:
    """Binary cluster tree over the points in tree order.

    perm[t] = original index of the point at tree position t.
    ranges[l][i] = (lo, hi): half-open range of node i of level l in tree order.
    """

    perm: np.ndarray
    levels: int
    ranges: list

    def size(self, l: int, i: int) -> int:
        lo, hi = self.ranges[l][i]
        return hi - lo


def num_levels(n: int, leaf: int) -> int:
    """L = ceil(log2(N / leaf)), 0 when N <= leaf."""
    if n <= leaf:
        return 0
    return int(math.ceil(math.log2(n / leaf) - 1e-12))


def build_tree(points: np.ndarray, leaf: int, levels: int | None = None) -> Tree:
    """Recursive coordinate bisection (binary-bisection ordering of the workloads;
    the paper's experiments use a uniform grid, Results section).

    At each node: split along the longest side of the bounding box of its points
    (ties: lowest axis); order the node's points by (coordinate on that axis,
    original index); the left child takes the first ceil(s/2) points.
    """
    n = points.shape[0]
    L = num_levels(n, leaf) if levels is None else levels
    perm = np.arange(n, dtype=np.int64)
    ranges = [[(0, n)]]
    for l in range(L):
        nxt = []
        for lo, hi in ranges[l]:
            idx = perm[lo:hi]
            P = points[idx]
            ext = P.max(axis=0) - P.min(axis=0)
            axis = int(np.argmax(ext))  # first maximum = lowest axis on ties
            order = np.lexsort((idx, P[:, axis]))  # primary key coordinate, secondary index
            perm[lo:hi] = idx[order]
            mid = lo + (hi - lo + 1) // 2
            nxt += [(lo, mid), (mid, hi)]
        ranges.append(nxt)
    return Tree(perm=perm, levels=L, ranges=ranges)


# ----------------------------------------------------------------------------
# Column-pivoted Householder QR (the pivoted QR of Eq. 2)
# ----------------------------------------------------------------------------


def qrcp(B: np.ndarray, kmax: int):
    """Column-pivoted Householder QR, stopped after kmax steps.

    At step j the pivot is the remaining column of largest Euclidean norm (norms
    recomputed from the current residual; the first index wins ties). Returns
    (Q, R, piv) with Q = n x k orthonormal (k = kmax), R = k x ncols upper
    trapezoidal in pivoted column order, B[:, piv] ~= Q R, and the sign
    convention R[j, j] >= 0.
    """
    A = np.array(B, dtype=np.float64, copy=True)
    n, c = A.shape
    k = min(kmax, n, c)
    piv = np.arange(c)
    vs = []
    for j in range(k):
        norms = np.sqrt(np.sum(A[j:, j:] ** 2, axis=0))
        p = j + int(np.argmax(norms))
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            piv[[j, p]] = piv[[p, j]]
        x = A[j:, j].copy()
        alpha = np.linalg.norm(x)
        v = x.copy()
        if alpha == 0.0:
            vs.append(None)
            continue
        # reflector mapping x to -sign(x0) * alpha * e0
        s = 1.0 if x[0] >= 0 else -1.0
        v[0] = x[0] + s * alpha
        v /= np.linalg.norm(v)
        A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
        vs.append(v)
    R = np.triu(A[:k, :])
    Q = np.zeros((n, k))
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        v = vs[j]
        if v is None:
            continue
        Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    # sign convention: nonnegative diagonal of R
    sgn = np.where(np.diag(R[:, :k]) < 0, -1.0, 1.0)
    Q = Q * sgn[None, :]
    R = R * sgn[:, None]
    return Q, R, piv


def choose_rank(R: np.ndarray, rank: int, tol: float, max_rank: int, n: int) -> int:
    """Truncation rank: fixed `rank` if rank > 0; otherwise the number of leading
    pivots with |R_jj| > tol*|R_00|, capped at max_rank. Always 1 <= k <= n."""
    if rank > 0:
        k = min(rank, R.shape[0])
    else:
        d = np.abs(np.diag(R[:, : R.shape[0]]))
        if d.size == 0 or d[0] == 0.0:
            k = 1
        else:
            k = 0
            while k < d.size and d[k] > tol * d[0]:
                k += 1
            k = max(k, 1)
        if max_rank > 0:
            k = min(k, max_rank)
    return max(1, min(k, n))


# ----------------------------------------------------------------------------
# HSS representation
# ----------------------------------------------------------------------------


@dataclass
class HSS:
    """An HSS matrix (Sec. 2): leaf dense blocks D, leaf bases U, transfer
    matrices E for levels 1..L-1, sibling couplings S for levels 0..L-1.

    rank[l][i] = column count of the basis of node (l, i), l = 1..L.
    E[l][i]: (rank[l+1][2i] + rank[l+1][2i+1]) x rank[l][i], for 1 <= l < L.
    S[l][i]: rank[l+1][2i] x rank[l+1][2i+1], coupling of the children of (l, i).
    """

    n: int
    levels: int
    ranges: list
    rank: list
    D: list
    U: list
    E: list
    S: list
    meta: dict = field(default_factory=dict)

    def node_size(self, l: int, i: int) -> int:
        """Row count of the level-l diagonal block of node i in the ULV sweep."""
        if l == self.levels:
            lo, hi = self.ranges[l][i]
            return hi - lo
        return self.rank[l + 1][2 * i] + self.rank[l + 1][2 * i + 1]

    def basis(self, l: int, i: int) -> np.ndarray:
        return self.U[i] if l == self.levels else self.E[l][i]


def _big_bases(h: HSS):
    """Ubig[l][i]: the nested basis of node (l, i) expressed over its points
    (Eq. 6: blkdiag(children's bases) times the transfer matrix)."""
    L = h.levels
    Ub = [None] * (L + 1)
    Ub[L] = list(h.U)
    for l in range(L - 1, 0, -1):
        row = []
        for i in range(2 ** l):
            c1, c2 = Ub[l + 1][2 * i], Ub[l + 1][2 * i + 1]
            blk = sla.block_diag(c1, c2)
            row.append(blk @ h.E[l][i])
        Ub[l] = row
    return Ub


def densify(h: HSS) -> np.ndarray:
    """Assemble the dense matrix represented by the HSS form (small N only).

    Diagonal leaf blocks are D; the block between the two children of node
    (l, i) is Ubig_c1 S Ubig_c2^T (Eq. 1 / Eq. 6), and its transpose below."""
    A = np.zeros((h.n, h.n))
    L = h.levels
    if L == 0:
        return np.array(h.D[0], copy=True)
    for i, (lo, hi) in enumerate(h.ranges[L]):
        A[lo:hi, lo:hi] = h.D[i]
    Ub = _big_bases(h)
    for l in range(0, L):
        for i in range(2 ** l):
            a1, b1 = h.ranges[l + 1][2 * i]
            a2, b2 = h.ranges[l + 1][2 * i + 1]
            blk = Ub[l + 1][2 * i] @ h.S[l][i] @ Ub[l + 1][2 * i + 1].T
            A[a1:b1, a2:b2] = blk
            A[a2:b2, a1:b1] = blk.T
    return A


# ----------------------------------------------------------------------------
# Construction, plain (Sec. 2: pivoted QR of the admissible row block, Eq. 2)
# ----------------------------------------------------------------------------


def construct_plain(X: np.ndarray, tree: Tree, kern: Kernel, rank: int = 0, tol: float = 0.0,
                    max_rank: int = 0, A: np.ndarray | None = None) -> HSS:
    """The paper's construction with exact blocks (small N only).

    Leaf i: the basis is the first k columns of the pivoted QR of the off-diagonal
    row block A[I_i, I_i^c] (= A_{+,i}^T by symmetry, Eq. 2). Level l < L, node p
    with children c1, c2: the transfer matrix comes from the pivoted QR of the
    children-projected row block blkdiag(Ubig_c1, Ubig_c2)^T A[I_p, I_p^c]. The
    coupling of siblings is the orthogonal projection Ubig_c1^T A[I_c1, I_c2] Ubig_c2.
    """
    Xt = X[tree.perm]
    if A is None:
        A = dense_matrix(kern, Xt)
    n = Xt.shape[0]
    L = tree.levels
    if L == 0:
        return HSS(n, 0, tree.ranges, [[]], [A.copy()], [], [], [], meta={"mode": "plain"})
    ranks = [[] for _ in range(L + 1)]
    U = []
    D = []
    Ub = [None] * (L + 1)
    Ub[L] = []
    for (lo, hi) in tree.ranges[L]:
        D.append(A[lo:hi, lo:hi].copy())
        B = np.concatenate([A[lo:hi, :lo], A[lo:hi, hi:]], axis=1)
        Q, R, _ = qrcp(B, rank if rank > 0 else min(B.shape))
        k = choose_rank(R, rank, tol, max_rank, hi - lo)
        U.append(Q[:, :k].copy())
        Ub[L].append(Q[:, :k].copy())
        ranks[L].append(k)
    E = [[] for _ in range(L)]
    for l in range(L - 1, 0, -1):
        Ub[l] = []
        for i, (lo, hi) in enumerate(tree.ranges[l]):
            c1, c2 = Ub[l + 1][2 * i], Ub[l + 1][2 * i + 1]
            blk = sla.block_diag(c1, c2)
            Brow = np.concatenate([A[lo:hi, :lo], A[lo:hi, hi:]], axis=1)
            B = blk.T @ Brow
            Q, R, _ = qrcp(B, rank if rank > 0 else min(B.shape))
            k = choose_rank(R, rank, tol, max_rank, B.shape[0])
            E[l].append(Q[:, :k].copy())
            Ub[l].append(blk @ Q[:, :k])
            ranks[l].append(k)
    S = [[] for _ in range(L)]
    for l in range(L):
        for i in range(2 ** l):
            a1, b1 = tree.ranges[l + 1][2 * i]
            a2, b2 = tree.ranges[l + 1][2 * i + 1]
            S[l].append(Ub[l + 1][2 * i].T @ A[a1:b1, a2:b2] @ Ub[l + 1][2 * i + 1])
    return HSS(n, L, tree.ranges, ranks, D, U, E, S, meta={"mode": "plain"})


def construct_plain_sampled(X: np.ndarray, tree: Tree, kern: Kernel, omega: np.ndarray, rank: int = 0,
                            tol: float = 0.0, max_rank: int = 0, A: np.ndarray | None = None) -> HSS:
    """The paper's construction (Sec. 2, Eq. 2 and Eq. 6) with the off-diagonal
    row blocks seen through random samples instead of formed (small N only).

    The test matrix Omega (N x s, tree order) is given. The samples of the leaves'
    off-diagonal row blocks are the block rows of (A - blkdiag(D)) Omega, i.e.
    A[I_i, I_i^c] Omega[I_i^c]. At every level, from the leaves, node p's basis
    (U at a leaf, the transfer matrix E above) is the first k columns of the
    pivoted QR of its samples Z_p. The coupling of siblings is the orthogonal
    projection Ubig_c1^T A[I_c1, I_c2] Ubig_c2. The samples move up by
    projecting onto the children's bases and removing the sibling block through
    its compressed form:
      Phi_p = [B_c1^T Phi_c1; B_c2^T Phi_c2]        (Phi = Omega at the leaves)
      Z_p   = [B_c1^T Z_c1 - S Phi_c2; B_c2^T Z_c2 - S^T Phi_c1]
    (B the child's basis), which samples the children-projected row block
    blkdiag(Ubig_c1, Ubig_c2)^T A[I_p, I_p^c] of the exact construction exactly
    when the sibling block equals its compressed form.
    """
    if A is None:
        A = dense_matrix(kern, X[tree.perm])
    n = A.shape[0]
    L = tree.levels
    if L == 0:
        return HSS(n, 0, tree.ranges, [[]], [A.copy()], [], [], [], meta={"mode": "plain_sampled"})
    s = omega.shape[1]
    ranks = [[] for _ in range(L + 1)]
    D = [A[lo:hi, lo:hi].copy() for (lo, hi) in tree.ranges[L]]
    Aoff = A.copy()
    for (lo, hi) in tree.ranges[L]:
        Aoff[lo:hi, lo:hi] = 0.0
    Zall = Aoff @ omega
    Z = [Zall[lo:hi] for (lo, hi) in tree.ranges[L]]
    Phi = [omega[lo:hi] for (lo, hi) in tree.ranges[L]]
    U = []
    E = [[] for _ in range(L)]
    S = [[] for _ in range(L)]
    Ubig_prev = None
    for l in range(L, 0, -1):
        nodes = 2 ** l
        Bs = []
        for p in range(nodes):
            Q, R, _ = qrcp(Z[p], rank if rank > 0 else min(Z[p].shape))
            k = choose_rank(R, rank, tol, max_rank, Z[p].shape[0])
            B = Q[:, :k].copy()
            Bs.append(B)
            ranks[l].append(k)
            if l == L:
                U.append(B)
            else:
                E[l].append(B)
        if l == L:
            Ubig = Bs
        else:
            Ubig = [sla.block_diag(Ubig_prev[2 * p], Ubig_prev[2 * p + 1]) @ Bs[p] for p in range(nodes)]
        newZ, newPhi = [], []
        for g in range(nodes // 2):
            p1, p2 = 2 * g, 2 * g + 1
            a1, b1 = tree.ranges[l][p1]
            a2, b2 = tree.ranges[l][p2]
            Sg = Ubig[p1].T @ A[a1:b1, a2:b2] @ Ubig[p2]
            S[l - 1].append(Sg)
            ph1 = Bs[p1].T @ Phi[p1]
            ph2 = Bs[p2].T @ Phi[p2]
            newPhi.append(np.vstack([ph1, ph2]))
            newZ.append(np.vstack([Bs[p1].T @ Z[p1] - Sg @ ph2, Bs[p2].T @ Z[p2] - Sg.T @ ph1]))
        Z, Phi, Ubig_prev = newZ, newPhi, Ubig
    return HSS(n, L, tree.ranges, ranks, D, U, E, S, meta={"mode": "plain_sampled", "s": s})


# ----------------------------------------------------------------------------
# Construction, scaled (Cholesky-scaled compression; keeps the HSS matrix SPD)
# ----------------------------------------------------------------------------


def _qr_posdiag(K: np.ndarray):
    """Thin Householder QR with R's diagonal made nonnegative."""
    Q, R = np.linalg.qr(K, mode="reduced")
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sgn[None, :], R * sgn[:, None]


def construct_scaled(X: np.ndarray, tree: Tree, kern: Kernel, omega: np.ndarray, rank: int = 0,
                     tol: float = 0.0, max_rank: int = 0, A: np.ndarray | None = None,
                     return_aux: bool = False):
    """Randomized, Cholesky-scaled construction of the HSS form (small N only).

    The paper's HSS format is kept (orthonormal leaf bases U, orthonormal transfer
    matrices E, couplings S), but each node's off-diagonal row block is compressed
    after scaling by the inverse Cholesky factor of the node's diagonal block, so
    the represented matrix stays symmetric positive definite for any truncation.

    Level by level from the leaves, with M_p the current diagonal block of node p
    (D at the leaves) and Z_p samples of its off-diagonal row block:
      Lc = chol(M_p);  Y = Lc^{-1} Z_p;  V = first k columns of the pivoted QR of Y;
      Lc V = B R (thin QR, diag(R) >= 0);  basis (U or E) = B;  Sigma_p = R R^T;
      W_p = Lc^{-T} V R^T  (so that W_p^T B = I and W_p^T M_p W_p = Sigma_p).
    Siblings p1, p2 of parent g: S_g = Wbig_p1^T A[I_p1, I_p2] Wbig_p2 with
    Wbig_p = blkdiag(Wbig_children) W_p; the parent's diagonal block is
    M_g = [[Sigma_p1, S_g], [S_g^T, Sigma_p2]].
    Sampling: the test matrix Omega (N x s) is given. Leaf samples use
    Psi_p = Lc_p^{-T} Omega_p and Z = (A - blkdiag(D)) Psi. Samples move up by
    Phi_g = [B_p1^T Phi_p1; B_p2^T Phi_p2] and
    Z_g = [W_p1^T Z_p1 - S_g Phi_p2; W_p2^T Z_p2 - S_g^T Phi_p1].
    """
    Xt = X[tree.perm]
    if A is None:
        A = dense_matrix(kern, Xt)
    n = Xt.shape[0]
    L = tree.levels
    if L == 0:
        return HSS(n, 0, tree.ranges, [[]], [A.copy()], [], [], [], meta={"mode": "scaled"})
    s = omega.shape[1]
    ranks = [[] for _ in range(L + 1)]
    D = []
    # leaf level setup
    M = []
    Psi = np.zeros_like(omega)
    for (lo, hi) in tree.ranges[L]:
        Dp = A[lo:hi, lo:hi].copy()
        D.append(Dp)
        M.append(Dp)
        Lc = np.linalg.cholesky(Dp)
        Psi[lo:hi] = sla.solve_triangular(Lc, omega[lo:hi], lower=True, trans="T")
    Aoff = A.copy()
    for (lo, hi) in tree.ranges[L]:
        Aoff[lo:hi, lo:hi] = 0.0
    Zall = Aoff @ Psi
    Z = [Zall[lo:hi] for (lo, hi) in tree.ranges[L]]
    Phi = [Psi[lo:hi] for (lo, hi) in tree.ranges[L]]
    Wbig_prev = None
    U = []
    E = [[] for _ in range(L)]
    S = [[] for _ in range(L)]
    aux = {"Sigma": [None] * (L + 1), "W": [None] * (L + 1)}
    for l in range(L, 0, -1):
        nodes = 2 ** l
        Bs, Ws, Sig = [], [], []
        for p in range(nodes):
            Lc = np.linalg.cholesky(M[p])
            Y = sla.solve_triangular(Lc, Z[p], lower=True)
            npts = M[p].shape[0]
            Q, R0, _ = qrcp(Y, rank if rank > 0 else min(Y.shape))
            k = choose_rank(R0, rank, tol, max_rank, npts)
            V = Q[:, :k]
            B, R = _qr_posdiag(Lc @ V)
            W = sla.solve_triangular(Lc, V @ R.T, lower=True, trans="T")
            Bs.append(B)
            Ws.append(W)
            Sig.append(R @ R.T)
            ranks[l].append(k)
            if l == L:
                U.append(B)
            else:
                E[l].append(B)
        # big W over points
        if l == L:
            Wbig = Ws
        else:
            Wbig = [sla.block_diag(Wbig_prev[2 * p], Wbig_prev[2 * p + 1]) @ Ws[p] for p in range(nodes)]
        aux["Sigma"][l] = Sig
        aux["W"][l] = Ws
        # couplings and parent blocks
        newM, newZ, newPhi = [], [], []
        for g in range(nodes // 2):
            p1, p2 = 2 * g, 2 * g + 1
            a1, b1 = tree.ranges[l][p1]
            a2, b2 = tree.ranges[l][p2]
            Sg = Wbig[p1].T @ A[a1:b1, a2:b2] @ Wbig[p2]
            S[l - 1].append(Sg)
            newM.append(np.block([[Sig[p1], Sg], [Sg.T, Sig[p2]]]))
            ph1 = Bs[p1].T @ Phi[p1]
            ph2 = Bs[p2].T @ Phi[p2]
            z1 = Ws[p1].T @ Z[p1] - Sg @ ph2
            z2 = Ws[p2].T @ Z[p2] - Sg.T @ ph1
            newPhi.append(np.vstack([ph1, ph2]))
            newZ.append(np.vstack([z1, z2]))
        M, Z, Phi, Wbig_prev = newM, newZ, newPhi, Wbig
    aux["root"] = M[0]
    h = HSS(n, L, tree.ranges, ranks, D, U, E, S, meta={"mode": "scaled", "s": s})
    return (h, aux) if return_aux else h


# ----------------------------------------------------------------------------
# HSS-ULV factorization (Alg. 2), log-determinant, solve (Eq. 17)
# ----------------------------------------------------------------------------


@dataclass
class ULVFactor:
    """Per node (l, i): Q = [U^R U^S] (Eq. 3 / Eq. 9), L_RR, L_SR (Eq. 10-11) and
    the Schur complement Sigma = A^SS - L_SR L_SR^T (Eq. 12) in U^S coordinates;
    the root's Cholesky factor L0 (Alg. 2, final factorization)."""

    levels: int
    Q: list
    LRR: list
    LSR: list
    Sigma: list
    L0: np.ndarray
    logdet: float
    root_block: np.ndarray


class NotSPD(Exception):
    def __init__(self, level, node):
        super().__init__(f"non-positive pivot at level {level}, node {node}")
        self.level, self.node = level, node


def complement_basis(Us: np.ndarray) -> np.ndarray:
    """An orthonormal complement U^R of the orthonormal basis U^S (full QR)."""
    n, k = Us.shape
    Qf, _ = sla.qr(Us, mode="full")
    return Qf[:, k:]


def _chol(M, l, i):
    try:
        return np.linalg.cholesky(M)
    except np.linalg.LinAlgError:
        raise NotSPD(l, i)


def ulv_factor(h: HSS, complement=complement_basis) -> ULVFactor:
    """HSS-ULV factorization, Alg. 2.

    For l = L..1 and each node: the diagonal product A_hat = Q^T M Q with
    Q = [U^R U^S] (Eq. 7 and Eq. 9); the partial Cholesky of Eq. 10-12
    (L_RR = chol(A_hat^RR), L_SR = A_hat^SR L_RR^{-T}, Sigma = A_hat^SS - L_SR L_SR^T);
    then the merge of sibling Schur complements with their coupling into the
    parent's diagonal block (the permutation P_l). Finally the root block is
    factored by a dense Cholesky. The log-determinant is twice the sum of the
    logarithms of all pivots, since |det Q| = 1.
    """
    L = h.levels
    if L == 0:
        L0 = _chol(h.D[0], 0, 0)
        return ULVFactor(0, [], [], [], [], L0, 2.0 * float(np.sum(np.log(np.diag(L0)))), h.D[0])
    Qs = [None] * (L + 1)
    LRRs = [None] * (L + 1)
    LSRs = [None] * (L + 1)
    Sigs = [None] * (L + 1)
    logdet = 0.0
    M = [np.array(d, copy=True) for d in h.D]
    for l in range(L, 0, -1):
        Ql, Rl, Sl, Gl = [], [], [], []
        for i in range(2 ** l):
            Us = h.basis(l, i)
            n, k = Us.shape
            m = n - k
            Q = np.hstack([complement(Us), Us])
            Ahat = Q.T @ M[i] @ Q
            if m > 0:
                LRR = _chol(Ahat[:m, :m], l, i)
                LSR = sla.solve_triangular(LRR, Ahat[:m, m:], lower=True).T  # A^SR L_RR^{-T}
                Sig = Ahat[m:, m:] - LSR @ LSR.T
                logdet += 2.0 * float(np.sum(np.log(np.diag(LRR))))
            else:
                LRR = np.zeros((0, 0))
                LSR = np.zeros((k, 0))
                Sig = Ahat
            Sig = 0.5 * (Sig + Sig.T)
            Ql.append(Q)
            Rl.append(LRR)
            Sl.append(LSR)
            Gl.append(Sig)
        Qs[l], LRRs[l], LSRs[l], Sigs[l] = Ql, Rl, Sl, Gl
        M = [np.block([[Gl[2 * g], h.S[l - 1][g]], [h.S[l - 1][g].T, Gl[2 * g + 1]]])
             for g in range(2 ** (l - 1))]
    L0 = _chol(M[0], 0, 0)
    logdet += 2.0 * float(np.sum(np.log(np.diag(L0))))
    return ULVFactor(L, Qs, LRRs, LSRs, Sigs, L0, logdet, M[0])


def ulv_solve(h: HSS, F: ULVFactor, b: np.ndarray) -> np.ndarray:
    """ULV solve, Eq. 17, read as ordered products (leaf level applied first).

    Forward, leaf to root: b_hat = Q^T b; y_R = L_RR^{-1} b_hat_R;
    z_S = b_hat_S - L_SR y_R; the parent's right-hand side stacks the children's z_S.
    Root: w = L0^{-T} L0^{-1} z. Backward, root to leaf: split w into the
    children's x_S; x_R = L_RR^{-T}(y_R - L_SR^T x_S); x = Q [x_R; x_S].
    Input and output are in tree order; columns are independent right-hand sides.
    """
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    B = b[:, None] if vec else b
    L = h.levels
    if L == 0:
        y = sla.solve_triangular(F.L0, B, lower=True)
        x = sla.solve_triangular(F.L0, y, lower=True, trans="T")
        return x[:, 0] if vec else x
    rhs = [B[lo:hi] for (lo, hi) in h.ranges[L]]
    ys = [None] * (L + 1)
    for l in range(L, 0, -1):
        yl, zl = [], []
        for i in range(2 ** l):
            Q, LRR, LSR = F.Q[l][i], F.LRR[l][i], F.LSR[l][i]
            m = LRR.shape[0]
            bh = Q.T @ rhs[i]
            yR = sla.solve_triangular(LRR, bh[:m], lower=True) if m > 0 else bh[:0]
            zS = bh[m:] - LSR @ yR
            yl.append(yR)
            zl.append(zS)
        ys[l] = yl
        rhs = [np.vstack([zl[2 * g], zl[2 * g + 1]]) for g in range(2 ** (l - 1))]
    w = sla.solve_triangular(F.L0, rhs[0], lower=True)
    w = sla.solve_triangular(F.L0, w, lower=True, trans="T")
    xs = [w]
    for l in range(1, L + 1):
        nxt = []
        for g in range(2 ** (l - 1)):
            k1 = F.Q[l][2 * g].shape[1] - F.LRR[l][2 * g].shape[0]
            parts = [xs[g][:k1], xs[g][k1:]]
            for c in range(2):
                i = 2 * g + c
                Q, LRR, LSR = F.Q[l][i], F.LRR[l][i], F.LSR[l][i]
                xS = parts[c]
                if LRR.shape[0] > 0:
                    xR = sla.solve_triangular(LRR, ys[l][i] - LSR.T @ xS, lower=True, trans="T")
                else:
                    xR = xS[:0]
                nxt.append(Q @ np.vstack([xR, xS]))
        xs = nxt
    x = np.vstack(xs)
    return x[:, 0] if vec else x


# ----------------------------------------------------------------------------
# BLR^2-ULV (Alg. 1): leaf-level partial factorization, then one dense Cholesky
# ----------------------------------------------------------------------------


@dataclass
class BLR2Factor:
    """BLR^2-ULV factors (Alg. 1): per leaf i, Q_i = [U^R_i U^S_i] (Eq. 9), L_RR
    and L_SR (Eq. 10-11); the dense Cholesky factor Lss of the permuted
    skeleton matrix (Eq. 13), whose block (i, j) is Sigma_i on the diagonal
    (Eq. 12) and U_i^T A_ij U_j off it; offs[i] = first skeleton row of leaf i."""

    Q: list
    LRR: list
    LSR: list
    Lss: np.ndarray
    offs: np.ndarray
    logdet: float


def blr2_skeleton_matrix(h: HSS):
    """The skeleton-space matrix of Alg. 1's last step before its Cholesky, with
    the per-leaf factors: Sigma_i on the diagonal and, between leaves i and j
    under the two children of node (l, g), the coupling S_(l,g) expressed in the
    leaves' own bases through the transfer matrices below it (Eq. 6)."""
    L = h.levels
    Qs, LRRs, LSRs, sig = [], [], [], []
    logdet = 0.0
    for i in range(2 ** L):
        Us = h.U[i]
        n, k = Us.shape
        m = n - k
        Q = np.hstack([complement_basis(Us), Us])
        Ahat = Q.T @ h.D[i] @ Q                                     # Eq. 7 with U^F of Eq. 9
        if m > 0:
            LRR = _chol(Ahat[:m, :m], L, i)                          # Eq. 10
            LSR = sla.solve_triangular(LRR, Ahat[:m, m:], lower=True).T  # Eq. 11
            logdet += 2.0 * float(np.sum(np.log(np.diag(LRR))))
            sig.append(Ahat[m:, m:] - LSR @ LSR.T)                   # Eq. 12
        else:
            LRR, LSR = np.zeros((0, 0)), np.zeros((k, 0))
            sig.append(Ahat)
        Qs.append(Q)
        LRRs.append(LRR)
        LSRs.append(LSR)
    offs = np.cumsum([0] + [u.shape[1] for u in h.U])
    K = int(offs[-1])
    Ass = np.zeros((K, K))
    for i in range(2 ** L):
        Ass[offs[i]:offs[i + 1], offs[i]:offs[i + 1]] = sig[i]
    for l in range(0, L):
        for g in range(2 ** l):
            c1, c2 = 2 * g, 2 * g + 1
            span = 2 ** (L - l - 1)
            T1 = _leaf_to_node(h, l + 1, c1)
            T2 = _leaf_to_node(h, l + 1, c2)
            blk = T1 @ h.S[l][g] @ T2.T
            r1 = np.arange(offs[c1 * span], offs[(c1 + 1) * span])
            r2 = np.arange(offs[c2 * span], offs[(c2 + 1) * span])
            Ass[np.ix_(r1, r2)] = blk
            Ass[np.ix_(r2, r1)] = blk.T
    return Ass, offs, Qs, LRRs, LSRs, logdet


def blr2_factor(h: HSS) -> BLR2Factor:
    """Alg. 1 applied to the HSS matrix viewed at its leaf level (a weakly
    admissible BLR^2 matrix with shared leaf bases): diagonal product and
    partial Cholesky of every leaf block (Eq. 7, 10-12), then the permutation of
    all skeleton rows to the end and one dense Cholesky of the resulting
    (sum of leaf ranks) square matrix (Eq. 13)."""
    L = h.levels
    if L == 0:
        L0 = _chol(h.D[0], 0, 0)
        return BLR2Factor([np.eye(h.n)], [L0], [np.zeros((0, h.n))], np.zeros((0, 0)), np.array([0, 0]),
                          2.0 * float(np.sum(np.log(np.diag(L0)))))
    Ass, offs, Qs, LRRs, LSRs, logdet = blr2_skeleton_matrix(h)
    Lss = _chol(Ass, 0, 0)
    logdet += 2.0 * float(np.sum(np.log(np.diag(Lss))))
    return BLR2Factor(Qs, LRRs, LSRs, Lss, offs, logdet)


def blr2_logdet(h: HSS) -> float:
    """log det of the matrix from its BLR^2-ULV factors: twice the sum of the
    logarithms of every leaf pivot and of the skeleton factor's diagonal."""
    return blr2_factor(h).logdet


def blr2_solve(h: HSS, F: BLR2Factor, b: np.ndarray) -> np.ndarray:
    """BLR^2-ULV solve (Eq. 14) in tree order, read as ordered products:
    per leaf, b^ = Q^T b, y_R = L_RR^{-1} b^_R and z_S = b^_S - L_SR y_R; the
    skeleton parts of all leaves, gathered in leaf order (the permutation P),
    are solved with Lss Lss^T; then per leaf x_R = L_RR^{-T}(y_R - L_SR^T x_S)
    and x = Q [x_R; x_S]."""
    vec = b.ndim == 1
    B = b[:, None] if vec else b
    L = h.levels
    if L == 0:
        L0 = F.LRR[0]
        x = sla.solve_triangular(L0, sla.solve_triangular(L0, B, lower=True), lower=True, trans="T")
        return x[:, 0] if vec else x
    ys, zs = [], []
    for i, (lo, hi) in enumerate(h.ranges[L]):
        m = F.LRR[i].shape[0]
        bh = F.Q[i].T @ B[lo:hi]
        yR = sla.solve_triangular(F.LRR[i], bh[:m], lower=True) if m > 0 else bh[:0]
        ys.append(yR)
        zs.append(bh[m:] - F.LSR[i] @ yR)
    z = np.vstack(zs)
    w = sla.solve_triangular(F.Lss, z, lower=True)
    w = sla.solve_triangular(F.Lss, w, lower=True, trans="T")
    X = np.zeros_like(B)
    for i, (lo, hi) in enumerate(h.ranges[L]):
        m = F.LRR[i].shape[0]
        xS = w[F.offs[i]:F.offs[i + 1]]
        if m > 0:
            xR = sla.solve_triangular(F.LRR[i], ys[i] - F.LSR[i].T @ xS, lower=True, trans="T")
        else:
            xR = xS[:0]
        X[lo:hi] = F.Q[i] @ np.vstack([xR, xS])
    return X[:, 0] if vec else X


def _leaf_to_node(h: HSS, l: int, i: int) -> np.ndarray:
    """Stacked leaf-skeleton coordinates of node (l, i)'s basis: the product of
    transfer matrices from level l down to the leaves (block diagonal nesting)."""
    L = h.levels
    if l == L:
        return np.eye(h.U[i].shape[1])
    c1 = _leaf_to_node(h, l + 1, 2 * i)
    c2 = _leaf_to_node(h, l + 1, 2 * i + 1)
    return sla.block_diag(c1, c2) @ h.E[l][i]


# ----------------------------------------------------------------------------
# HSS matrix-vector product
# ----------------------------------------------------------------------------


def matvec(h: HSS, x: np.ndarray) -> np.ndarray:
    """y = A x for the HSS form (tree order): up-sweep x_i^ = U_i^T x_i and
    x_p^ = E_p^T [x_c1^; x_c2^]; sibling couplings y_c1^ += S x_c2^,
    y_c2^ += S^T x_c1^; down-sweep [y_c1^; y_c2^] += E_p y_p^; leaves
    y_i = D_i x_i + U_i y_i^."""
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = x[:, None] if vec else x
    L = h.levels
    if L == 0:
        y = h.D[0] @ X
        return y[:, 0] if vec else y
    xt = [None] * (L + 1)
    xt[L] = [h.U[i].T @ X[lo:hi] for i, (lo, hi) in enumerate(h.ranges[L])]
    for l in range(L - 1, 0, -1):
        xt[l] = [h.E[l][i].T @ np.vstack([xt[l + 1][2 * i], xt[l + 1][2 * i + 1]]) for i in range(2 ** l)]
    yt = [None] * (L + 1)
    for l in range(1, L + 1):
        yt[l] = [np.zeros_like(xt[l][i]) for i in range(2 ** l)]
    for l in range(0, L):
        for g in range(2 ** l):
            S = h.S[l][g]
            yt[l + 1][2 * g] += S @ xt[l + 1][2 * g + 1]
            yt[l + 1][2 * g + 1] += S.T @ xt[l + 1][2 * g]
    for l in range(1, L):
        for g in range(2 ** l):
            k1 = yt[l + 1][2 * g].shape[0]
            t = h.E[l][g] @ yt[l][g]
            yt[l + 1][2 * g] += t[:k1]
            yt[l + 1][2 * g + 1] += t[k1:]
    Y = np.zeros_like(X)
    for i, (lo, hi) in enumerate(h.ranges[L]):
        Y[lo:hi] = h.D[i] @ X[lo:hi] + h.U[i] @ yt[L][i]
    return Y[:, 0] if vec else Y


# ----------------------------------------------------------------------------
# Error metrics of the Results section (Eq. 18, Eq. 19) and helpers
# ----------------------------------------------------------------------------


def construction_error(A_dense_b: np.ndarray, h: HSS, b: np.ndarray) -> float:
    """Eq. 18: |A_dense b - A b| / |A_dense b| with A the HSS matrix."""
    return float(np.linalg.norm(A_dense_b - matvec(h, b)) / np.linalg.norm(A_dense_b))


def solve_error(h: HSS, F: ULVFactor, b: np.ndarray) -> float:
    """Eq. 19: |b - A^{-1} A b| / |b|."""
    return float(np.linalg.norm(b - ulv_solve(h, F, matvec(h, b))) / np.linalg.norm(b))


def relative_residual(h: HSS, x: np.ndarray, b: np.ndarray) -> float:
    """|b - A x|_2 / |b|_2 with A the HSS matrix (its FP64 matvec)."""
    return float(np.linalg.norm(b - matvec(h, x)) / np.linalg.norm(b))


def to_tree_order(tree: Tree, v: np.ndarray) -> np.ndarray:
    return v[tree.perm]


def from_tree_order(tree: Tree, v: np.ndarray) -> np.ndarray:
    out = np.empty_like(v)
    out[tree.perm] = v
    return out
