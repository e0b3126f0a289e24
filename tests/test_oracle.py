"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the plausible mistake it would catch. None of these tests
compares the oracle with itself: references are dense Cholesky solves, closed
forms, library routines for special cases, brute force on tiny inputs, and
invariants of the HSS-ULV method.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as ssp

import synth
from oracle import hss_oracle as O


def hss_from_dict(d):
    return O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])


@pytest.fixture(scope="module")
def cfg1():
    """The exp(-r/0.1)+1e-4 workload: N=2048 in [0,1]^2, leaf 128, 4 levels, rank 32, plain."""
    w = synth.WORKLOADS["exp2d_n2048"]
    X = w.points()
    kern = O.Kernel("exponential", w.length, w.nugget)
    tree = O.build_tree(X, w.leaf)
    A = O.dense_matrix(kern, X[tree.perm])
    h = O.construct_plain(X, tree, kern, rank=w.rank, A=A)
    F = O.ulv_factor(h)
    b = w.rhs()[:, 0][tree.perm]
    return dict(w=w, X=X, kern=kern, tree=tree, A=A, h=h, F=F, b=b)


# --------------------------------------------------------------------------
# kernels (Table 3) reduce to the general Matern formula / library Bessel K
# --------------------------------------------------------------------------


def matern_general(d, nu, ell, sigma2=1.0):
    z = np.sqrt(2 * nu) * d / ell
    with np.errstate(invalid="ignore"):
        v = sigma2 * 2 ** (1 - nu) / ssp.gamma(nu) * z ** nu * ssp.kv(nu, z)
    return np.where(d == 0, sigma2, v)


def test_kernel_matern32_matches_bessel_form():
    d = np.linspace(0.0, 1.0, 101)
    k = O.Kernel("matern32", 0.2).f(d)
    np.testing.assert_allclose(k, matern_general(d, 1.5, 0.2), rtol=1e-12, atol=1e-14)


def test_paper_matern_half_is_exponential():
    # Table 3: sigma=1, mu=0.03, rho=nu=1/2 with argument d/mu.
    d = np.linspace(0.0, 0.5, 51)
    z = d / 0.03
    with np.errstate(invalid="ignore"):
        paper = np.where(d == 0, 1.0, 2 ** (1 - 0.5) / ssp.gamma(0.5) * z ** 0.5 * ssp.kv(0.5, z))
    np.testing.assert_allclose(O.Kernel("exponential", 0.03).f(d), paper, rtol=1e-12, atol=1e-300)


def test_table3_constants():
    # Laplace 2D: -ln(1e-9 + d); Yukawa: exp(-(1e-9+d))/(1e-9+d) at alpha = 1.
    d = np.array([0.0, 0.5, 1.0])
    np.testing.assert_allclose(O.Kernel("laplace2d").f(d), -np.log(1e-9 + d))
    np.testing.assert_allclose(O.Kernel("yukawa").f(d), np.exp(-(1e-9 + d)) / (1e-9 + d))
    assert abs(O.Kernel("laplace2d").f(np.array([0.0]))[0] - 20.7232658) < 1e-6


def test_nugget_only_on_diagonal():
    X = synth.points_uniform(20, 2, 1)
    K = O.dense_matrix(O.Kernel("gaussian", 0.3, 0.5), X)
    K0 = O.dense_matrix(O.Kernel("gaussian", 0.3, 0.0), X)
    np.testing.assert_allclose(K - K0, 0.5 * np.eye(20), atol=1e-15)


def test_gaussian_kernel_closed_form_values():
    # exp(-d^2/l^2) without a factor 1/2 (the workload's literal form): the value at
    # d = l is 1/e (exp(-d^2/(2 l^2)) would give e^-1/2 there), the value at 0 is
    # sigma2, and squaring the kernel doubles d^2 (f(d)^2 = f(sqrt2 d)), which no
    # other power of d in the exponent satisfies.
    for ell in (0.05, 0.3, 1.7):
        k = O.Kernel("gaussian", ell, sigma2=1.0)
        assert abs(k.f(np.array([ell]))[0] - math.e ** -1) < 1e-15
        d = np.linspace(0.0, 3 * ell, 31)
        np.testing.assert_allclose(k.f(d) ** 2, k.f(math.sqrt(2.0) * d), rtol=1e-13, atol=1e-300)
    assert O.Kernel("gaussian", 0.3, sigma2=2.5).f(np.array([0.0]))[0] == 2.5
    # a known value: d = l/2 gives exp(-1/4) = 0.77880078307...
    assert abs(O.Kernel("gaussian", 0.2).f(np.array([0.1]))[0] - 0.7788007830714049) < 1e-15


def test_yukawa_known_values_and_helmholtz_equation():
    # Table 3's Yukawa potential exp(-alpha t)/t with t = theta + d: at t = 1 it is
    # e^-alpha, and for d > 0 it solves the radial modified Helmholtz equation
    # f'' + (2/t) f' - alpha^2 f = 0 (the screened Coulomb Green's function in 3-D),
    # checked by central differences; a dropped 1/t or a wrong sign fails it.
    k = O.Kernel("yukawa")
    assert abs(k.f(np.array([1.0 - 1e-9]))[0] - math.e ** -1) < 1e-15
    k2 = O.Kernel("yukawa", alpha=2.0, eps=0.0)
    assert abs(k2.f(np.array([0.5]))[0] - 2.0 * math.e ** -1) < 1e-14
    for alpha in (1.0, 3.0):
        kk = O.Kernel("yukawa", alpha=alpha, eps=1e-9)
        t = np.linspace(0.2, 2.0, 10)
        h = 1e-4
        f0, fp, fm = kk.f(t), kk.f(t + h), kk.f(t - h)
        d2 = (fp - 2 * f0 + fm) / h ** 2
        d1 = (fp - fm) / (2 * h)
        res = d2 + 2.0 / (t + 1e-9) * d1 - alpha ** 2 * f0
        assert np.max(np.abs(res) / (alpha ** 2 * np.abs(f0))) < 1e-5


def test_pairwise_dist_matches_scipy_cdist():
    import scipy.spatial.distance as ssd

    for dim, seed in ((1, 1), (2, 2), (3, 3)):
        X = synth.points_uniform(37, dim, seed)
        Y = synth.points_uniform(23, dim, seed + 10)
        np.testing.assert_allclose(O.pairwise_dist(X, Y), ssd.cdist(X, Y), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(np.diag(O.pairwise_dist(X, X)), 0.0, atol=0.0)


def _r_with_diag(d):
    R = np.triu(np.full((len(d), len(d) + 3), 0.25))
    R[np.arange(len(d)), np.arange(len(d))] = d
    return R


def test_choose_rank_tolerance_rule():
    # the adaptive rule keeps the leading pivots with |R_jj| > tol |R_00| and stops
    # at the first one that is not (k = min{j : |R_jj| <= tol |R_00|}): hand-built
    # diagonals with a known k, exact ties (powers of two), a non-monotone diagonal,
    # the max_rank cap, a zero R and the fixed-rank path
    R = _r_with_diag([10.0, 5.0, 1.0, 0.1, 0.01, 0.001])
    assert O.choose_rank(R, 0, 0.05, 0, 64) == 3        # 10, 5, 1 > 0.5
    assert O.choose_rank(R, 0, 0.2, 0, 64) == 2         # 1 > 2 fails
    assert O.choose_rank(-R, 0, 0.05, 0, 64) == 3       # magnitudes, not signed values
    Rt = _r_with_diag([8.0, 4.0, 2.0, 1.0])
    assert O.choose_rank(Rt, 0, 0.25, 0, 64) == 2       # 2 == 0.25 * 8 is not kept (strict)
    assert O.choose_rank(Rt, 0, 0.25 - 2 ** -20, 0, 64) == 3
    Rn = _r_with_diag([8.0, 1.0, 4.0, 4.0])
    assert O.choose_rank(Rn, 0, 0.25, 0, 64) == 1       # stops at the first failing pivot
    assert O.choose_rank(R, 0, 1e-12, 0, 64) == 6       # every pivot kept
    assert O.choose_rank(R, 0, 1e-12, 4, 64) == 4       # cap
    assert O.choose_rank(R, 0, 1e-12, 0, 5) == 5        # never above the block size
    assert O.choose_rank(R, 0, 0.99, 0, 64) == 1        # at least one column
    assert O.choose_rank(np.zeros((4, 6)), 0, 0.1, 0, 64) == 1
    assert O.choose_rank(R, 4, 0.5, 2, 64) == 4         # a fixed rank ignores tol and cap
    assert O.choose_rank(R, 9, 0.0, 0, 64) == 6         # ... but not the columns there are


# --------------------------------------------------------------------------
# tree (brute force on tiny inputs)
# --------------------------------------------------------------------------


def test_tree_bisection_brute_force():
    X = synth.points_uniform(50, 3, 7)
    t = O.build_tree(X, 4)
    assert t.levels == math.ceil(math.log2(50 / 4))
    assert sorted(t.perm.tolist()) == list(range(50))
    for l in range(t.levels):
        for i, (lo, hi) in enumerate(t.ranges[l]):
            (a1, b1), (a2, b2) = t.ranges[l + 1][2 * i], t.ranges[l + 1][2 * i + 1]
            assert a1 == lo and b2 == hi and b1 == a2
            assert b1 - a1 == (hi - lo + 1) // 2
            P = X[t.perm[lo:hi]]
            axis = int(np.argmax(P.max(0) - P.min(0)))
            left = X[t.perm[a1:b1], axis]
            right = X[t.perm[a2:b2], axis]
            assert left.max() <= right.min()
    # leaves: the last split's order holds inside each leaf
    for lo, hi in t.ranges[t.levels]:
        assert hi - lo <= 4


def test_tree_levels_small_n():
    assert O.num_levels(100, 128) == 0
    assert O.num_levels(2048, 128) == 4
    assert O.num_levels(262144, 256) == 10
    assert O.num_levels(5000, 128) == 6


# --------------------------------------------------------------------------
# QRCP (Eq. 2) vs LAPACK's pivoted QR on generic input
# --------------------------------------------------------------------------


def test_qrcp_matches_lapack_pivots_and_r():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((40, 30)) @ np.diag(np.logspace(0, -6, 30))
    Q, R, piv = O.qrcp(B, 30)
    Ql, Rl, pl = sla.qr(B, pivoting=True, mode="economic")
    assert piv.tolist() == pl.tolist()
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-10)
    np.testing.assert_allclose(Q @ R, B[:, piv], atol=1e-13)
    assert np.all(np.diag(R) >= 0)
    np.testing.assert_allclose(Q.T @ Q, np.eye(30), atol=1e-14)


def test_qrcp_pivot_is_max_residual_norm():
    rng = np.random.default_rng(9)
    B = rng.standard_normal((12, 9))
    Q, R, piv = O.qrcp(B, 9)
    for j in range(9):
        # residual of B[:, piv[j:]] after projecting out Q[:, :j]
        Res = B[:, piv] - Q[:, :j] @ (Q[:, :j].T @ B[:, piv])
        norms = np.linalg.norm(Res[:, j:], axis=0)
        assert abs(R[j, j] - norms.max()) < 1e-12
        assert int(np.argmax(norms)) == 0


# --------------------------------------------------------------------------
# P1: factor + solve + logdet equal dense Cholesky of the densified matrix
# --------------------------------------------------------------------------


def test_cfg1_plain_is_spd_and_solve_matches_dense(cfg1):
    At = O.densify(cfg1["h"])
    assert np.allclose(At, At.T, atol=1e-14)
    c = sla.cho_factor(At, lower=True)
    x_dense = sla.cho_solve(c, cfg1["b"])
    x = O.ulv_solve(cfg1["h"], cfg1["F"], cfg1["b"])
    assert np.linalg.norm(x - x_dense) / np.linalg.norm(x_dense) < 1e-11
    ld_dense = 2 * np.sum(np.log(np.diag(c[0])))
    assert abs(cfg1["F"].logdet - ld_dense) <= 1e-12 * abs(ld_dense)


def test_random_hss_solve_and_logdet_match_dense():
    d = synth.random_hss(3, 24, 6, seed=11)
    h = hss_from_dict(d)
    At = O.densify(h)
    assert np.linalg.eigvalsh(At)[0] > 0
    F = O.ulv_factor(h)
    b = synth.rhs_normal(h.n, 3, 2)
    x = O.ulv_solve(h, F, b)
    np.testing.assert_allclose(x, np.linalg.solve(At, b), rtol=1e-11, atol=1e-12)
    assert abs(F.logdet - np.linalg.slogdet(At)[1]) < 1e-10


def test_matvec_matches_densified(cfg1):
    h = cfg1["h"]
    At = O.densify(h)
    b = synth.rhs_normal(h.n, 2, 4)
    np.testing.assert_allclose(O.matvec(h, b), At @ b, rtol=1e-12, atol=1e-12)


def test_densify_matches_hand_assembly_one_level():
    # L = 1: A = [[D0, U0 S U1^T], [U1 S^T U0^T, D1]] by Eq. 1
    d = synth.random_hss(1, 10, 3, seed=3)
    h = hss_from_dict(d)
    At = O.densify(h)
    blk = d["U"][0] @ d["S"][0][0] @ d["U"][1].T
    ref = np.block([[d["D"][0], blk], [blk.T, d["D"][1]]])
    np.testing.assert_allclose(At, ref, atol=1e-15)


# --------------------------------------------------------------------------
# P2: closed-form Schur complement and determinant identity per node
# --------------------------------------------------------------------------


def test_schur_complement_closed_form(cfg1):
    h, F = cfg1["h"], cfg1["F"]
    L = h.levels
    for i in range(4):
        M = h.D[i]
        Us = h.U[i]
        closed = np.linalg.inv(Us.T @ np.linalg.solve(M, Us))
        np.testing.assert_allclose(F.Sigma[L][i], closed, rtol=1e-9, atol=1e-12)
        ld_M = np.linalg.slogdet(M)[1]
        ld = 2 * np.sum(np.log(np.diag(F.LRR[L][i]))) + np.linalg.slogdet(F.Sigma[L][i])[1]
        assert abs(ld_M - ld) < 1e-9 * abs(ld_M)


# --------------------------------------------------------------------------
# P3: results do not depend on the choice of the complement U^R
# --------------------------------------------------------------------------


def test_complement_invariance(cfg1):
    rng = np.random.default_rng(17)

    def rotated(Us):
        Ur = O.complement_basis(Us)
        W, _ = np.linalg.qr(rng.standard_normal((Ur.shape[1], Ur.shape[1])))
        return Ur @ W

    F2 = O.ulv_factor(cfg1["h"], complement=rotated)
    x1 = O.ulv_solve(cfg1["h"], cfg1["F"], cfg1["b"])
    x2 = O.ulv_solve(cfg1["h"], F2, cfg1["b"])
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-11
    assert abs(F2.logdet - cfg1["F"].logdet) < 1e-10 * abs(cfg1["F"].logdet)


# --------------------------------------------------------------------------
# P4: orthonormality and the zero structure of Eq. 8
# --------------------------------------------------------------------------


def test_bases_orthonormal_and_full_q(cfg1):
    h, F = cfg1["h"], cfg1["F"]
    for U in h.U:
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-13
    for l in range(1, h.levels):
        for E in h.E[l]:
            assert np.abs(E.T @ E - np.eye(E.shape[1])).max() <= 1e-13
    for l in range(1, h.levels + 1):
        for Q in F.Q[l]:
            assert np.abs(Q.T @ Q - np.eye(Q.shape[0])).max() <= 1e-13


def test_low_rank_blocks_vanish_in_redundant_rows(cfg1):
    # Eq. 8: U^R_i^T A_ij = 0 for every admissible block of the leaf's row.
    h = cfg1["h"]
    At = O.densify(h)
    nrm = np.linalg.norm(At, 2)
    for i, (lo, hi) in enumerate(h.ranges[h.levels]):
        Ur = O.complement_basis(h.U[i])
        row = np.concatenate([At[lo:hi, :lo], At[lo:hi, hi:]], axis=1)
        assert np.abs(Ur.T @ row).max() <= 1e-13 * nrm


# --------------------------------------------------------------------------
# P5: special cases
# --------------------------------------------------------------------------


def test_single_level_zero_is_plain_cholesky():
    X = synth.points_uniform(60, 2, 3)
    kern = O.Kernel("exponential", 0.2, 1e-3)
    t = O.build_tree(X, 64)
    assert t.levels == 0
    A = O.dense_matrix(kern, X[t.perm])
    h = O.construct_plain(X, t, kern, rank=8, A=A)
    F = O.ulv_factor(h)
    np.testing.assert_allclose(F.L0, np.linalg.cholesky(A), atol=1e-14)
    b = synth.rhs_normal(60, 1, 1)[:, 0]
    np.testing.assert_allclose(O.ulv_solve(h, F, b), np.linalg.solve(A, b), rtol=1e-10)


@pytest.mark.parametrize("mode", ["plain", "scaled"])
def test_full_rank_reproduces_dense_matrix(mode):
    X = synth.points_uniform(128, 3, 4)
    kern = O.Kernel("matern32", 0.2, 1e-6)
    t = O.build_tree(X, 16)
    A = O.dense_matrix(kern, X[t.perm])
    if mode == "plain":
        h = O.construct_plain(X, t, kern, rank=1000, A=A)
    else:
        h = O.construct_scaled(X, t, kern, synth.test_matrix(128, 130, 3), rank=1000, A=A)
    np.testing.assert_allclose(O.densify(h), A, atol=1e-12)
    F = O.ulv_factor(h)
    b = synth.rhs_normal(128, 1, 9)[:, 0]
    x = O.ulv_solve(h, F, b)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-10


def test_blr2_ulv_equals_hss_ulv_logdet(cfg1):
    # Alg. 1 (leaf partial factorization + dense Cholesky of all skeleton rows)
    # and Alg. 2 (nested) factor the same matrix.
    assert abs(O.blr2_logdet(cfg1["h"]) - cfg1["F"].logdet) < 1e-10 * abs(cfg1["F"].logdet)


def test_blr2_solve_equals_dense_solve(cfg1):
    # Eq. 14 on the exp2d workload against a dense solve of the matrix the HSS
    # form represents, and against the HSS-ULV solve of Alg. 2 / Eq. 17.
    h, b = cfg1["h"], cfg1["b"]
    A = O.densify(h)
    F2 = O.blr2_factor(h)
    x = O.blr2_solve(h, F2, b)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    xh = O.ulv_solve(h, cfg1["F"], b)
    assert np.linalg.norm(x - xh) / np.linalg.norm(xh) < 1e-10
    sign, ld = np.linalg.slogdet(A)
    assert sign > 0 and abs(F2.logdet - ld) < 1e-10 * abs(ld)


@pytest.mark.parametrize("levels,leaf,rank", [(1, 16, 5), (3, 24, 7), (4, 12, 12)])
def test_blr2_on_random_hss(levels, leaf, rank):
    # random HSS matrices (rank = leaf: uncompressed leaves, m = 0), several
    # right-hand sides; the skeleton matrix has sum(leaf ranks) rows
    h = hss_from_dict(synth.random_hss(levels, leaf, rank, seed=40 + levels))
    A = O.densify(h)
    F2 = O.blr2_factor(h)
    assert F2.Lss.shape == (rank * 2 ** levels,) * 2
    B = synth.rhs_normal(h.n, 3, 41)
    X = O.blr2_solve(h, F2, B)
    assert np.linalg.norm(A @ X - B) / np.linalg.norm(B) < 1e-12
    sign, ld = np.linalg.slogdet(A)
    assert sign > 0 and abs(F2.logdet - ld) < 1e-11 * max(1.0, abs(ld))


def test_blr2_skeleton_matrix_is_the_schur_complement():
    # The skeleton matrix equals the Schur complement of the redundant rows in
    # Q^T A Q (Q = blkdiag of the leaves' [U^R U^S]), formed here densely: a
    # dropped or transposed coupling, or a wrong leaf offset, breaks it.
    h = hss_from_dict(synth.random_hss(3, 20, 6, seed=47))
    A = O.densify(h)
    Ass, offs, Qs, _, _, _ = O.blr2_skeleton_matrix(h)
    Q = sla.block_diag(*Qs)
    Ah = Q.T @ A @ Q
    ms = [q.shape[1] - (offs[i + 1] - offs[i]) for i, q in enumerate(Qs)]
    lo = np.cumsum([0] + [q.shape[1] for q in Qs])
    R = np.concatenate([np.arange(lo[i], lo[i] + ms[i]) for i in range(len(Qs))])
    S = np.concatenate([np.arange(lo[i] + ms[i], lo[i + 1]) for i in range(len(Qs))])
    schur = Ah[np.ix_(S, S)] - Ah[np.ix_(S, R)] @ np.linalg.solve(Ah[np.ix_(R, R)], Ah[np.ix_(R, S)])
    assert np.abs(Ass - schur).max() < 1e-11 * np.abs(schur).max()


def test_two_leaf_hand_derivation():
    # L = 1, hand-derived: with Q_i = [U^R_i U_i], the root block is
    # [[Sigma_0, S], [S^T, Sigma_1]] with Sigma_i = (U_i^T D_i^{-1} U_i)^{-1}.
    d = synth.random_hss(1, 8, 3, seed=21)
    h = hss_from_dict(d)
    F = O.ulv_factor(h)
    sig = [np.linalg.inv(d["U"][i].T @ np.linalg.solve(d["D"][i], d["U"][i])) for i in range(2)]
    root = np.block([[sig[0], d["S"][0][0]], [d["S"][0][0].T, sig[1]]])
    np.testing.assert_allclose(F.root_block, root, rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# construction: Eckart-Young bound, SPD of the scaled form, Eq. 18/19
# --------------------------------------------------------------------------


def test_plain_leaf_truncation_respects_eckart_young(cfg1):
    h, A = cfg1["h"], cfg1["A"]
    for i, (lo, hi) in enumerate(h.ranges[h.levels][:4]):
        B = np.concatenate([A[lo:hi, :lo], A[lo:hi, hi:]], axis=1)
        U = h.U[i]
        k = U.shape[1]
        err = np.linalg.norm(B - U @ (U.T @ B), 2)
        s = np.linalg.svd(B, compute_uv=False)
        assert err >= s[k] * (1 - 1e-10)
        # pivoted QR stays within a modest factor of optimal here
        assert err <= 50 * s[k]


def _exact_hss_dense(levels, leaf, rank, seed):
    d = synth.random_hss(levels, leaf, rank, seed=seed)
    h0 = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    return h0, O.densify(h0), O.Tree(np.arange(h0.n), levels, h0.ranges)


@pytest.mark.parametrize("levels,leaf,rank", [(3, 32, 6), (2, 48, 10), (4, 16, 5)])
def test_plain_sampled_recovers_an_exact_hss_matrix(levels, leaf, rank):
    # A matrix that is exactly HSS with rank r: every off-diagonal row block has
    # rank <= r, so r + 8 random samples see its whole range, the pivoted QR keeps
    # it, and the sibling blocks equal their compressed forms; the construction
    # must reproduce the matrix to rounding. A dropped sibling subtraction, S in
    # place of S^T, or the children's bases left out of the projection breaks it.
    h0, A, tree = _exact_hss_dense(levels, leaf, rank, seed=9 + levels)
    h = O.construct_plain_sampled(None, tree, None, synth.test_matrix(h0.n, rank + 8, 3 + levels), rank=rank, A=A)
    assert np.abs(O.densify(h) - A).max() <= 1e-13 * np.abs(A).max()
    assert h.rank[levels] == [rank] * 2 ** levels


def test_plain_sampled_full_rank_is_exact_and_bases_orthonormal():
    # with as many samples as rows and no truncation every basis is square:
    # the HSS form is the matrix itself
    _, A, tree = _exact_hss_dense(3, 24, 4, seed=21)
    rng = np.random.default_rng(2)
    R = rng.standard_normal(A.shape)
    B = A + 0.5 * np.eye(A.shape[0]) + 1e-2 * (R + R.T)  # full-rank off-diagonal blocks
    h = O.construct_plain_sampled(None, tree, None, synth.test_matrix(B.shape[0], B.shape[0], 5), rank=B.shape[0],
                                  A=B)
    assert np.abs(O.densify(h) - B).max() <= 1e-13 * np.abs(B).max()
    for Q in list(h.U) + [e for l in range(1, h.levels) for e in h.E[l]]:
        assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() <= 1e-13


def test_plain_sampled_truncation_near_the_optimum(cfg1):
    # leaf bases from samples: the truncation error of each leaf's off-diagonal
    # row block is at least sigma_{k+1} (Eckart-Young) and, with 8 samples of
    # oversampling on this fast-decaying kernel, within a small factor of it; the
    # whole matrix is about as accurate as the exact-block construction.
    w, tree, kern, A, h_exact = cfg1["w"], cfg1["tree"], cfg1["kern"], cfg1["A"], cfg1["h"]
    h = O.construct_plain_sampled(cfg1["X"], tree, kern, synth.test_matrix(w.n, w.rank + 8, 3001)[tree.perm],
                                  rank=w.rank, A=A)
    L = tree.levels
    for i, (lo, hi) in enumerate(tree.ranges[L]):
        Boff = np.concatenate([A[lo:hi, :lo], A[lo:hi, hi:]], axis=1)
        sv = np.linalg.svd(Boff, compute_uv=False)
        U = h.U[i]
        err = np.linalg.norm(Boff - U @ (U.T @ Boff), 2)
        assert sv[w.rank] * (1 - 1e-10) <= err <= 20 * sv[w.rank]
    e_s = np.linalg.norm(O.densify(h) - A) / np.linalg.norm(A)
    e_x = np.linalg.norm(O.densify(h_exact) - A) / np.linalg.norm(A)
    assert e_s <= 3 * e_x


def test_scaled_construction_spd_where_plain_is_not():
    # Matern-3/2, l = 0.2, nugget 1e-6 in the unit cube: the plain projection
    # loses definiteness at these ranks, the scaled compression keeps it.
    X = synth.points_uniform(1024, 3, 1002)
    kern = O.Kernel("matern32", 0.2, 1e-6)
    t = O.build_tree(X, 64)
    A = O.dense_matrix(kern, X[t.perm])
    hp = O.construct_plain(X, t, kern, rank=16, A=A)
    assert np.linalg.eigvalsh(O.densify(hp))[0] < 0
    with pytest.raises(O.NotSPD):
        O.ulv_factor(hp)
    hs, aux = O.construct_scaled(X, t, kern, synth.test_matrix(1024, 24, 3), rank=16, A=A,
                                 return_aux=True)
    At = O.densify(hs)
    assert np.linalg.eigvalsh(At)[0] > 0
    F = O.ulv_factor(hs)
    # The ULV's leaf Schur complements equal R R^T of the scaled basis QR.
    for i in range(4):
        np.testing.assert_allclose(F.Sigma[t.levels][i], aux["Sigma"][t.levels][i], rtol=1e-8, atol=1e-10)
    b = synth.rhs_normal(1024, 1, 1)[:, 0]
    x = O.ulv_solve(hs, F, b)
    np.testing.assert_allclose(x, np.linalg.solve(At, b), rtol=1e-8)


def test_eq19_solve_error_roundoff(cfg1):
    e = O.solve_error(cfg1["h"], cfg1["F"], cfg1["b"])
    assert e < 1e-12
    e18 = O.construction_error(cfg1["A"] @ cfg1["b"], cfg1["h"], cfg1["b"])
    assert 1e-6 < e18 < 5e-2
