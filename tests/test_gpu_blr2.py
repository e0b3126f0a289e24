"""GPU parity of the BLR^2-ULV (Alg. 1, Eq. 13-14) against the CPU oracle's
blr2_factor / blr2_solve on the same imported HSS matrices, and against the
GPU's own HSS-ULV on the same matrix (two exact factorizations of one matrix).

Tolerances as for the HSS-ULV: both sides are backward-stable FP64 solvers of
one system, so solutions agree to about kappa * u (gate 1e-10 relative,
normwise and elementwise) and log-determinants to 1e-10 * (|logdet| + 1).
Shapes cover a skeleton order below one 64-row panel, ragged last panels,
leaves on each partial-Cholesky path (m <= 96, m = 160, rank above 128) and
more right-hand sides than one pass of the skeleton solve carries (16).
"""
import numpy as np
import pytest

import synth
from oracle import hss_oracle as O

from gpu_util import maxrel, oracle_to_dict, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_2311_00921_amd import hss

    c = hss.hss_ctx_create(0)
    yield c
    torch_dev.cuda.synchronize()
    hss.hss_ctx_destroy(c)


def _dev(torch, b):
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()


def blr2_compare(ctx, torch, h, nrhs=1, seed=7, xtol=1e-10):
    from paper_2311_00921_amd import hss

    F2 = O.blr2_factor(h)
    print(f"case n={h.n} levels={h.levels} K={F2.Lss.shape[0]} nrhs={nrhs}", flush=True)
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        K, _ = hss.hss_blr2_stats(m)
        assert K == F2.Lss.shape[0]
        hss.hss_blr2_factor(ctx, m)
        b = synth.rhs_normal(h.n, nrhs, seed)
        x_or = O.blr2_solve(h, F2, b)
        x = hss.hss_blr2_solve(ctx, m, _dev(torch, b)).cpu().numpy()
        assert rel(x, x_or) <= xtol, rel(x, x_or)
        assert maxrel(x, x_or) <= xtol, maxrel(x, x_or)
        ld = hss.hss_blr2_logdet(ctx, m)
        assert abs(ld - F2.logdet) <= 1e-10 * (abs(F2.logdet) + 1.0), (ld, F2.logdet)
        _, ms = hss.hss_blr2_stats(m)
        assert ms > 0.0
        return x, x_or
    finally:
        hss.hss_matrix_destroy(m)


def test_exp2d_n2048_plain(ctx, torch_dev):
    # 16 leaves of rank 32: K = 512, eight panels; against the dense solve too
    w = synth.WORKLOADS["exp2d_n2048"]
    X = w.points()
    kern = O.Kernel("exponential", w.length, w.nugget)
    tree = O.build_tree(X, w.leaf)
    h = O.construct_plain(X, tree, kern, rank=w.rank, A=O.dense_matrix(kern, X[tree.perm]))
    x, _ = blr2_compare(ctx, torch_dev, h)
    b = synth.rhs_normal(h.n, 1, 7)
    assert np.linalg.norm(O.densify(h) @ x - b) / np.linalg.norm(b) < 1e-11


@pytest.mark.parametrize("levels,leaf,rank,nrhs", [
    (3, 24, 7, 1),      # K = 56: one partial panel
    (5, 32, 13, 3),     # K = 416: ragged last panel
    (4, 64, 40, 17),    # K = 640, 17 right-hand sides: two skeleton-solve passes, a ragged leaf pass
    (5, 64, 37, 5),     # K = 1184: four-panel outer blocks whose trailing update is split between
                        # the next block and the rest (three rests), a partial last block and panel
    (2, 256, 96, 2),    # the benchmark's leaf shape (m = 160)
    (2, 512, 200, 1),   # rank above 128
    (1, 40, 40, 2),     # uncompressed leaves (m = 0): the skeleton matrix is the whole matrix
])
def test_random_hss_shapes(ctx, torch_dev, levels, leaf, rank, nrhs):
    d = synth.random_hss(levels, leaf, rank, seed=300 + levels * 10 + rank)
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    blr2_compare(ctx, torch_dev, h, nrhs=nrhs)


def test_ragged_tree_scaled_matern(ctx, torch_dev):
    # leaves of 46-47 points (N = 1500, leaf 64), scaled construction
    X = synth.points_uniform(1500, 3, 1002)
    kern = O.Kernel("matern32", 0.2, 1e-6)
    tree = O.build_tree(X, 64)
    h = O.construct_scaled(X, tree, kern, synth.test_matrix(1500, 24, 3)[tree.perm], rank=16)
    blr2_compare(ctx, torch_dev, h, nrhs=2, xtol=1e-9)


def test_blr2_equals_hss_ulv_on_a_constructed_matrix(ctx, torch_dev):
    # Matern-3/2, N = 16384, leaf 256, rank 64, built on the GPU: K = 4096.
    # Both factorizations of the same matrix on the GPU, and the residual by
    # the FP64 HSS matvec.
    from paper_2311_00921_amd import hss

    torch = torch_dev
    n, leaf, r = 16384, 256, 64
    X = torch.from_numpy(synth.points_uniform(n, 3, 1002)).cuda()
    Om = _dev(torch, synth.test_matrix(n, r + 8, 3))
    m = hss.hss_construct(ctx, X, "matern32", leaf, rank=r, omega=Om, length=0.2, nugget=1e-6)
    try:
        b = _dev(torch, synth.rhs_normal(n, 2, 11))
        hss.hss_ulv_factor(ctx, m)
        x_h = hss.hss_ulv_solve(ctx, m, b).cpu().numpy()
        ld_h = hss.hss_logdet(ctx, m)
        hss.hss_blr2_factor(ctx, m)
        assert hss.hss_blr2_stats(m)[0] == (n // leaf) * r
        xb = hss.hss_blr2_solve(ctx, m, b)
        x_b = xb.cpu().numpy()
        ld_b = hss.hss_blr2_logdet(ctx, m)
        print(f"hss vs blr2: x {rel(x_b, x_h):.2e} logdet {abs(ld_b - ld_h):.2e}", flush=True)
        assert rel(x_b, x_h) <= 1e-9 and maxrel(x_b, x_h) <= 1e-9
        assert abs(ld_b - ld_h) <= 1e-10 * (abs(ld_h) + 1.0)
        res = (b - hss.hss_matvec(ctx, m, xb)).cpu().numpy()
        assert np.linalg.norm(res) / np.linalg.norm(b.cpu().numpy()) <= 1e-8
    finally:
        hss.hss_matrix_destroy(m)


def test_factorizations_leave_each_other_stale(ctx, torch_dev):
    from paper_2311_00921_amd import hss

    d = synth.random_hss(2, 32, 8, seed=5)
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        b = _dev(torch_dev, synth.rhs_normal(h.n, 1, 3))
        with pytest.raises(RuntimeError, match="BLR"):
            hss.hss_blr2_solve(ctx, m, b)
        hss.hss_blr2_factor(ctx, m)
        with pytest.raises(RuntimeError, match="not factored"):
            hss.hss_ulv_solve(ctx, m, b)
        hss.hss_ulv_factor(ctx, m)
        with pytest.raises(RuntimeError, match="BLR"):
            hss.hss_blr2_solve(ctx, m, b)
        x_h = hss.hss_ulv_solve(ctx, m, b).cpu().numpy()
        hss.hss_blr2_factor(ctx, m)
        x_b = hss.hss_blr2_solve(ctx, m, b).cpu().numpy()
        assert rel(x_b, x_h) <= 1e-10
    finally:
        hss.hss_matrix_destroy(m)


def test_indefinite_skeleton_is_reported(ctx, torch_dev):
    # couplings scaled up: every leaf block stays SPD (its partial Cholesky
    # passes), the skeleton matrix does not; the oracle fails the same way
    from paper_2311_00921_amd import hss

    d = synth.random_hss(3, 24, 7, seed=5)
    d["S"] = [[50.0 * s for s in lev] for lev in d["S"]]
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    with pytest.raises(O.NotSPD):
        O.blr2_factor(h)
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        with pytest.raises(RuntimeError, match="skeleton"):
            hss.hss_blr2_factor(ctx, m)
        with pytest.raises(RuntimeError, match="BLR"):
            hss.hss_blr2_solve(ctx, m, _dev(torch_dev, synth.rhs_normal(h.n, 1, 3)))
    finally:
        hss.hss_matrix_destroy(m)
