"""Mixed precision (hss_precision FP32, BF16, BF16X3): the leaf stage's four
contractions of the diagonal product on FP32 or BF16 matrix cores, every pivot,
Cholesky, triangular solve, Schur complement, the basis QR and the upper stages
in FP64, leaves whose FP64 pivots fail or fall under the accuracy guard after
the low-precision products redone in FP64; refinement by the FP64 HSS matvec
(classical, then PCG when the residual stalls).

The refined solution meets the requested relative residual against the same
HSS matrix and agrees with the oracle's FP64 solve to about kappa times that
residual. The unrefined mixed solve and log-determinant are compared with the
FP64 oracle with the errors stated in the assertions (the rounding of the leaf
products perturbs each leaf block by about u * |D|, u = 2^-24, 2^-8 and about
2^-16 for FP32, BF16 and the split BF16 products)."""
import numpy as np
import pytest

import synth
from oracle import hss_oracle as O

from gpu_util import maxrel, oracle_to_dict, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2311_00921_amd import hss

    assert torch.cuda.is_available()
    ctx = hss.hss_ctx_create(0)
    yield torch, hss, ctx
    torch.cuda.synchronize()
    hss.hss_ctx_destroy(ctx)


def _dev_rhs(torch, b):
    if b.shape[1] == 1:
        return torch.from_numpy(b[:, 0].copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()


def run_mixed(env, h, tol, nrhs=1, seed=3, prec=None):
    """Mixed factorization + unrefined solve + refined solve of the oracle HSS
    matrix h, beside the oracle's FP64 factorization."""
    torch, hss, ctx = env
    prec = hss.HSS_P_FP32 if prec is None else prec
    print(f"mixed precision {prec} n={h.n} levels={h.levels} tol={tol} nrhs={nrhs}", flush=True)
    F = O.ulv_factor(h)
    b = synth.rhs_normal(h.n, nrhs, seed)
    x_or = O.ulv_solve(h, F, b)
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        hss.hss_ulv_factor(ctx, m, prec)
        promoted = int(hss.hss_get_info(m).promoted_nodes)
        bd = _dev_rhs(torch, b)
        x0 = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy().reshape(h.n, nrhs)
        ld32 = hss.hss_logdet(ctx, m)
        x, iters, rr, ok = hss.hss_ulv_solve_refined(ctx, m, bd, tol, 100)
        x = x.cpu().numpy().reshape(h.n, nrhs)
        print(f"  promoted {promoted} unrefined err {rel(x0, x_or):.2e} logdet err "
              f"{abs(ld32 - F.logdet) / abs(F.logdet):.2e} corrections {iters} relres {rr:.2e}", flush=True)
        return dict(F=F, b=b, x_or=x_or, x0=x0, x=x, iters=iters, rr=rr, ok=ok, ld32=ld32, promoted=promoted)
    finally:
        hss.hss_matrix_destroy(m)


def test_mixed_random_hss_refines_to_roundoff(env):
    d = synth.random_hss(3, 128, 32, seed=4)
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    r = run_mixed(env, h, 1e-12, nrhs=2)
    assert rel(r["x0"], r["x_or"]) < 1e-5          # FP32 leaf products, kappa ~ 3
    assert abs(r["ld32"] - r["F"].logdet) < 1e-5 * abs(r["F"].logdet)
    assert r["ok"] and r["rr"] <= 1e-12 and r["iters"] <= 6
    assert rel(r["x"], r["x_or"]) < 1e-11
    assert maxrel(r["x"], r["x_or"]) < 1e-11


def test_bf16_precisions_on_diagonally_dominant_leaves(env):
    # Leaves D = G G^T / 128 + 12.8 I: eigenvalues in [12.8, 16.8] and
    # |D|_inf at most 26, so every redundant pivot (>= 12.8) passes the BF16 guard
    # (2^-2 |D|_inf) and the split-BF16 one: no leaf is redone in FP64, and the
    # unrefined errors order as the products' unit roundoffs (FP32 2^-24, split
    # BF16 about 2^-16, BF16 2^-8), which shows each precision ran its own
    # products. Refinement reaches 1e-12 from each.
    torch, hss, ctx = env
    d = synth.random_hss(3, 128, 32, seed=4, margin=11.0)
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    err = {}
    for prec in (hss.HSS_P_FP32, hss.HSS_P_BF16X3, hss.HSS_P_BF16):
        r = run_mixed(env, h, 1e-12, nrhs=2, prec=prec)
        assert r["promoted"] == 0
        err[prec] = rel(r["x0"], r["x_or"])
        assert r["ok"] and r["rr"] <= 1e-12, (prec, r["iters"], r["rr"])
        assert rel(r["x"], r["x_or"]) < 1e-11 and maxrel(r["x"], r["x_or"]) < 1e-11
        lderr = abs(r["ld32"] - r["F"].logdet) / abs(r["F"].logdet)
        assert lderr < {hss.HSS_P_FP32: 1e-6, hss.HSS_P_BF16X3: 1e-4, hss.HSS_P_BF16: 1e-2}[prec]
    assert err[hss.HSS_P_FP32] < 1e-5
    assert 2e-4 > err[hss.HSS_P_BF16X3] > 10 * err[hss.HSS_P_FP32]
    assert 0.1 > err[hss.HSS_P_BF16] > 10 * err[hss.HSS_P_BF16X3]


def test_bf16_guard_redoes_smooth_kernel_leaves(env):
    # The benchmark's leaf shape and density (leaf 256, rank 96, Matern-3/2
    # nugget 1e-6): redundant pivots near 1e-5 against |D|_inf near 240, far
    # under both BF16 guards, so every leaf is redone in FP64 and the result is
    # the FP64 factorization bit for bit; the next factorization in the same
    # precision skips the BF16 products (still reported as redone leaves).
    torch, hss, ctx = env
    X = synth.points_uniform(4096, 3, 1011) * 0.25
    kern = O.Kernel("matern32", 0.2, 1e-6)
    tree = O.build_tree(X, 256)
    h = O.construct_scaled(X, tree, kern, synth.test_matrix(4096, 104, 3011)[tree.perm], rank=96)
    b = synth.rhs_normal(h.n, 1, 5)
    bd = torch.from_numpy(b[:, 0].copy()).cuda()
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP64)
        x64 = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
        ld64 = hss.hss_logdet(ctx, m)
        for prec in (hss.HSS_P_BF16, hss.HSS_P_BF16X3):
            for call in range(2):
                hss.hss_ulv_factor(ctx, m, prec)
                info = hss.hss_get_info(m)
                print(f"precision {prec} call {call}: promoted {info.promoted_nodes} of 16", flush=True)
                assert info.factored == 1 and info.precision == prec and info.promoted_nodes == 16
                assert np.array_equal(hss.hss_ulv_solve(ctx, m, bd).cpu().numpy(), x64)
                assert hss.hss_logdet(ctx, m) == ld64
    finally:
        hss.hss_matrix_destroy(m)


def test_mixed_exp2d_refines_to_1e10(env):
    w = synth.WORKLOADS["exp2d_n2048"]
    X = w.points()
    kern = O.Kernel("exponential", w.length, w.nugget)
    tree = O.build_tree(X, w.leaf)
    h = O.construct_plain(X, tree, kern, rank=w.rank)
    r = run_mixed(env, h, 1e-10)
    assert r["ok"] and r["rr"] <= 1e-10
    # kappa ~ 3e4: forward error within kappa * residual
    assert rel(r["x"], r["x_or"]) < 3e4 * 1e-10 * 10
    assert abs(r["ld32"] - r["F"].logdet) < 1e-4 * abs(r["F"].logdet)


def test_mixed_matern3d_scaled_refines_to_1e8(env):
    X = synth.points_uniform(4096, 3, 1003)
    kern = O.Kernel("matern32", 0.2, 1e-6)
    tree = O.build_tree(X, 256)
    h = O.construct_scaled(X, tree, kern, synth.test_matrix(4096, 72, 3003)[tree.perm], rank=64)
    r = run_mixed(env, h, 1e-8)
    assert r["ok"] and r["rr"] <= 1e-8
    res = r["b"] - O.matvec(h, r["x"])
    assert np.linalg.norm(res) / np.linalg.norm(r["b"]) <= 1.01e-8


def test_mixed_leaf256_rank96_at_benchmark_density(env):
    # The leaf shape of the N = 262144 benchmark (leaf 256, rank 96, m = 160:
    # the R-block Cholesky and S-row kernels) at its point density: 4096 points
    # uniform in a cube of side 1/4 (262144 points per unit volume), Matern-3/2
    # l = 0.2, nugget 1e-6, scaled construction.
    X = synth.points_uniform(4096, 3, 1011) * 0.25
    kern = O.Kernel("matern32", 0.2, 1e-6)
    tree = O.build_tree(X, 256)
    h = O.construct_scaled(X, tree, kern, synth.test_matrix(4096, 104, 3011)[tree.perm], rank=96)
    assert all(u.shape == (256, 96) for u in h.U)
    r = run_mixed(env, h, 1e-8)
    # the unrefined solve carries the leaf perturbation (about u32 |D| against
    # leaf R blocks whose smallest eigenvalues are ~1e-5): stated, loosely bounded
    assert rel(r["x0"], r["x_or"]) < 1.0
    assert abs(r["ld32"] - r["F"].logdet) < 1e-3 * abs(r["F"].logdet)
    assert r["ok"] and r["rr"] <= 1e-8
    res = r["b"] - O.matvec(h, r["x"])
    assert np.linalg.norm(res) / np.linalg.norm(r["b"]) <= 1.01e-8


def test_mixed_promotes_failed_leaves_to_fp64(env):
    # Gaussian kernel with nugget 1e-8: the leaf blocks have eigenvalues near
    # 1e-8, far below the FP32 rounding of the leaf products (~1e-5), so the
    # FP64 pivots after the FP32 products fail; the library redoes those leaves
    # in FP64. Where every leaf is redone the factorization is the FP64 one, bit
    # for bit. 16 leaves: the node-by-node path; 128 leaves: the whole-stage path.
    # The matrix is too ill-conditioned for a residual of 1e-10 even in FP64, so
    # refinement is asked for a few times the FP64 solve's own residual.
    torch, hss, ctx = env
    for n, leaf, rank in ((2048, 128, 24), (4096, 32, 8)):
        X = synth.points_uniform(n, 2, 1020 + leaf)
        kern = O.Kernel("gaussian", 0.3, 1e-8)
        tree = O.build_tree(X, leaf)
        h = O.construct_scaled(X, tree, kern, synth.test_matrix(n, rank + 8, 3020 + leaf)[tree.perm], rank=rank)
        b = synth.rhs_normal(n, 1, 7)
        bd = torch.from_numpy(b[:, 0].copy()).cuda()
        m = hss.hss_import(ctx, oracle_to_dict(h))
        try:
            hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP64)
            x64d = hss.hss_ulv_solve(ctx, m, bd)
            rr64 = float(torch.linalg.norm(bd - hss.hss_matvec(ctx, m, x64d)) / torch.linalg.norm(bd))
            x64 = x64d.cpu().numpy()
            ld64 = hss.hss_logdet(ctx, m)
            hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
            info = hss.hss_get_info(m)
            print(f"n={n} leaf={leaf}: promoted {info.promoted_nodes} of {2 ** h.levels} leaves, "
                  f"FP64 relres {rr64:.2e}", flush=True)
            assert info.factored == 1 and info.precision == hss.HSS_P_FP32
            assert info.promoted_nodes >= 1
            x32 = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
            ld32 = hss.hss_logdet(ctx, m)
            if info.promoted_nodes == 2 ** h.levels:
                assert np.array_equal(x32, x64) and ld32 == ld64
            xr, iters, rr, ok = hss.hss_ulv_solve_refined(ctx, m, bd, max(4.0 * rr64, 1e-12), 100)
            assert ok, (iters, rr, rr64)
        finally:
            hss.hss_matrix_destroy(m)
