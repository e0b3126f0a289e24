"""Batches of independent HSS systems (one forest, stages by height), HIP-graph
replay and the GEMM tile autotuner.

Each system of a batch is the same HSS matrix as when factored alone, so:
  - FP64: every system's solution and log-determinant meet the single-matrix
    parity gates against the oracle (max(1e-10, 10 kappa u) in x, 1e-10
    relative in log det), and agree with the single-system GPU run to 1e-13;
  - FP32: every system agrees with its single-system FP32 run to 1e-6;
  - the per-system results do not depend on the order of the batch;
  - graph replays reproduce the eager launches exactly (same kernels, same
    arguments), replay after replay, with eager work in between;
  - tuned tile shapes change only rounding (1e-12 against the untuned run).
"""
import numpy as np
import pytest

import synth
from oracle import hss_oracle as O

from gpu_util import oracle_to_dict, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2311_00921_amd import hss

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = hss.hss_ctx_create(0)
    yield torch, hss, ctx
    torch.cuda.synchronize()
    hss.hss_ctx_destroy(ctx)


def _hss(levels, leaf, rank, seed):
    d = synth.random_hss(levels, leaf, rank, seed=seed)
    return O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])


def _systems():
    """Uneven sizes and depths: a single block, shallow and deep trees, ragged leaves."""
    hs = [_hss(3, 64, 16, 11), _hss(1, 32, 8, 12), _hss(4, 48, 12, 13), _hss(2, 256, 96, 14)]
    X = synth.points_uniform(1500, 3, 1002)
    kern = O.Kernel("matern32", 0.2, 1e-6)
    tree = O.build_tree(X, 64)
    hs.append(O.construct_scaled(X, tree, kern, synth.test_matrix(1500, 24, 3)[tree.perm], rank=16))
    X1 = synth.points_uniform(100, 2, 3)
    t1 = O.build_tree(X1, 128)
    hs.append(O.construct_plain(X1, t1, O.Kernel("exponential", 0.2, 1e-3), rank=8))
    return hs


def _stack(torch, bs):
    b = np.concatenate(bs, axis=0)
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()


def _single_run(env, h, b, precision):
    torch, hss, ctx = env
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        hss.hss_ulv_factor(ctx, m, precision)
        x = hss.hss_ulv_solve(ctx, m, torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()).cpu().numpy()
        return x, hss.hss_logdet(ctx, m)
    finally:
        hss.hss_matrix_destroy(m)


def _batch(env, hs):
    torch, hss, ctx = env
    singles = [hss.hss_import(ctx, oracle_to_dict(h)) for h in hs]
    try:
        return hss.hss_batch_create(ctx, singles)
    finally:
        for s in singles:
            hss.hss_matrix_destroy(s)


def test_batch_fp64_matches_oracle_and_single_runs(env):
    torch, hss, ctx = env
    hs = _systems()
    nrhs = 2
    bs = [synth.rhs_normal(h.n, nrhs, 40 + i) for i, h in enumerate(hs)]
    print("batch fp64 sizes", [h.n for h in hs], flush=True)
    m = _batch(env, hs)
    try:
        info = hss.hss_get_info(m)
        assert info.systems == len(hs) and info.n == sum(h.n for h in hs)
        off, _, _ = hss.hss_batch_query(ctx, m, len(hs), factored=False)
        assert list(off) == list(np.cumsum([0] + [h.n for h in hs]))
        hss.hss_ulv_factor(ctx, m)
        bd = _stack(torch, bs)
        x = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
        y = hss.hss_matvec(ctx, m, bd).cpu().numpy()
        _, failed, lds = hss.hss_batch_query(ctx, m, len(hs))
        assert not failed.any()
        assert abs(hss.hss_logdet(ctx, m) - lds.sum()) <= 1e-12 * (np.abs(lds).sum() + 1)
        for k, h in enumerate(hs):
            F = O.ulv_factor(h)
            xk = x[off[k]:off[k + 1]]
            assert rel(xk, O.ulv_solve(h, F, bs[k])) <= 1e-10, k
            assert abs(lds[k] - F.logdet) <= 1e-10 * (abs(F.logdet) + 1.0), k
            assert rel(y[off[k]:off[k + 1]], O.matvec(h, bs[k])) <= 1e-13, k
            xs, lds_single = _single_run(env, h, bs[k], hss.HSS_P_FP64)
            assert rel(xk, xs) <= 1e-13, k
            assert abs(lds[k] - lds_single) <= 1e-12 * (abs(lds_single) + 1.0), k
    finally:
        hss.hss_matrix_destroy(m)


def test_batch_order_invariance(env):
    torch, hss, ctx = env
    hs = _systems()
    bs = [synth.rhs_normal(h.n, 1, 60 + i) for i, h in enumerate(hs)]
    order = list(range(len(hs)))[::-1]
    res = []
    for perm in (list(range(len(hs))), order):
        m = _batch(env, [hs[i] for i in perm])
        try:
            hss.hss_ulv_factor(ctx, m)
            x = hss.hss_ulv_solve(ctx, m, _stack(torch, [bs[i] for i in perm])).cpu().numpy()
            off, _, lds = hss.hss_batch_query(ctx, m, len(hs))
            per = {}
            for j, i in enumerate(perm):
                per[i] = (x[off[j]:off[j + 1]], lds[j])
            res.append(per)
        finally:
            hss.hss_matrix_destroy(m)
    for i in range(len(hs)):
        assert rel(res[0][i][0], res[1][i][0]) <= 1e-13
        assert abs(res[0][i][1] - res[1][i][1]) <= 1e-12 * (abs(res[0][i][1]) + 1.0)


def test_batch_fp32_matches_single_fp32_runs(env):
    torch, hss, ctx = env
    hs = [_hss(3, 64, 16, 21), _hss(2, 128, 32, 22), _hss(4, 32, 8, 23), _systems()[-1]]
    bs = [synth.rhs_normal(h.n, 1, 80 + i) for i, h in enumerate(hs)]
    m = _batch(env, hs)
    try:
        hss.hss_ulv_factor(ctx, m, hss.HSS_P_FP32)
        x = hss.hss_ulv_solve(ctx, m, _stack(torch, bs)).cpu().numpy()
        off, failed, lds = hss.hss_batch_query(ctx, m, len(hs))
        assert not failed.any()
        for k, h in enumerate(hs):
            xs, ls = _single_run(env, h, bs[k], hss.HSS_P_FP32)
            assert rel(x[off[k]:off[k + 1]], xs) <= 1e-6, k
            assert abs(lds[k] - ls) <= 1e-6 * (abs(ls) + 1.0), k
        # refinement with the FP64 batch matvec reaches FP64 accuracy for every system
        xr, iters, rr, ok = hss.hss_ulv_solve_refined(ctx, m, _stack(torch, bs), 1e-12, 50)
        assert ok and rr <= 1e-12
        xr = xr.cpu().numpy()
        for k, h in enumerate(hs):
            F = O.ulv_factor(h)
            assert rel(xr[off[k]:off[k + 1]], O.ulv_solve(h, F, bs[k])) <= 1e-10, k
    finally:
        hss.hss_matrix_destroy(m)


def test_batch_reports_failing_system(env):
    torch, hss, ctx = env
    X = synth.points_uniform(1024, 3, 1002)
    t = O.build_tree(X, 64)
    bad = O.construct_plain(X, t, O.Kernel("matern32", 0.2, 1e-6), rank=16)  # indefinite (PLAIN)
    hs = [_hss(2, 64, 16, 31), bad, _hss(3, 32, 8, 32)]
    m = _batch(env, hs)
    try:
        with pytest.raises(hss.HSSError) as e:
            hss.hss_ulv_factor(ctx, m)
        assert e.value.status == hss.HSS_ERR_NOT_SPD
        info = hss.hss_get_info(m)
        assert info.failed_system == 1
        _, failed, _ = hss.hss_batch_query(ctx, m, 3)
        assert list(failed) == [0, 1, 0]
    finally:
        hss.hss_matrix_destroy(m)


def test_graph_replay_matches_eager(env):
    torch, hss, ctx = env
    hs = _systems()
    bs = [synth.rhs_normal(h.n, 1, 90 + i) for i, h in enumerate(hs)]
    bd = torch.from_numpy(np.concatenate(bs, axis=0)[:, 0].copy()).cuda()  # 1-D: the same buffer every call
    for prec in (hss.HSS_P_FP64, hss.HSS_P_FP32):
        print("graph replay precision", prec, flush=True)
        m = _batch(env, hs)
        try:
            hss.hss_ulv_factor(ctx, m, prec)
            x_eager = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
            ld_eager = hss.hss_logdet(ctx, m)
            hss.hss_use_graphs(ctx, m, True)
            xg = torch.empty_like(bd)
            for rep in range(3):
                hss.hss_ulv_factor(ctx, m, prec)          # rep 0 records, later reps replay
                hss.hss_ulv_solve(ctx, m, bd, xg)
                torch.cuda.synchronize()
                junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
                torch.cuda.synchronize()
                assert np.array_equal(xg.cpu().numpy(), x_eager), rep
                assert hss.hss_logdet(ctx, m) == ld_eager, rep
                del junk
            # refined solves go through the recorded solve as well
            xr, iters, rr, ok = hss.hss_ulv_solve_refined(ctx, m, bd, 1e-12, 50)
            assert ok and rr <= 1e-12
        finally:
            hss.hss_matrix_destroy(m)


def test_autotune_changes_only_rounding(env):
    torch, hss, ctx = env
    hs = [_hss(3, 256, 64, 41), _hss(2, 128, 32, 42), _hss(3, 64, 16, 43)]
    bs = [synth.rhs_normal(h.n, 1, 100 + i) for i, h in enumerate(hs)]
    bd = _stack(torch, bs)
    m = _batch(env, hs)
    try:
        hss.hss_ulv_factor(ctx, m)
        x0 = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
        rep = hss.hss_autotune(ctx, m, hss.HSS_P_FP64, 2)
        nt = len(hss.GEMM_TILES)
        assert len(rep) == nt + 1 and all(v > 0 for v in rep)
        assert rep[-1] <= min(rep[:-1]) * 1.05 + 1e-3  # the per-batch choice is no worse than any uniform shape
        var = hss.hss_gemm_variants(m, hss.HSS_P_FP64)
        assert len(var) > 0 and all(0 <= v < nt for v in var)
        with pytest.raises(hss.HSSError):
            hss.hss_ulv_solve(ctx, m, bd)  # tuning leaves the matrix unfactored
        hss.hss_ulv_factor(ctx, m)
        x1 = hss.hss_ulv_solve(ctx, m, bd).cpu().numpy()
        assert rel(x1, x0) <= 1e-12
    finally:
        hss.hss_matrix_destroy(m)


def test_construct_batched_equals_single_constructs(env):
    torch, hss, ctx = env
    specs = [(2000, 0.1, 64), (3000, 0.25, 128), (700, 0.05, 64)]
    pts, oms = [], []
    for i, (n, l, leaf) in enumerate(specs):
        pts.append(torch.from_numpy(synth.points_uniform(n, 3, 1000 + i)).cuda())
        oms.append(torch.from_numpy(synth.test_matrix(n, 40, 3000 + i)).cuda())
    kw = dict(kernels=["gaussian"] * 3, leafs=[s[2] for s in specs], tols=[1e-6] * 3, max_ranks=[32] * 3,
              omegas=oms, lengths=[s[1] for s in specs], nuggets=[1e-5] * 3)
    m = hss.hss_construct_batched(ctx, pts, **kw)
    bs = [synth.rhs_normal(n, 1, 120 + i) for i, (n, _, _) in enumerate(specs)]
    try:
        hss.hss_ulv_factor(ctx, m)
        x = hss.hss_ulv_solve(ctx, m, _stack(torch, bs)).cpu().numpy()
        off, _, lds = hss.hss_batch_query(ctx, m, 3)
        for k, (n, l, leaf) in enumerate(specs):
            s = hss.hss_construct(ctx, pts[k], "gaussian", leaf, tol=1e-6, max_rank=32, omega=oms[k], length=l,
                                  nugget=1e-5)
            try:
                hss.hss_ulv_factor(ctx, s)
                bk = torch.from_numpy(np.ascontiguousarray(bs[k].T)).cuda().t()
                xs = hss.hss_ulv_solve(ctx, s, bk).cpu().numpy()
                assert rel(x[off[k]:off[k + 1]], xs) <= 1e-13, k
                assert abs(lds[k] - hss.hss_logdet(ctx, s)) <= 1e-12 * (abs(lds[k]) + 1.0), k
            finally:
                hss.hss_matrix_destroy(s)
    finally:
        hss.hss_matrix_destroy(m)
