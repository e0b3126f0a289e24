"""The no-allocation solve (hss_ulv_solve_noalloc) through the C ABI: the same
results as hss_ulv_solve, bit for bit (the same kernels on a workspace in a
static device array), on two calls in a row -- a larger system with three
right-hand sides, then a smaller one with one -- plus the rejection of a
request beyond the static array and of a solve before factorization. Both
solves are also checked against the oracle's FP64 solve (1e-10, the parity
gate of the ULV tests)."""
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


def _colmajor(torch, b):
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()


def test_noalloc_solve_equals_solve_twice(env):
    torch, hss, ctx = env
    cases = [(3, 256, 64, 3, 11), (2, 128, 24, 1, 12)]  # (levels, leaf, rank, nrhs, seed): second is smaller
    for levels, leaf, rank, nrhs, seed in cases:
        d = synth.random_hss(levels, leaf, rank, seed=seed)
        h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
        print(f"noalloc case n={h.n} levels={levels} nrhs={nrhs}", flush=True)
        F = O.ulv_factor(h)
        b = synth.rhs_normal(h.n, nrhs, seed + 100)
        x_or = O.ulv_solve(h, F, b)
        m = hss.hss_import(ctx, oracle_to_dict(h))
        try:
            bd = _colmajor(torch, b)
            xa = torch.full_like(bd, float("nan"))
            with pytest.raises(hss.HSSError) as e:
                hss.hss_ulv_solve_noalloc(ctx, m, bd, xa)
            assert e.value.status == hss.HSS_ERR_BAD_STATE
            hss.hss_ulv_factor(ctx, m)
            hss.hss_ulv_solve_noalloc(ctx, m, bd, xa)
            xs = hss.hss_ulv_solve(ctx, m, bd)
            torch.cuda.synchronize()
            xa_h, xs_h = xa.cpu().numpy(), xs.cpu().numpy()
            assert np.array_equal(xa_h, xs_h)
            assert rel(xa_h, x_or) <= 1e-10 and maxrel(xa_h, x_or) <= 1e-10
        finally:
            hss.hss_matrix_destroy(m)


def test_noalloc_solve_rejects_beyond_scratch(env):
    torch, hss, ctx = env
    d = synth.random_hss(4, 256, 96, seed=5)
    h = O.HSS(d["n"], d["levels"], d["ranges"], d["rank"], d["D"], d["U"], d["E"], d["S"])
    m = hss.hss_import(ctx, oracle_to_dict(h))
    try:
        hss.hss_ulv_factor(ctx, m)
        sum_n = h.n + (2 ** 4 - 1) * 2 * 96  # the leaves, plus each non-leaf node's block of its children's ranks
        too_many = (1 << 22) // sum_n + 1
        b = torch.zeros((too_many, h.n), dtype=torch.float64, device="cuda").t()
        x = torch.empty_like(b)
        with pytest.raises(hss.HSSError) as e:
            hss.hss_ulv_solve_noalloc(ctx, m, b, x)
        assert e.value.status == hss.HSS_ERR_UNSUPPORTED
        assert "static scratch" in str(e.value)
        ok = (1 << 22) // sum_n
        b1, x1 = b[:, :ok], x[:, :ok]
        b1.normal_()
        hss.hss_ulv_solve_noalloc(ctx, m, b1, x1)
        ref = hss.hss_ulv_solve(ctx, m, b1)
        torch.cuda.synchronize()
        assert torch.equal(x1, ref)
    finally:
        hss.hss_matrix_destroy(m)
