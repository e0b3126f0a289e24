"""GPU checks at the 16-right-hand-side workload: Matern-3/2 on N = 65536
points in the unit cube, leaf 256, rank 64, scaled randomized construction
(8 levels, 256 leaves).

At this size the oracle factors and solves the whole exported matrix in about
a second, so the solution of all 16 right-hand sides and the log-determinant
are compared with the oracle's in full, not on samples. The BLR^2-ULV of the
same matrix (skeleton order 256 x 64 = 16384) is compared with both.

Tolerances: both sides are backward-stable FP64 factorizations of one matrix,
so the solutions agree to about kappa * u; at nugget 1e-6 kappa reaches about
1e7, so the gates are 1e-8 relative (normwise per column and elementwise over
the block; a wrong term shows at O(1)) and 1e-10 * (|logdet| + 1). The
residual gate against the FP64 HSS matvec is the 1e-8 level of the
benchmark's metric.
"""
import numpy as np
import pytest

import synth
from oracle import hss_oracle as O

from gpu_util import maxrel, rel

pytestmark = pytest.mark.gpu

W = synth.WORKLOADS["matern32_n65536"]


@pytest.fixture(scope="module")
def cfg2():
    import torch

    from paper_2311_00921_amd import hss

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = hss.hss_ctx_create(0)
    s = W.rank + W.oversample
    print(f"case {W.name}: construct N={W.n} leaf={W.leaf} rank={W.rank} s={s}", flush=True)
    X = torch.from_numpy(W.points()).cuda()
    Om = torch.from_numpy(np.ascontiguousarray(W.omega(s).T)).cuda().t()
    m = hss.hss_construct(ctx, X, W.kernel, W.leaf, rank=W.rank, omega=Om, length=W.length, nugget=W.nugget)
    del Om, X
    B = W.rhs()
    assert B.shape == (W.n, 16)
    b = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()
    rep = hss.unpack_desc(hss.hss_export(ctx, m))
    h = O.HSS(rep["n"], rep["levels"], rep["ranges"], rep["rank"], rep["D"], rep["U"], rep["E"], rep["S"])
    perm = np.asarray(rep["perm"])
    print("case oracle factor + solve of the exported matrix", flush=True)
    F = O.ulv_factor(h)
    x_or = np.empty_like(B)
    x_or[perm] = O.ulv_solve(h, F, B[perm])
    try:
        yield torch, hss, ctx, m, b, B, x_or, F.logdet
    finally:
        torch.cuda.synchronize()
        hss.hss_matrix_destroy(m)
        hss.hss_ctx_destroy(ctx)


def test_config2_sixteen_rhs_vs_oracle(cfg2):
    torch, hss, ctx, m, b, B, x_or, ld_or = cfg2
    print(f"case {W.name}: factor + solve, 16 right-hand sides", flush=True)
    hss.hss_ulv_factor(ctx, m)
    x = hss.hss_ulv_solve(ctx, m, b)
    xc = x.cpu().numpy()
    worst = max(rel(xc[:, c], x_or[:, c]) for c in range(16))
    print(f"x vs oracle: worst column {worst:.2e}, elementwise {maxrel(xc, x_or):.2e}", flush=True)
    assert worst <= 1e-8
    assert maxrel(xc, x_or) <= 1e-8
    ld = hss.hss_logdet(ctx, m)
    assert abs(ld - ld_or) <= 1e-10 * (abs(ld_or) + 1.0), (ld, ld_or)
    r = (b - hss.hss_matvec(ctx, m, x)).cpu().numpy()
    for c in range(16):
        assert np.linalg.norm(r[:, c]) / np.linalg.norm(B[:, c]) <= 1e-8, c


def test_config2_fused_factor_solve_equals_separate(cfg2):
    torch, hss, ctx, m, b, B, x_or, ld_or = cfg2
    hss.hss_ulv_factor(ctx, m)
    x1 = hss.hss_ulv_solve(ctx, m, b).cpu().numpy()
    x2 = hss.hss_ulv_factor_solve(ctx, m, b).cpu().numpy()
    assert np.array_equal(x1, x2)


def test_config2_blr2_vs_oracle_and_hss(cfg2):
    torch, hss, ctx, m, b, B, x_or, ld_or = cfg2
    hss.hss_ulv_factor(ctx, m)
    x_h = hss.hss_ulv_solve(ctx, m, b).cpu().numpy()
    assert hss.hss_blr2_stats(m)[0] == 256 * 64
    print(f"case {W.name}: BLR^2 factor, skeleton order 16384", flush=True)
    hss.hss_blr2_factor(ctx, m)
    xb = hss.hss_blr2_solve(ctx, m, b)
    x_b = xb.cpu().numpy()
    worst = max(rel(x_b[:, c], x_or[:, c]) for c in range(16))
    print(f"BLR^2 x vs oracle: worst column {worst:.2e}, vs HSS-ULV {rel(x_b, x_h):.2e}; "
          f"factor {hss.hss_blr2_stats(m)[1]:.2f} ms", flush=True)
    assert worst <= 1e-8 and maxrel(x_b, x_or) <= 1e-8
    assert rel(x_b, x_h) <= 1e-8 and maxrel(x_b, x_h) <= 1e-8
    ld = hss.hss_blr2_logdet(ctx, m)
    assert abs(ld - ld_or) <= 1e-10 * (abs(ld_or) + 1.0), (ld, ld_or)
