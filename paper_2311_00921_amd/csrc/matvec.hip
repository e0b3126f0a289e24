// FP64 HSS matrix-vector product y = A x in the nested-basis form of Sec. 2
// (Eq. 6): the product A b of the construction error (Eq. 18) and the residual
// of the iterative refinement.
//
//   leaves      x~_i = U_i^T x_i  and  y_i = D_i x_i            (one launch)
//   up-sweep    x~_p = E_p^T [x~_c1; x~_c2]                     (one launch per stage)
//   down-sweep  y~_c1 = S_p x~_c2 + E_p[:r1, :] y~_p,
//               y~_c2 = S_p^T x~_c1 + E_p[r1:, :] y~_p          (one launch per stage)
//   leaves      y_i += U_i y~_i                                 (one launch)
//
// The sibling couplings of a node are applied in the same launch that passes
// the node's own y~ down to its children, so the product takes one launch per
// stage each way. Every operand is read once per sweep in coalesced 128-byte
// lines: row products give one row per thread (a column of the column-major
// block is contiguous across the threads), transposed products give one column
// per 16-lane group (lane p reads rows p, p + 16, ..., then the group sums).
// The bound is HBM: D, U twice, E twice and S once.
#include "hss_internal.h"

namespace hss {

namespace {

constexpr int MV_NT = 256;

// out[j] = sum_{i < rows} A[i + j lda] v[i] for j < cols (v in LDS), one column
// per 16-lane group; `add` accumulates into out.
__device__ __forceinline__ void tprod(const double* __restrict__ A, int64_t lda, int rows, int cols,
                                      const double* v, double* out, bool add) {
  const int lane16 = threadIdx.x & 15, grp = threadIdx.x >> 4, ngrp = MV_NT / 16;
  for (int j = grp; j < cols; j += ngrp) {
    const double* a = A + (int64_t)j * lda;
    double acc = 0.0;
    int i = lane16;
#pragma unroll 4
    for (; i + 48 < rows; i += 64) {
      const double a0 = a[i], a1 = a[i + 16], a2 = a[i + 32], a3 = a[i + 48];
      acc += a0 * v[i] + a1 * v[i + 16] + a2 * v[i + 32] + a3 * v[i + 48];
    }
    for (; i < rows; i += 16) acc += a[i] * v[i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (lane16 == 0) out[j] = add ? out[j] + acc : acc;
  }
}

// out[i] = sum_{j < cols} A[i + j lda] w[j] for i < rows (w in LDS), one row per
// thread; returns through `out` (LDS or global), `add` accumulates.
__device__ __forceinline__ void rprod(const double* __restrict__ A, int64_t lda, int rows, int cols,
                                      const double* w, double* out, bool add) {
  for (int i = threadIdx.x; i < rows; i += MV_NT) {
    const double* a = A + i;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
#pragma unroll 4
    for (; j + 1 < cols; j += 2) {
      acc0 += a[(int64_t)j * lda] * w[j];
      acc1 += a[(int64_t)(j + 1) * lda] * w[j + 1];
    }
    if (j < cols) acc0 += a[(int64_t)j * lda] * w[j];
    out[i] = add ? out[i] + acc0 + acc1 : acc0 + acc1;
  }
}

}  // namespace

// Leaves: gather x through perm, x~ = U^T x into the rank slot, y = D x
// scattered back through perm.
__global__ __launch_bounds__(MV_NT) void k_mv_leaf_up(const NodeDesc* __restrict__ nodes, int first,
                                                      const double* __restrict__ Db, const double* __restrict__ Bb,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      int64_t ld, int64_t nrhs, const int64_t* __restrict__ perm,
                                                      double* __restrict__ xt) {
  const NodeDesc nd = nodes[first + blockIdx.x];
  const int n = nd.n, r = nd.r;
  __shared__ double sx[kMaxBlock];
  __shared__ double sy[kMaxBlock];
  for (int64_t c = 0; c < nrhs; ++c) {
    for (int i = threadIdx.x; i < n; i += MV_NT) sx[i] = x[perm[nd.lo + i] + c * ld];
    __syncthreads();
    if (r > 0) tprod(Bb + nd.offB, n, n, r, sx, xt + nd.offR * nrhs + c * r, false);
    rprod(Db + nd.offD, n, n, n, sx, sy, false);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += MV_NT) y[perm[nd.lo + i] + c * ld] = sy[i];
    __syncthreads();
  }
}

// Up-sweep of one stage: x~_p = E_p^T [x~_c1; x~_c2] for its non-root nodes.
__global__ __launch_bounds__(MV_NT) void k_mv_up(const NodeDesc* __restrict__ nodes, int first,
                                                 const double* __restrict__ Bb, int64_t nrhs,
                                                 double* __restrict__ xt) {
  const NodeDesc nd = nodes[first + blockIdx.x];
  if (nd.r == 0) return;
  const NodeDesc c1 = nodes[nd.c1], c2 = nodes[nd.c2];
  const int n = nd.n;
  __shared__ double sv[kMaxBlock];
  for (int64_t c = 0; c < nrhs; ++c) {
    for (int i = threadIdx.x; i < n; i += MV_NT)
      sv[i] = i < c1.r ? xt[c1.offR * nrhs + i + c * c1.r] : xt[c2.offR * nrhs + (i - c1.r) + c * c2.r];
    __syncthreads();
    tprod(Bb + nd.offB, n, n, nd.r, sv, xt + nd.offR * nrhs + c * nd.r, false);
    __syncthreads();
  }
}

// Down-sweep of one stage: the children's y~ from the sibling coupling S_p and
// from the node's own y~_p through E_p (roots have no y~_p).
__global__ __launch_bounds__(MV_NT) void k_mv_down(const NodeDesc* __restrict__ nodes, int first,
                                                   const double* __restrict__ Bb, const double* __restrict__ Sb,
                                                   int64_t nrhs, const double* __restrict__ xt,
                                                   double* __restrict__ yt) {
  const NodeDesc nd = nodes[first + blockIdx.x];
  const NodeDesc c1 = nodes[nd.c1], c2 = nodes[nd.c2];
  const int r1 = c1.r, r2 = c2.r, r = nd.r;
  const double* S = Sb + nd.offS;
  __shared__ double s1[kMaxRank], s2[kMaxRank], sp[kMaxRank], o[kMaxBlock];
  for (int64_t c = 0; c < nrhs; ++c) {
    for (int i = threadIdx.x; i < r1; i += MV_NT) s1[i] = xt[c1.offR * nrhs + i + c * r1];
    for (int i = threadIdx.x; i < r2; i += MV_NT) s2[i] = xt[c2.offR * nrhs + i + c * r2];
    for (int i = threadIdx.x; i < r; i += MV_NT) sp[i] = yt[nd.offR * nrhs + i + c * r];
    __syncthreads();
    rprod(S, r1, r1, r2, s2, o, false);            // S x~_c2
    tprod(S, r1, r1, r2, s1, o + r1, false);       // S^T x~_c1
    __syncthreads();
    if (r > 0) rprod(Bb + nd.offB, r1 + r2, r1 + r2, r, sp, o, true);  // + E_p y~_p
    __syncthreads();
    for (int i = threadIdx.x; i < r1 + r2; i += MV_NT) {
      if (i < r1)
        yt[c1.offR * nrhs + i + c * r1] = o[i];
      else
        yt[c2.offR * nrhs + (i - r1) + c * r2] = o[i];
    }
    __syncthreads();
  }
}

// Leaves: y_i += U_i y~_i, scattered through perm.
__global__ __launch_bounds__(MV_NT) void k_mv_leaf_down(const NodeDesc* __restrict__ nodes, int first,
                                                        const double* __restrict__ Bb, double* __restrict__ y,
                                                        int64_t ld, int64_t nrhs, const int64_t* __restrict__ perm,
                                                        const double* __restrict__ yt) {
  const NodeDesc nd = nodes[first + blockIdx.x];
  const int n = nd.n, r = nd.r;
  if (r == 0) return;
  __shared__ double sw[kMaxRank];
  __shared__ double sy[kMaxBlock];
  for (int64_t c = 0; c < nrhs; ++c) {
    for (int j = threadIdx.x; j < r; j += MV_NT) sw[j] = yt[nd.offR * nrhs + j + c * r];
    __syncthreads();
    rprod(Bb + nd.offB, n, n, r, sw, sy, false);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += MV_NT) y[perm[nd.lo + i] + c * ld] += sy[i];
    __syncthreads();
  }
}

// y = A x over the stages (leaves first). Block sizes up to kMaxBlock and ranks
// up to kMaxRank (checked at construction and import).
void matvec_fp64(hss_matrix_t m, const double* x, double* y, int64_t nrhs, int64_t ld) {
  hipStream_t s = m->ctx->stream;
  ensure_vec_ws(m, nrhs);
  const int64_t* perm = m->dperm;
  const int ns = (int)m->stages.size();
  const LevelPlan& leaves = m->stages[0];
  hipLaunchKernelGGL(k_mv_leaf_up, dim3(leaves.count), dim3(MV_NT), 0, s, m->dnodes, leaves.first,
                     (const double*)m->dD, (const double*)m->dB, x, y, ld, nrhs, perm, m->dxt);
  HSS_HIP(hipGetLastError());
  for (int si = 1; si < ns; ++si) {
    const LevelPlan& lp = m->stages[si];
    hipLaunchKernelGGL(k_mv_up, dim3(lp.count), dim3(MV_NT), 0, s, m->dnodes, lp.first, (const double*)m->dB, nrhs,
                       m->dxt);
    HSS_HIP(hipGetLastError());
  }
  for (int si = ns - 1; si >= 1; --si) {
    const LevelPlan& lp = m->stages[si];
    hipLaunchKernelGGL(k_mv_down, dim3(lp.count), dim3(MV_NT), 0, s, m->dnodes, lp.first, (const double*)m->dB,
                       (const double*)m->dS, nrhs, (const double*)m->dxt, m->dyt);
    HSS_HIP(hipGetLastError());
  }
  if (ns > 1) {
    hipLaunchKernelGGL(k_mv_leaf_down, dim3(leaves.count), dim3(MV_NT), 0, s, m->dnodes, leaves.first,
                       (const double*)m->dB, y, ld, nrhs, perm, (const double*)m->dyt);
    HSS_HIP(hipGetLastError());
  }
}

}  // namespace hss
