// ULV solve (Sec. 3.2, Eq. 17, applied as ordered products) and the FP64 HSS
// matrix-vector product, one kernel boundary per level.
//
// Forward, leaf to root, node p with block size n, rank r, m = n - r:
//   b^ = H^T b            (H = I - V T V^T, H[:, :r] = B diag(Sg))
//   y_R = L_RR^{-1} b^_R  (redundant part, coordinates r..n-1 of b^)
//   z_S = b^_S - L_SR y_R (skeleton part, coordinates 0..r-1 of b^)
//   parent's right-hand side rows = Sg * z_S (back to the basis coordinates)
// Root: L0 L0^T w = z. Backward, root to leaf:
//   x_S = Sg * (parent's solution rows); x_R = L_RR^{-T} (y_R - L_SR^T x_S)
//   x = H [x_S; x_R]
// One wavefront per node; RC right-hand sides are carried together.
#include "hss_internal.h"

namespace hss {

// Threads per node (NT): 1024 for stages of at most 512 nodes (two per compute
// unit), where a node's own memory-level parallelism bounds the time, 256 for
// the wide stages.
constexpr int kSolveWideNodes = 512;
constexpr int SNB = 16;   // block size of the blocked triangular solves
constexpr int RC = 4;     // right-hand sides per pass

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// out[j, c] = sum_{i < rows} A[i + j lda] x[i + c ldx] for j < cols: one wave per
// column (coalesced reads of the column), wave reduction. x, out in LDS.
template <int NT, typename T>
__device__ __forceinline__ void col_dots(const T* __restrict__ A, int64_t lda, int rows, int cols, const T* x,
                                         int ldx, T* out, int ldo, int nc) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int CW = 4;  // columns per wave per pass
  for (int j0 = wid * CW; j0 < cols; j0 += (NT / 64) * CW) {
    T acc[CW][RC];
#pragma unroll
    for (int q = 0; q < CW; ++q)
#pragma unroll
      for (int c = 0; c < RC; ++c) acc[q][c] = 0;
    for (int i = lane; i < rows; i += 64) {
      T a[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) a[q] = (j0 + q < cols) ? A[i + (int64_t)(j0 + q) * lda] : (T)0;
#pragma unroll
      for (int q = 0; q < CW; ++q)
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c < nc) acc[q][c] += a[q] * x[i + c * ldx];
    }
#pragma unroll
    for (int q = 0; q < CW; ++q)
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (c < nc) {
          const T v = wave_sum(acc[q][c]);
          if (lane == 0 && j0 + q < cols) out[j0 + q + c * ldo] = v;
        }
      }
  }
}

// The same product for wide blocks (NT >= 1024, few nodes per launch), in
// 16-lane groups: lane p of a group reads rows p, p + 16, ... of the group's
// columns, so that each load of a group is one 128-byte line, and a column's
// 16 partial sums meet by shuffles within the group. Group q takes columns q
// and q + NT / 16 of each pass; up to 16 * kColSegs rows of both columns are
// loaded before any product (one memory latency per pass). Ends with a
// barrier (red is not needed).
constexpr int kColSegs = 12;
template <int NT, typename T>
__device__ __forceinline__ void col_dots_split(const T* __restrict__ A, int64_t lda, int rows, int cols,
                                               const T* x, int ldx, T* out, int ldo, int nc, T* red) {
  constexpr int NG = NT / 16;
  const int p = threadIdx.x & 15, grp = threadIdx.x >> 4;
  for (int j0 = 0; j0 < cols; j0 += 2 * NG) {
    int jc[2];
    bool ok[2];
    const T* __restrict__ a[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      jc[h] = j0 + grp + h * NG;
      ok[h] = jc[h] < cols;
      a[h] = A + (int64_t)min(jc[h], cols - 1) * lda;
    }
    T acc[2][RC];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < RC; ++c) acc[h][c] = 0;
    for (int s0 = 0; s0 < rows; s0 += 16 * kColSegs) {
      T v[2][kColSegs];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < kColSegs; ++q) {
          const int i = s0 + 16 * q + p;
          v[h][q] = (ok[h] && i < rows) ? a[h][i] : (T)0;
        }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < kColSegs; ++q) {
          const int i = min(s0 + 16 * q + p, rows - 1);
#pragma unroll
          for (int c = 0; c < RC; ++c)
            if (c < nc) acc[h][c] += v[h][q] * x[i + c * ldx];
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (c < nc) {
          T sum = acc[h][c];
#pragma unroll
          for (int o = 1; o < 16; o <<= 1) sum += __shfl_xor(sum, o, 64);
          if (p == 0 && ok[h]) out[jc[h] + c * ldo] = sum;
        }
      }
  }
  __syncthreads();
}

// col_dots for the solve kernels: the chunked form when a node has 1024 threads.
template <int NT, typename T>
__device__ __forceinline__ void col_dots_node(const T* __restrict__ A, int64_t lda, int rows, int cols, const T* x,
                                              int ldx, T* out, int ldo, int nc, T* red) {
  if constexpr (NT >= 1024)
    col_dots_split<NT>(A, lda, rows, cols, x, ldx, out, ldo, nc, red);
  else
    col_dots<NT>(A, lda, rows, cols, x, ldx, out, ldo, nc);
}

// y[i, c] (+)= sign * sum_{j < cols} A[i + j lda] u[j + c ldu] for i < rows: one thread per row.
template <int NT, typename T>
__device__ __forceinline__ void row_gemv(const T* __restrict__ A, int64_t lda, int rows, int cols, const T* u,
                                         int ldu, T* y, int ldy, int nc, T sign) {
  for (int i = threadIdx.x; i < rows; i += NT) {
    T acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = 0;
    int j = 0;
    for (; j + 16 <= cols; j += 16) {
      T a[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = A[i + (int64_t)(j + q) * lda];
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c < nc) acc[c] += a[q] * u[j + q + c * ldu];
    }
    for (; j < cols; ++j) {
      const T a = A[i + (int64_t)j * lda];
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < nc) acc[c] += a * u[j + c * ldu];
    }
#pragma unroll
    for (int c = 0; c < RC; ++c)
      if (c < nc) y[i + c * ldy] += sign * acc[c];
  }
}

// row_gemv with the columns split over NT / 256 groups of 256 threads (one
// right-hand side, rows <= 512): a node's rows are too few to keep 1024
// threads busy, so each group covers a slice of the columns and the partial
// sums meet in LDS (red: (NT / 256) * 512 entries). Caller synchronizes after.
template <int NT, typename T>
__device__ __forceinline__ void row_gemv_wide(const T* __restrict__ A, int64_t lda, int rows, int cols,
                                              const T* u, int ldu, T* y, int ldy, int nc, T sign, T* red) {
  constexpr int G = NT / 256;
  if (G == 1 || nc != 1 || rows > 512) {
    row_gemv<NT>(A, lda, rows, cols, u, ldu, y, ldy, nc, sign);
    return;
  }
  const int g = threadIdx.x >> 8, tl = threadIdx.x & 255;
  const int c0 = (g * cols) / G, c1 = ((g + 1) * cols) / G;
  for (int i = tl; i < rows; i += 256) {
    T acc = 0;
    int j = c0;
    for (; j + 8 <= c1; j += 8) {
      T a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = A[i + (int64_t)(j + q) * lda];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += a[q] * u[j + q];
    }
    for (; j < c1; ++j) acc += A[i + (int64_t)j * lda] * u[j];
    red[g * 512 + i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows; i += NT) {
    T sum = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) sum += red[q * 512 + i];
    y[i] += sign * sum;
  }
}

// Value of v held by lane l (l wave-uniform), through scalar registers.
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bcast_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// In place y = L^{-1} y, L = F[0:m, 0:m] lower (ld ldf); y in LDS (ld ldy).
// 16-row diagonal blocks are solved by one wave; the rows below are updated by all threads.
template <int NT, typename T>
__device__ __forceinline__ void lower_solve(const T* __restrict__ F, int ldf, int m, T* y, int ldy, int nc) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int b0 = 0; b0 < m; b0 += SNB) {
    const int bb = min(SNB, m - b0);
    if (wid == 0) {
      // lane i < bb owns row b0 + i of the block
      T Lrow[SNB];
#pragma unroll
      for (int k = 0; k < SNB; ++k) Lrow[k] = (lane < bb && k <= lane && k < bb) ? F[(b0 + lane) + (int64_t)(b0 + k) * ldf] : (T)0;
      T v[RC];
#pragma unroll
      for (int c = 0; c < RC; ++c) v[c] = (lane < bb && c < nc) ? y[b0 + lane + c * ldy] : (T)0;
      // reciprocal of this lane's diagonal entry, taken off the serial chain
      const T rinv = (lane < bb) ? (T)1 / F[(b0 + lane) + (int64_t)(b0 + lane) * ldf] : (T)1;
#pragma unroll
      for (int k = 0; k < SNB; ++k) {
        if (k < bb) {
          const T rk = bcast_lane(rinv, k);
#pragma unroll
          for (int c = 0; c < RC; ++c) {
            if (c < nc) {
              const T yk = bcast_lane(v[c], k) * rk;
              if (lane == k) v[c] = yk;
              else if (lane > k) v[c] -= Lrow[k] * yk;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (lane < bb && c < nc) y[b0 + lane + c * ldy] = v[c];
    }
    __syncthreads();
    row_gemv<NT>(F + (b0 + bb) + (int64_t)b0 * ldf, ldf, m - b0 - bb, bb, y + b0, ldy, y + b0 + bb, ldy, nc, (T)-1);
    __syncthreads();
  }
}

// In place x = L^{-T} x, L = F[0:m, 0:m] lower.
template <int NT, typename T>
__device__ __forceinline__ void lower_t_solve(const T* __restrict__ F, int ldf, int m, T* x, int ldx, int nc,
                                              T* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nblk = (m + SNB - 1) / SNB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int b0 = bi * SNB, bb = min(SNB, m - b0);
    // scratch[k] = sum_{i >= b0+bb} L[i, b0+k] x[i]
    col_dots<NT>(F + (b0 + bb) + (int64_t)b0 * ldf, ldf, m - b0 - bb, bb, x + b0 + bb, ldx, scratch, SNB, nc);
    __syncthreads();
    if (wid == 0) {
      // lane i < bb owns column b0 + i of the block (L^T row)
      T Lcol[SNB];
#pragma unroll
      for (int k = 0; k < SNB; ++k) Lcol[k] = (lane < bb && k >= lane && k < bb) ? F[(b0 + k) + (int64_t)(b0 + lane) * ldf] : (T)0;
      T v[RC];
#pragma unroll
      for (int c = 0; c < RC; ++c) v[c] = (lane < bb && c < nc) ? x[b0 + lane + c * ldx] - scratch[lane + c * SNB] : (T)0;
      const T rinv = (lane < bb) ? (T)1 / F[(b0 + lane) + (int64_t)(b0 + lane) * ldf] : (T)1;
#pragma unroll
      for (int kk = SNB - 1; kk >= 0; --kk) {
        if (kk < bb) {
          const T rk = bcast_lane(rinv, kk);
#pragma unroll
          for (int c = 0; c < RC; ++c) {
            if (c < nc) {
              const T xk = bcast_lane(v[c], kk) * rk;
              if (lane == kk) v[c] = xk;
              else if (lane < kk) v[c] -= Lcol[kk] * xk;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (lane < bb && c < nc) x[b0 + lane + c * ldx] = v[c];
    }
    __syncthreads();
  }
}

// Forward substitution with the first m columns of F (n x n, lower, ld ldf)
// over all n rows at once (n <= NT): rows i < m end as y_R = L_RR^{-1} b_R,
// rows m..n-1 as b_S - L_SR y_R. Thread t owns row t, kept at y[pos(t)] with
// pos(t) = rS + t for t < m and t - m after. Each 16-column block is solved on
// the wave holding its rows (readlane chain; that wave's rows below the block
// take the block's update in the same chain); the other waves below apply the
// update with the block's solution from LDS (ys: 2 * SNB * RC entries, double
// buffered, so one barrier per block). A row's entries of the next block are
// loaded while the current one is solved, all loads coalesced along the rows.
template <int NT, typename T>
__device__ __forceinline__ void lower_solve_rows(const T* __restrict__ F, int ldf, int m, int n, T* y, int ldy,
                                                 int rS, int nc, T* ys) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const bool act = t < n;
  const int pos = t < m ? rS + t : t - m;
  T v[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) v[c] = (act && c < nc) ? y[pos + c * ldy] : (T)0;
  const T rinv = (t < m) ? (T)1 / F[t + (int64_t)t * ldf] : (T)1;
  const T* __restrict__ Frow = F + t;
  T cur[SNB], nxt[SNB];
  auto fetch = [&](int b0, T(&d)[SNB]) {
#pragma unroll
    for (int q = 0; q < SNB; ++q) {
      const int c = b0 + q;
      d[q] = (act && c < m && c <= t) ? Frow[(int64_t)c * ldf] : (T)0;
    }
  };
  fetch(0, cur);
  const int nblk = (m + SNB - 1) / SNB;
  for (int j = 0; j < nblk; ++j) {
    const int b0 = j * SNB, bb = min(SNB, m - b0);
    if (j + 1 < nblk) fetch(b0 + SNB, nxt);
    T* yb = ys + (j & 1) * SNB * RC;
    const int cw = b0 >> 6;  // blocks start at multiples of 16, so one wave holds all rows of a block
    if (wid == cw) {
      const int base = b0 & 63;
#pragma unroll
      for (int k = 0; k < SNB; ++k) {
        if (k < bb) {
          const T rk = bcast_lane(rinv, base + k);
#pragma unroll
          for (int c = 0; c < RC; ++c) {
            if (c < nc) {
              const T yk = bcast_lane(v[c], base + k) * rk;
              if (lane == base + k) v[c] = yk;
              else if (lane > base + k) v[c] -= cur[k] * yk;
            }
          }
        }
      }
      if (lane >= base && lane < base + bb)
#pragma unroll
        for (int c = 0; c < RC; ++c)
          if (c < nc) yb[(lane - base) + c * SNB] = v[c];
    }
    __syncthreads();
    if (wid > cw && act) {
#pragma unroll
      for (int q = 0; q < SNB; ++q)
        if (q < bb)
#pragma unroll
          for (int c = 0; c < RC; ++c)
            if (c < nc) v[c] -= cur[q] * yb[q + c * SNB];
    }
#pragma unroll
    for (int q = 0; q < SNB; ++q) cur[q] = nxt[q];
  }
  if (act)
#pragma unroll
    for (int c = 0; c < RC; ++c)
      if (c < nc) y[pos + c * ldy] = v[c];
}

// Columns per lane group in lower_t_solve_cols: L_RR of at most 16 * kTBlocks
// columns.
constexpr int kTBlocks = 10;

// x_R = L_RR^{-T} (y_R - L_SR^T x_S), L = the first m columns of F (n x n,
// lower, ld ldf), one right-hand side, four waves, m <= 16 * kTBlocks. x holds
// x_S at 0..r-1 and y_R at r..r+m-1 on entry, x_R there on exit. Lane (p, g)
// of wave w (p = lane & 15, g = lane >> 4) keeps in acc[k] its products of the
// rows = p (mod 16) already solved with column 16 k + 4 w + g; the 16 sums of a
// block are reduced over the lanes of each 16-lane group only when the
// backward sweep reaches that block. So every entry of L is loaded once, each
// load covering 16 consecutive rows of one column per 16 lanes, and a block's
// rows are loaded while the previous block is solved. The 16 x 16 diagonal
// block goes through LDS to wave 0, which solves it with a readlane chain
// (sh: 16 * 17 + 32 entries). Two barriers per block.
template <typename T>
__device__ __forceinline__ void lower_t_solve_cols(const T* __restrict__ F, int ldf, int m, int r, T* x, T* sh) {
  constexpr int KB = kTBlocks;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = lane & 15, cl = 4 * w + (lane >> 4);  // row within a block, column within a block
  T* dg = sh;             // dg[i * 17 + c]: entry (i, c) of the diagonal block
  T* sums = sh + 16 * 17;  // the block's reduced column sums
  T* rdg = sums + 16;      // reciprocals of its diagonal entries
  const int nblk = (m + 15) / 16;
  T acc[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) acc[k] = 0;
  // the S rows m..m+r-1, whose x_S is known
  for (int s0 = 0; s0 < r; s0 += 16) {
    const bool ok = s0 + p < r;
    const T xs = ok ? x[s0 + p] : (T)0;
    const T* __restrict__ Fr = F + (m + s0 + p);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int c = 16 * k + cl;
      if (ok && c < m) acc[k] += Fr[(int64_t)c * ldf] * xs;
    }
  }
  T cur[KB], nxt[KB];
  auto fetch = [&](int jj, T(&d)[KB]) {
    const int row = 16 * jj + p;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int c = 16 * k + cl;
      d[k] = (k <= jj && row < m && c <= row) ? F[row + (int64_t)c * ldf] : (T)0;
    }
  };
  if (nblk > 0) fetch(nblk - 1, cur);
  for (int jj = nblk - 1; jj >= 0; --jj) {
    const int R0 = 16 * jj, bb = min(16, m - R0);
    if (jj > 0) fetch(jj - 1, nxt);
    T a = 0, d = 0;
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (k == jj) {
        a = acc[k];
        d = cur[k];
      }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) a += __shfl_xor(a, o, 64);
    if (p == 0) sums[cl] = a;
    dg[p * 17 + cl] = d;
    if (p == cl) rdg[cl] = (p < bb) ? (T)1 / d : (T)1;
    __syncthreads();
    if (w == 0) {
      // lane q < 16 owns column R0 + q
      T v = (lane < bb) ? x[r + R0 + lane] - sums[lane] : (T)0;
      const T rq = (lane < 16) ? rdg[lane] : (T)1;
#pragma unroll
      for (int kk = 15; kk >= 0; --kk) {
        if (kk < bb) {
          const T xk = bcast_lane(v, kk) * bcast_lane(rq, kk);
          if (lane == kk) v = xk;
          else if (lane < kk) v -= dg[kk * 17 + lane] * xk;
        }
      }
      if (lane < bb) x[r + R0 + lane] = v;
    }
    __syncthreads();
    const T xp = (p < bb) ? x[r + R0 + p] : (T)0;
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (k < jj) acc[k] += cur[k] * xp;
#pragma unroll
    for (int k = 0; k < KB; ++k) cur[k] = nxt[k];
  }
}

template <typename T, int NT, int RMX, int NMX>
__global__ __launch_bounds__(NT, 1024 / NT) void k_solve_fwd(const NodeDesc* __restrict__ nodes, int first,
                                                  const T* __restrict__ Fb, const T* __restrict__ Vb,
                                                  const T* __restrict__ Yb, const T* __restrict__ Sgb,
                                                  T* __restrict__ vec, int64_t nrhs, int c0, int nc,
                                                  const double* __restrict__ b, int64_t ld,
                                                  const int64_t* __restrict__ perm, int leaf,
                                                  const T* __restrict__ Lib, const int64_t* __restrict__ offLi,
                                                  int use_inv) {
  const int p = first + blockIdx.x;
  const NodeDesc nd = nodes[p];
  const int n = nd.n, r = nd.r, m = nd.m;
  __shared__ T sb[NMX * RC];
  __shared__ T st[RMX * RC];
  __shared__ T su[RMX * RC];
  __shared__ T tm[RMX * RC];
  __shared__ T red[NT * RC];  // row_gemv_wide needs (NT / 256) * 512, col_dots_split NT * RC
  T* vp = vec + nd.offVec * nrhs;
  const T* F = Fb + nd.offF;
  const T* V = Vb + nd.offV;
  const T* Y = Yb + nd.offW;
  const T* Sg = Sgb + nd.offSg;
  for (int i = threadIdx.x; i < n; i += NT)
    for (int c = 0; c < nc; ++c)
      sb[i + c * n] = leaf ? (T)b[perm[nd.lo + i] + (int64_t)(c0 + c) * ld] : vp[i + (int64_t)(c0 + c) * n];
  __syncthreads();
  // b^ = H^T b = b - V (Y^T b) with Y = V T kept by the factorization
  col_dots_node<NT>(Y, n, n, r, sb, n, st, r, nc, red);
  __syncthreads();
  row_gemv_wide<NT>(V, n, n, r, st, r, sb, n, nc, (T)-1, red);
  __syncthreads();
  // y_R = L_RR^{-1} b^_R  (b^_R = sb[r:n])
  if (use_inv == 2) {
    // a root factored in two blocks at h: y1 = L11^{-1} b1, y2 = L22^{-1} (b2 - L21 y1)
    const int h = root_split_h(n), h2 = n - h;
    const T* Li1 = Lib + offLi[p];
    const T* Li2 = Li1 + (int64_t)h * h;
    for (int i = threadIdx.x; i < h * RC; i += NT) tm[i] = 0;
    __syncthreads();
    row_gemv_wide<NT>(Li1, h, h, h, sb, n, tm, h, nc, (T)1, red);
    __syncthreads();
    for (int i = threadIdx.x; i < h; i += NT)
      for (int c = 0; c < nc; ++c) sb[i + c * n] = tm[i + c * h];
    __syncthreads();
    row_gemv_wide<NT>(F + h, n, h2, h, sb, n, sb + h, n, nc, (T)-1, red);
    __syncthreads();
    for (int i = threadIdx.x; i < h2 * RC; i += NT) tm[i] = 0;
    __syncthreads();
    row_gemv_wide<NT>(Li2, h2, h2, h2, sb + h, n, tm, h2, nc, (T)1, red);
    __syncthreads();
    for (int i = threadIdx.x; i < h2; i += NT)
      for (int c = 0; c < nc; ++c) sb[h + i + c * n] = tm[i + c * h2];
    __syncthreads();
  } else if (use_inv) {
    const T* Li = Lib + offLi[p];
    for (int i = threadIdx.x; i < m * RC; i += NT) tm[i] = 0;
    __syncthreads();
    row_gemv_wide<NT>(Li, m, m, m, sb + r, n, tm, m, nc, (T)1, red);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += NT)
      for (int c = 0; c < nc; ++c) sb[r + i + c * n] = tm[i + c * m];
    __syncthreads();
  } else if (n <= NT) {
    // y_R and z_S = b^_S - L_SR y_R in one sweep over the first m columns of F
    lower_solve_rows<NT>(F, n, m, n, sb, n, r, nc, tm);
    __syncthreads();
  } else {
    lower_solve<NT>(F, n, m, sb + r, n, nc);
  }
  if (use_inv || n > NT) {
    // z_S = b^_S - L_SR y_R   (L_SR = F[m:n, 0:m])
    row_gemv_wide<NT>(F + m, n, r, m, sb + r, n, sb, n, nc, (T)-1, red);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < m; i += NT)
    for (int c = 0; c < nc; ++c) vp[i + (int64_t)(c0 + c) * n] = sb[r + i + c * n];
  if (nd.parent < 0) return;  // a root: y = L^{-1} b is all that is left
  const NodeDesc par = nodes[nd.parent];
  T* pp = vec + par.offVec * nrhs;
  for (int j = threadIdx.x; j < r; j += NT)
    for (int c = 0; c < nc; ++c) pp[nd.child_row + j + (int64_t)(c0 + c) * par.n] = Sg[j] * sb[j + c * n];
}

template <typename T, int NT, int RMX, int NMX>
__global__ __launch_bounds__(NT, 1024 / NT) void k_solve_bwd(const NodeDesc* __restrict__ nodes, int first,
                                                  const T* __restrict__ Fb, const T* __restrict__ Vb,
                                                  const T* __restrict__ Yb, const T* __restrict__ Sgb,
                                                  T* __restrict__ vec, int64_t nrhs, int c0, int nc,
                                                  double* __restrict__ x, int64_t ld,
                                                  const int64_t* __restrict__ perm, int leaf,
                                                  const T* __restrict__ Lib, const int64_t* __restrict__ offLi,
                                                  int use_inv) {
  const int p = first + blockIdx.x;
  const NodeDesc nd = nodes[p];
  const int n = nd.n, r = nd.r, m = nd.m;
  __shared__ T sx[NMX * RC];
  __shared__ T st[RMX * RC];
  __shared__ T su[RMX * RC];
  __shared__ T scr[SNB * RC];
  __shared__ T tm[NMX * RC];
  __shared__ T red[NT * RC];  // row_gemv_wide needs (NT / 256) * 512, col_dots_split NT * RC
  T* vp = vec + nd.offVec * nrhs;
  const T* F = Fb + nd.offF;
  const T* V = Vb + nd.offV;
  const T* Y = Yb + nd.offW;
  const T* Sg = Sgb + nd.offSg;
  // x_S (H coordinates) into sx[0:r], y_R into sx[r:n]; a root has r = 0
  if (nd.parent >= 0) {
    const NodeDesc par = nodes[nd.parent];
    const T* pp = vec + par.offVec * nrhs;
    for (int j = threadIdx.x; j < r; j += NT)
      for (int c = 0; c < nc; ++c) sx[j + c * n] = Sg[j] * pp[nd.child_row + j + (int64_t)(c0 + c) * par.n];
  }
  for (int i = threadIdx.x; i < m; i += NT)
    for (int c = 0; c < nc; ++c) sx[r + i + c * n] = vp[i + (int64_t)(c0 + c) * n];
  __syncthreads();
  // L_RR^{-T} (y_R - L_SR^T x_S) in one backward sweep over the first m columns of F
  const bool by_cols = NT == 256 && !use_inv && nc == 1 && m <= 16 * kTBlocks;
  if (!by_cols) {
    // t = y_R - L_SR^T x_S: tm[k] = sum_j L_SR[j, k] x_S[j] (column k of L_SR is contiguous)
    col_dots_node<NT>(F + m, n, r, m, sx, n, tm, n, nc, red);
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += NT)
      for (int c = 0; c < nc; ++c) sx[r + k + c * n] -= tm[k + c * n];
    __syncthreads();
  }
  if (by_cols) {
    if constexpr (NT == 256) lower_t_solve_cols(F, n, m, r, sx, tm);
    __syncthreads();
  } else if (use_inv == 2) {
    // a root factored in two blocks at h: x2 = L22^{-T} y2, x1 = L11^{-T} (y1 - L21^T x2)
    const int h = root_split_h(n), h2 = n - h;
    const T* Li1 = Lib + offLi[p];
    const T* Li2 = Li1 + (int64_t)h * h;
    col_dots_node<NT>(Li2, h2, h2, h2, sx + h, n, tm, n, nc, red);
    __syncthreads();
    for (int i = threadIdx.x; i < h2; i += NT)
      for (int c = 0; c < nc; ++c) sx[h + i + c * n] = tm[i + c * n];
    __syncthreads();
    col_dots_node<NT>(F + h, n, h2, h, sx + h, n, tm, n, nc, red);
    __syncthreads();
    for (int k = threadIdx.x; k < h; k += NT)
      for (int c = 0; c < nc; ++c) sx[k + c * n] -= tm[k + c * n];
    __syncthreads();
    col_dots_node<NT>(Li1, h, h, h, sx, n, tm, n, nc, red);
    __syncthreads();
    for (int i = threadIdx.x; i < h; i += NT)
      for (int c = 0; c < nc; ++c) sx[i + c * n] = tm[i + c * n];
    __syncthreads();
  } else if (use_inv) {
    // x_R = L_RR^{-T} t: x_R[j] = sum_i Li[i, j] t_i  (columns of Li are contiguous)
    const T* Li = Lib + offLi[p];
    col_dots_node<NT>(Li, m, m, m, sx + r, n, tm, n, nc, red);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += NT)
      for (int c = 0; c < nc; ++c) sx[r + i + c * n] = tm[i + c * n];
    __syncthreads();
  } else {
    lower_t_solve<NT>(F, n, m, sx + r, n, nc, scr);
  }
  // x = H x^ = x^ - Y (V^T x^)
  col_dots_node<NT>(V, n, n, r, sx, n, st, r, nc, red);
  __syncthreads();
  row_gemv_wide<NT>(Y, n, n, r, st, r, sx, n, nc, (T)-1, red);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT)
    for (int c = 0; c < nc; ++c) {
      if (leaf)
        x[perm[nd.lo + i] + (int64_t)(c0 + c) * ld] = (double)sx[i + c * n];
      else
        vp[i + (int64_t)(c0 + c) * n] = sx[i + c * n];
    }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

void ensure_vec_ws(hss_matrix_t m, int64_t nrhs) {
  if (m->ws_nrhs >= nrhs) return;
  // a recorded solve graph holds the addresses of the buffers freed below
  if (m->gexec_solve) {
    (void)hipGraphExecDestroy(m->gexec_solve);
    m->gexec_solve = nullptr;
    m->solve_key = hss_matrix_s::SolveKey{};
  }
  if (m->dvec) dev_free(m->dvec);
  if (m->dxt) dev_free(m->dxt);
  if (m->dyt) dev_free(m->dyt);
  m->dvec = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->sum_n * nrhs, 1));
  m->dxt = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->sum_r * nrhs, 1));
  m->dyt = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->sum_r * nrhs, 1));
  m->ws_nrhs = nrhs;
}

// LDS frame of a stage's solve kernels: (rank, rows) up to (128, 512),
// (256, 512), (128, 1024) or (512, 1024).
static int solve_shape(const LevelPlan& lp) {
  if (lp.nmax <= 512) return lp.rmax <= 128 ? 0 : 1;
  return lp.rmax <= 128 ? 2 : 3;
}

// One stage of the forward sweep (roots finish with y = L^{-1} b) and of the
// backward sweep, for right-hand sides c0 .. c0 + nc - 1, on stream s.
template <typename T>
static void launch_fwd(hss_matrix_t m, int si, const T* F, const T* V, const T* Yw, const T* Sg, T* vec, const T* Li,
                       int inv, const double* b, int64_t nrhs, int64_t c0, int nc, int64_t ld, hipStream_t s) {
  const LevelPlan& lp = m->stages[si];
#define HSS_FWD(NT, RMX, NMX)                                                                                   \
  hipLaunchKernelGGL((k_solve_fwd<T, NT, RMX, NMX>), dim3(lp.count), dim3(NT), 0, s, m->dnodes, lp.first, F, V, Yw, \
                     Sg, vec, nrhs, (int)c0, nc, b, ld, (const int64_t*)m->dperm, lp.leaf, Li,                     \
                     (const int64_t*)m->dOffLi, inv)
  HSS_CHECK(lp.rmax <= kMaxRank && lp.nmax <= kMaxBlock, HSS_ERR_UNSUPPORTED,
            "solve: rank above 512 or block above 1024");
  const int shape = solve_shape(lp);
  if (lp.count <= kSolveWideNodes) {
    switch (shape) {
      case 0: HSS_FWD(1024, 128, 512); break;
      case 1: HSS_FWD(1024, 256, 512); break;
      case 2: HSS_FWD(1024, 128, 1024); break;
      default: HSS_FWD(1024, 512, 1024); break;
    }
  } else {
    switch (shape) {
      case 0: HSS_FWD(256, 128, 512); break;
      case 1: HSS_FWD(256, 256, 512); break;
      case 2: HSS_FWD(256, 128, 1024); break;
      default: HSS_FWD(256, 512, 1024); break;
    }
  }
#undef HSS_FWD
  HSS_HIP(hipGetLastError());
}

template <typename T>
static void launch_bwd(hss_matrix_t m, int si, const T* F, const T* V, const T* Yw, const T* Sg, T* vec, const T* Li,
                       int inv, double* x, int64_t nrhs, int64_t c0, int nc, int64_t ld, hipStream_t s) {
  const LevelPlan& lp = m->stages[si];
#define HSS_BWD(NT, RMX, NMX)                                                                                   \
  hipLaunchKernelGGL((k_solve_bwd<T, NT, RMX, NMX>), dim3(lp.count), dim3(NT), 0, s, m->dnodes, lp.first, F, V, Yw, \
                     Sg, vec, nrhs, (int)c0, nc, x, ld, (const int64_t*)m->dperm, lp.leaf, Li,                     \
                     (const int64_t*)m->dOffLi, inv)
  const int shape = solve_shape(lp);
  if (lp.count <= kSolveWideNodes) {
    switch (shape) {
      case 0: HSS_BWD(1024, 128, 512); break;
      case 1: HSS_BWD(1024, 256, 512); break;
      case 2: HSS_BWD(1024, 128, 1024); break;
      default: HSS_BWD(1024, 512, 1024); break;
    }
  } else {
    switch (shape) {
      case 0: HSS_BWD(256, 128, 512); break;
      case 1: HSS_BWD(256, 256, 512); break;
      case 2: HSS_BWD(256, 128, 1024); break;
      default: HSS_BWD(256, 512, 1024); break;
    }
  }
#undef HSS_BWD
  HSS_HIP(hipGetLastError());
}

// Forward sweep over the stages leaves-first, then the backward sweep in the
// reverse order, RC right-hand sides at a time (from column c_begin on).
template <typename T>
static void solve_impl(hss_matrix_t m, const T* F, const T* V, const T* Yw, const T* Sg, T* vec, const T* Li,
                       const std::vector<char>& inv_used, const double* b, double* x, int64_t nrhs, int64_t ld,
                       int64_t c_begin = 0) {
  hipStream_t s = m->ctx->stream;
  const int ns = (int)m->stages.size();
  for (int64_t c0 = c_begin; c0 < nrhs; c0 += RC) {
    const int nc = (int)std::min<int64_t>(RC, nrhs - c0);
    for (int si = 0; si < ns; ++si) {
      Prof pf(m->ctx, "solve_forward", m->stages[si].level);
      launch_fwd<T>(m, si, F, V, Yw, Sg, vec, Li, inv_used[si], b, nrhs, c0, nc, ld, s);
    }
    for (int si = ns - 1; si >= 0; --si) {
      Prof pf(m->ctx, "solve_backward", m->stages[si].level);
      launch_bwd<T>(m, si, F, V, Yw, Sg, vec, Li, inv_used[si], x, nrhs, c0, nc, ld, s);
    }
  }
}

// One sweep of the leaf stage alone (FP64 factors): forward (b in, the
// parents' slots of the vector workspace out) or backward (the parents' slots
// in, x out), for right-hand sides c0 .. c0 + nc - 1 (nc <= solve_chunk()).
void solve_leaf_sweep(hss_matrix_t m, bool forward, const double* b, double* x, int64_t nrhs, int64_t c0, int nc,
                      int64_t ld) {
  hipStream_t s = m->ctx->stream;
  if (forward)
    launch_fwd<double>(m, 0, m->dF, m->dV, m->dW, m->dSg, m->dvec, m->dLi, m->inv_used64[0], b, nrhs, c0, nc, ld, s);
  else
    launch_bwd<double>(m, 0, m->dF, m->dV, m->dW, m->dSg, m->dvec, m->dLi, m->inv_used64[0], x, nrhs, c0, nc, ld, s);
}

int solve_chunk() { return RC; }

void solve_fp64(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  ensure_vec_ws(m, nrhs);
  solve_fp64_ws(m, b, x, nrhs, ld, m->dvec);
}

// The solve with a caller-provided per-node vector workspace (sum_n x nrhs
// doubles); launches kernels only.
void solve_fp64_ws(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld, double* vec) {
  solve_impl<double>(m, m->dF, m->dV, m->dW, m->dSg, vec, m->dLi, m->inv_used64, b, x, nrhs, ld);
}


// FP64 factorization and solve in one pass. The forward sweep of a stage
// needs only that stage's factors and its children's forward results, so it
// is enqueued on the second stream as soon as the stage's factorization
// kernels are, and runs while the stages above are factored (their kernels
// are few and latency-bound and leave most compute units idle). The main
// stream joins the second one after the root, then runs the backward sweep.
// The first RC right-hand sides ride along; any further ones follow.
void factor_solve_fp64(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  hss_ctx_t cx = m->ctx;
  hipStream_t s = cx->stream;
  ensure_vec_ws(m, nrhs);
  if (!cx->aux_stream) HSS_HIP(hipStreamCreateWithFlags(&cx->aux_stream, hipStreamNonBlocking));
  if (!cx->ev_trail) HSS_HIP(hipEventCreateWithFlags(&cx->ev_trail, hipEventDisableTiming));
  hipStream_t a = cx->aux_stream;
  const int nc = (int)std::min<int64_t>(RC, nrhs);
  m->after_stage = [&](int si) {
    HSS_HIP(hipEventRecord(cx->ev_trail, s));
    HSS_HIP(hipStreamWaitEvent(a, cx->ev_trail, 0));
    launch_fwd<double>(m, si, m->dF, m->dV, m->dW, m->dSg, m->dvec, m->dLi, m->inv_used64[si], b, nrhs, 0, nc, ld,
                       a);
  };
  try {
    factor_fp64(m);
  } catch (...) {
    m->after_stage = nullptr;
    throw;
  }
  m->after_stage = nullptr;
  HSS_HIP(hipEventRecord(cx->ev_trail, a));
  HSS_HIP(hipStreamWaitEvent(s, cx->ev_trail, 0));
  for (int si = (int)m->stages.size() - 1; si >= 0; --si)
    launch_bwd<double>(m, si, m->dF, m->dV, m->dW, m->dSg, m->dvec, m->dLi, m->inv_used64[si], x, nrhs, 0, nc, ld,
                       s);
  if (nrhs > RC)
    solve_impl<double>(m, m->dF, m->dV, m->dW, m->dSg, m->dvec, m->dLi, m->inv_used64, b, x, nrhs, ld, RC);
}

}  // namespace hss
