// HSS construction on the GPU (Sec. 2: shared bases from a pivoted QR, Eq. 2;
// nested bases and skeleton couplings, Eq. 6), from random samples of the
// off-diagonal row blocks, in two modes. PLAIN is the paper's construction: each
// node's basis is the pivoted QR of the samples of its off-diagonal row block,
// and the couplings are orthogonal projections. SCALED (the default of the
// workloads) first scales each node's samples by the inverse Cholesky factor of
// its diagonal block, which keeps the represented matrix SPD:
//
//   tree      recursive coordinate bisection on the device (tree.hip: longest box
//             side, ties -> lowest axis, order by (coordinate, index), left child =
//             ceil(size/2))
//   leaves    D_i = K(X_i, X_i) + nugget I, Psi_i = chol(D_i)^{-T} Omega_i,
//             Z = (A - blkdiag D) Psi  (one kernel-evaluating product over all pairs)
//   level l   for each node p with diagonal block M_p and samples Z_p:
//               Lc = chol(M_p), Y = Lc^{-1} Z_p, V = first k columns of QRCP(Y),
//               Lc V = B R (thin QR, diag R >= 0), basis = B, Sigma_p = R R^T,
//               W_p = Lc^{-T} V R^T, Wbig_p = blkdiag(Wbig_children) W_p
//             siblings p1, p2 of g: S_g = Wbig_p1^T A[I_p1, I_p2] Wbig_p2,
//               M_g = [[Sigma_p1, S_g], [S_g^T, Sigma_p2]],
//               Phi_g = [B_p1^T Phi_p1; B_p2^T Phi_p2],
//               Z_g = [W_p1^T Z_p1 - S_g Phi'_p2; W_p2^T Z_p2 - S_g^T Phi'_p1]
// PLAIN is the same sweep with Lc = I: Psi = Omega, Y = Z_p, basis = W_p = V,
// and no merged diagonal blocks.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hss_internal.h"

namespace hss {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// construction-time node table (per level)
// ---------------------------------------------------------------------------

struct CNode {
  int64_t lo;      // first tree position
  int32_t npts;    // points
  int32_t n;       // block size at this level
  int32_t k;       // rank found (output of QRCP)
  int32_t pad;
  int64_t offM, offL, offI;      // M, Lc, Linv (n x n)
  int64_t offZ, offPhi;          // samples and test matrix rows (n x s)
  int64_t offY, offH, offQ;      // Y (n x s), reflectors (n x kmax), Q (n x kmax)
  int64_t offR;                  // R (kmax x s)
};

// ---------------------------------------------------------------------------
// kernel evaluation
// ---------------------------------------------------------------------------

struct KParams {
  int32_t kind;
  double length, sigma2, nugget, alpha, eps;
};

__device__ __forceinline__ double kfun(const KParams& k, double d) {
  switch (k.kind) {
    case HSS_K_EXPONENTIAL:
      return k.sigma2 * exp(-d / k.length);
    case HSS_K_MATERN32: {
      const double t = 1.7320508075688772 * d / k.length;
      return k.sigma2 * (1.0 + t) * exp(-t);
    }
    case HSS_K_GAUSSIAN:
      return k.sigma2 * exp(-(d * d) / (k.length * k.length));
    case HSS_K_LAPLACE2D:
      return -log(k.eps + d);
    default: {
      const double t = k.eps + d;
      return exp(-k.alpha * t) / t;
    }
  }
}

// coordinates in tree order, structure of arrays: X[a * N + t]
__device__ __forceinline__ double kentry(const KParams& kp, const double* __restrict__ X, int64_t N, int dim,
                                         int64_t i, int64_t j) {
  double acc = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double d = X[a * N + i] - X[a * N + j];
    acc += d * d;
  }
  double v = kfun(kp, sqrt(acc));
  if (i == j) v += kp.nugget;
  return v;
}

// D blocks of the leaves: D_i[a + b n] = K(x_lo+a, x_lo+b) (+ nugget on the diagonal)
__global__ __launch_bounds__(256) void k_leaf_blocks(const NodeDesc* __restrict__ nodes, int first, KParams kp,
                                                     const double* __restrict__ X, int64_t N, int dim,
                                                     double* __restrict__ D) {
  const NodeDesc nd = nodes[first + blockIdx.y];
  const int n = nd.n;
  double* Dp = D + nd.offD;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < (int64_t)n * n; e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e % n), b = (int)(e / n);
    Dp[e] = kentry(kp, X, N, dim, nd.lo + a, nd.lo + b);
  }
}

// Batched product with an evaluated kernel block:
//   Out[i, c] (+)= sum_j K(x_{r0+i}, x_{c0+j}) In[j, c],  i < nr, j < nc, c < s
// 64 output rows x 128 columns per workgroup; K tiles of 64 x 16 are evaluated
// into LDS and contracted on the matrix cores (FP64 16x16x4).
struct KGemmDesc {
  int64_t r0, c0;
  int32_t nr, nc, s;
  int32_t ldin, ldout;
  const double* In;
  double* Out;
};

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int KBM = 64, KBN = 128, KBK = 16;

// With blk (the leaf of each tree position), pairs of points in one leaf count
// as zero: the product with A - blkdiag(D) without forming A x and subtracting
// D x (a kernel whose diagonal dwarfs its off-diagonal entries would lose
// digits to the cancellation).
__global__ __launch_bounds__(256) void k_kgemm(const KGemmDesc* __restrict__ descs, KParams kp,
                                               const double* __restrict__ X, int64_t N, int dim, int accumulate,
                                               const int32_t* __restrict__ blk) {
  const KGemmDesc d = descs[blockIdx.y];
  const int tilesM = (d.nr + KBM - 1) / KBM;
  const int tilesN = (d.s + KBN - 1) / KBN;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int row0 = (blockIdx.x % tilesM) * KBM;
  const int col0 = (blockIdx.x / tilesM) * KBN;
  __shared__ double Ks[KBK][KBM + 1];
  __shared__ double Bs[KBK][KBN + 1];
  __shared__ double xr[3][KBM];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  for (int e = tid; e < dim * KBM; e += 256) {
    const int a = e / KBM, r = e % KBM;
    xr[a][r] = (row0 + r < d.nr) ? X[a * N + d.r0 + row0 + r] : 0.0;
  }
  v4d acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;
  __syncthreads();
  for (int k0 = 0; k0 < d.nc; k0 += KBK) {
    // evaluate a 64 x 16 kernel tile: thread -> (row r = e % 64, column kk = e / 64)
#pragma unroll
    for (int e0 = 0; e0 < KBM * KBK; e0 += 256) {
      const int e = e0 + tid;
      const int r = e % KBM, kk = e / KBM;
      const int64_t gi = d.r0 + row0 + r, gj = d.c0 + k0 + kk;
      double v = 0.0;
      if (row0 + r < d.nr && k0 + kk < d.nc && !(blk && blk[gi] == blk[gj])) {
        double acc2 = 0.0;
        for (int a = 0; a < dim; ++a) {
          const double df = xr[a][r] - X[a * N + gj];
          acc2 += df * df;
        }
        v = kfun(kp, sqrt(acc2));
        if (gi == gj) v += kp.nugget;
      }
      Ks[kk][r] = v;
    }
#pragma unroll
    for (int e0 = 0; e0 < KBN * KBK; e0 += 256) {
      const int e = e0 + tid;
      const int kk = e % KBK, c = e / KBK;
      Bs[kk][c] = (k0 + kk < d.nc && col0 + c < d.s) ? d.In[(k0 + kk) + (int64_t)(col0 + c) * d.ldin] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KBK; kk += 4) {
      double a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Ks[kk + lk][wm + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk + lk][wn + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wm + 16 * i + lk + 4 * v;
        const int col = col0 + wn + 16 * j + lr;
        if (row < d.nr && col < d.s) {
          double* o = d.Out + row + (int64_t)col * d.ldout;
          *o = accumulate ? *o + acc[i][j][v] : acc[i][j][v];
        }
      }
}

// ---------------------------------------------------------------------------
// small per-node dense kernels
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Inverse of the lower Cholesky factor: Li = Lc^{-1}; also zeroes Lc's upper part.
__global__ __launch_bounds__(256) void k_trinv(const CNode* __restrict__ cn, double* __restrict__ Lb,
                                               double* __restrict__ Ib) {
  const CNode c = cn[blockIdx.x];
  const int n = c.n;
  double* Lc = Lb + c.offL;
  double* Li = Ib + c.offI;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e % n, j = e / n;
    if (i < j) Lc[e] = 0.0;
  }
  __syncthreads();
  for (int col = threadIdx.x; col < n; col += 256) {
    double* x = Li + (int64_t)col * n;
    for (int i = 0; i < col; ++i) x[i] = 0.0;
    x[col] = 1.0 / Lc[col + (int64_t)col * n];
    for (int k = col + 1; k < n; ++k) {
      double acc = 0.0;
      for (int j = col; j < k; ++j) acc += Lc[k + (int64_t)j * n] * x[j];
      x[k] = -acc / Lc[k + (int64_t)k * n];
    }
  }
}

// Column-pivoted (or plain) Householder QR of Y (n x ncols, in place), stopped
// after k steps: k = kfix if kfix > 0, else the number of leading pivots with
// |R_jj| > tol |R_00| (at least 1), capped by kcap. Pivot = remaining column
// of largest norm, norms recomputed every step, first index on ties. Writes
// Q (n x k, diag R >= 0), R (k x ncols, pivoted column order) and k.
__global__ __launch_bounds__(256) void k_qrcp(CNode* __restrict__ cn, double* __restrict__ Yb,
                                              double* __restrict__ Hb, double* __restrict__ Qb,
                                              double* __restrict__ Rb, int ncols, int kfix, double tol, int kcap,
                                              int pivot, int ldr) {
  CNode c = cn[blockIdx.x];
  const int n = c.n;
  double* Y = Yb + c.offY;
  double* H = Hb + c.offH;
  double* Q = Qb + c.offQ;
  double* R = Rb + c.offR;
  __shared__ double cnorm[kMaxSamples];
  __shared__ double sgn[kMaxSamples];
  __shared__ int sp, sk;
  __shared__ double salpha, sR00;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int kmax = min(n, ncols);
  if (kcap > 0) kmax = min(kmax, kcap);
  if (kfix > 0) kmax = min(kmax, kfix);
  if (tid == 0) sk = kmax;
  __syncthreads();
  for (int j = 0; j < kmax; ++j) {
    if (pivot) {
      for (int cc = j + wid; cc < ncols; cc += 4) {
        double p = 0.0;
        for (int i = j + lane; i < n; i += 64) {
          const double y = Y[i + (int64_t)cc * n];
          p += y * y;
        }
        p = wsum(p);
        if (lane == 0) cnorm[cc] = sqrt(p);
      }
    } else if (wid == 0) {
      double p = 0.0;
      for (int i = j + lane; i < n; i += 64) {
        const double y = Y[i + (int64_t)j * n];
        p += y * y;
      }
      p = wsum(p);
      if (lane == 0) cnorm[j] = sqrt(p);
    }
    __syncthreads();
    if (tid == 0) {
      int p = j;
      if (pivot)
        for (int cc = j + 1; cc < ncols; ++cc)
          if (cnorm[cc] > cnorm[p]) p = cc;
      sp = p;
      salpha = cnorm[p];
      if (j == 0) sR00 = cnorm[p];
      if (kfix <= 0 && j > 0 && !(cnorm[p] > tol * sR00)) sk = j;
    }
    __syncthreads();
    if (sk == j) break;
    const int p = sp;
    const double alpha = salpha;
    if (p != j) {
      for (int i = tid; i < n; i += 256) {
        const double t = Y[i + (int64_t)j * n];
        Y[i + (int64_t)j * n] = Y[i + (int64_t)p * n];
        Y[i + (int64_t)p * n] = t;
      }
      __syncthreads();
    }
    const double x0 = Y[j + (int64_t)j * n];
    const double s = (x0 >= 0.0) ? 1.0 : -1.0;
    const double vnorm = sqrt(2.0 * alpha * (alpha + fabs(x0)));
    for (int i = tid; i < n; i += 256) {
      double v = 0.0;
      if (alpha > 0.0 && i >= j) v = ((i == j) ? x0 + s * alpha : Y[i + (int64_t)j * n]) / vnorm;
      H[i + (int64_t)j * n] = v;
    }
    if (tid == 0) sgn[j] = -s;
    __syncthreads();
    // R row j for the pivot column, then reflect the remaining columns
    if (tid == 0) R[j + (int64_t)j * ldr] = alpha;  // (-s*alpha) * sgn = alpha
    for (int cc = j + 1 + wid; cc < ncols; cc += 4) {
      double p2 = 0.0;
      for (int i = j + lane; i < n; i += 64) p2 += H[i + (int64_t)j * n] * Y[i + (int64_t)cc * n];
      p2 = 2.0 * wsum(p2);
      for (int i = j + lane; i < n; i += 64) Y[i + (int64_t)cc * n] -= p2 * H[i + (int64_t)j * n];
      if (lane == 0) R[j + (int64_t)cc * ldr] = -s * Y[j + (int64_t)cc * n];
    }
    __syncthreads();
  }
  const int k = sk;
  // Q = H_0 ... H_{k-1} [I_k; 0], then the sign convention
  for (int e = tid; e < n * k; e += 256) {
    const int i = e % n, cc = e / n;
    Q[e] = (i == cc) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    for (int cc = j + wid; cc < k; cc += 4) {
      double p2 = 0.0;
      for (int i = j + lane; i < n; i += 64) p2 += H[i + (int64_t)j * n] * Q[i + (int64_t)cc * n];
      p2 = 2.0 * wsum(p2);
      for (int i = j + lane; i < n; i += 64) Q[i + (int64_t)cc * n] -= p2 * H[i + (int64_t)j * n];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * k; e += 256) {
    const int cc = e / n;
    Q[e] *= sgn[cc];
  }
  if (tid == 0) cn[blockIdx.x].k = k;
}

// M_g = [[Sigma_p1, S], [S^T, Sigma_p2]]
__global__ __launch_bounds__(256) void k_cmerge(const CNode* __restrict__ parents, const CNode* __restrict__ kids,
                                                const double* __restrict__ Sig, const int64_t* __restrict__ offSig,
                                                const double* __restrict__ Sb, const int64_t* __restrict__ offS,
                                                double* __restrict__ Mb) {
  const int g = blockIdx.x;
  const CNode P = parents[g];
  const int r1 = kids[2 * g].k, r2 = kids[2 * g + 1].k;
  const int n = r1 + r2;
  const double* S1 = Sig + offSig[2 * g];
  const double* S2 = Sig + offSig[2 * g + 1];
  const double* S = Sb + offS[g];
  double* M = Mb + P.offM;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e % n, j = e / n;
    double v;
    if (i < r1 && j < r1)
      v = S1[i + j * r1];
    else if (i >= r1 && j >= r1)
      v = S2[(i - r1) + (j - r1) * r2];
    else if (i < r1)
      v = S[i + (int64_t)(j - r1) * r1];
    else
      v = S[j + (int64_t)(i - r1) * r1];
    M[e] = v;
  }
}

// rows of a (tree-ordered) matrix gathered from the caller's order
__global__ void k_gather_rows(const double* __restrict__ src, int64_t lds, const int64_t* __restrict__ perm,
                              int64_t n, int s, double* __restrict__ dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * s; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    dst[i + c * ldd] = src[perm[i] + c * lds];
  }
}

// Judge of a node's basis: with Q (n x k, orthonormal) from the pivoted QR of
// the first s_b sample columns, the relative residual of the probe columns
// Y[:, s_b : s_b + p] is |(I - Q Q^T) Y_p|_F / |Y_p|_F; fail[i] = 1 when it
// exceeds thr. One block per node.
__global__ __launch_bounds__(256) void k_judge(const CNode* __restrict__ cn, const double* __restrict__ Yb,
                                               const double* __restrict__ Qb, int sb, int probes, double thr,
                                               int32_t* __restrict__ fail) {
  const CNode c = cn[blockIdx.x];
  const int n = c.n, k = c.k;
  const double* Y = Yb + c.offY + (int64_t)sb * n;
  const double* Q = Qb + c.offQ;
  __shared__ double y[kMaxBlock];
  __shared__ double cq[kMaxRank];
  __shared__ double red[2][256];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double num = 0.0, den = 0.0;
  for (int j = 0; j < probes; ++j) {
    for (int i = tid; i < n; i += 256) y[i] = Y[i + (int64_t)j * n];
    __syncthreads();
    for (int q = wid; q < k; q += 4) {  // cq = Q^T y, one column per wave
      double acc = 0.0;
      for (int i = lane; i < n; i += 64) acc += Q[i + (int64_t)q * n] * y[i];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) cq[q] = acc;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
      double r = y[i];
      for (int q = 0; q < k; ++q) r -= Q[i + (int64_t)q * n] * cq[q];
      num += r * r;
      den += y[i] * y[i];
    }
    __syncthreads();
  }
  red[0][tid] = num;
  red[1][tid] = den;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) fail[blockIdx.x] = (red[1][0] > 0.0 && sqrt(red[0][0] / red[1][0]) > thr) ? 1 : 0;
}

__global__ void k_points_soa(const double* __restrict__ pts, const int64_t* __restrict__ perm, int64_t n, int dim,
                             double* __restrict__ X) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    for (int a = 0; a < dim; ++a) X[a * n + t] = pts[perm[t] * dim + a];
}

// dst[i + j ldd] = src[i + j lds] for i < rows, j < cols, one descriptor per grid.y
struct Copy2D {
  const double* src;
  double* dst;
  int32_t rows, cols, lds, ldd;
};

__global__ void k_copy2d(const Copy2D* __restrict__ descs) {
  const Copy2D d = descs[blockIdx.y];
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % d.rows), j = (int)(e / d.rows);
    d.dst[i + (int64_t)j * d.ldd] = d.src[i + (int64_t)j * d.lds];
  }
}

__global__ void k_copy_blocks(const double* __restrict__ src, const int64_t* __restrict__ soff,
                              double* __restrict__ dst, const int64_t* __restrict__ doff,
                              const int64_t* __restrict__ len) {
  const int b = blockIdx.y;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len[b]; e += (int64_t)gridDim.x * blockDim.x)
    dst[doff[b] + e] = src[soff[b] + e];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct DevBuf {
  double* p = nullptr;
  int64_t len = 0;
  void ensure(int64_t n) {
    if (n <= len) return;
    if (p) dev_free(p);
    p = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(n, 1));
    len = n;
  }
  ~DevBuf() {
    if (p) dev_free(p);
  }
};

template <typename X>
struct DevArr {
  X* p = nullptr;
  size_t cnt = 0;
  void upload(const std::vector<X>& h, hipStream_t s) {
    if (h.size() > cnt) {
      if (p) dev_free(p);
      p = (X*)dev_alloc(sizeof(X) * std::max<size_t>(h.size(), 1));
      cnt = h.size();
    }
    if (!h.empty()) HSS_HIP(hipMemcpyAsync(p, h.data(), sizeof(X) * h.size(), hipMemcpyHostToDevice, s));
  }
  ~DevArr() {
    if (p) dev_free(p);
  }
};

static void run_copy2d(const std::vector<Copy2D>& h, hipStream_t st) {
  if (h.empty()) return;
  DevArr<Copy2D> d;
  d.upload(h, st);
  for (size_t c0 = 0; c0 < h.size(); c0 += 65535) {
    const int cnt = (int)std::min<size_t>(65535, h.size() - c0);
    hipLaunchKernelGGL(k_copy2d, dim3(16, cnt), dim3(256), 0, st, (const Copy2D*)(d.p + c0));
    HSS_HIP(hipGetLastError());
  }
  HSS_HIP(hipStreamSynchronize(st));
}

static void run_gemm(std::vector<GemmDesc>&& v, bool ta, bool tb, double alpha, double beta, hipStream_t s) {
  GemmBatch b;
  b.host = std::move(v);
  gemm_upload(b, s);
  gemm_launch_f64(b, ta, tb, alpha, beta, s);
  HSS_HIP(hipStreamSynchronize(s));  // the descriptor buffer is freed below
  gemm_free(b);
}

static void run_kgemm(const std::vector<KGemmDesc>& v, const KParams& kp, const double* X, int64_t N, int dim,
                      int accumulate, hipStream_t s, const int32_t* blk = nullptr) {
  if (v.empty()) return;
  int tiles = 0;
  for (auto& d : v) tiles = std::max(tiles, ((d.nr + KBM - 1) / KBM) * ((d.s + KBN - 1) / KBN));
  DevArr<KGemmDesc> dv;
  dv.upload(v, s);
  for (size_t b0 = 0; b0 < v.size(); b0 += 65535) {
    const int cnt = (int)std::min<size_t>(65535, v.size() - b0);
    hipLaunchKernelGGL(k_kgemm, dim3(tiles, cnt), dim3(256), 0, s, dv.p + b0, kp, X, N, dim, accumulate, blk);
    HSS_HIP(hipGetLastError());
  }
  HSS_HIP(hipStreamSynchronize(s));
}

void launch_pchol_external(const NodeDesc* nodes, int first, int count, int nmax, double* F, int32_t* info,
                           double* logdet, hipStream_t s);

// Features of the learned rank model for every non-root node, in heap order
// (node k >= 1): log2 of the point count clipped at 13, bounding-box extents in
// decreasing order over the kernel length, gap to the sibling's box over the
// kernel length, log10 of the length, -log10 of the tolerance.
// The leaves' boxes come from the tree kernels (leafbox: 2^L x 6, lo then hi,
// zero beyond dim); the boxes above are unions of their children's.
static std::vector<float> node_features(const std::vector<double>& leafbox, int L, const std::vector<int64_t>& leaf_lo,
                                        double length, double tol) {
  const int nn = (2 << L) - 1, nl = 1 << L;
  std::vector<double> lo((size_t)nn * 3, 0.0), hi((size_t)nn * 3, 0.0);
  std::vector<int64_t> np(nn, 0);
  for (int i = 0; i < nl; ++i) {
    const int k = nl - 1 + i;
    for (int d = 0; d < 3; ++d) {
      lo[3 * k + d] = leafbox[(size_t)i * 6 + d];
      hi[3 * k + d] = leafbox[(size_t)i * 6 + 3 + d];
    }
    np[k] = leaf_lo[i + 1] - leaf_lo[i];
  }
  for (int k = nl - 2; k >= 0; --k) {
    for (int d = 0; d < 3; ++d) {
      lo[3 * k + d] = std::min(lo[3 * (2 * k + 1) + d], lo[3 * (2 * k + 2) + d]);
      hi[3 * k + d] = std::max(hi[3 * (2 * k + 1) + d], hi[3 * (2 * k + 2) + d]);
    }
    np[k] = np[2 * k + 1] + np[2 * k + 2];
  }
  std::vector<float> f((size_t)(nn - 1) * 7);
  for (int k = 1; k < nn; ++k) {
    const int sib = (k & 1) ? k + 1 : k - 1;
    double e[3], g2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      e[d] = hi[3 * k + d] - lo[3 * k + d];
      const double gap = std::max(0.0, std::max(lo[3 * sib + d] - hi[3 * k + d], lo[3 * k + d] - hi[3 * sib + d]));
      g2 += gap * gap;
    }
    std::sort(e, e + 3, [](double a, double b) { return a > b; });
    float* row = &f[(size_t)(k - 1) * 7];
    row[0] = (float)std::min(std::log2((double)std::max<int64_t>(np[k], 1)), 13.0);
    row[1] = (float)(e[0] / length);
    row[2] = (float)(e[1] / length);
    row[3] = (float)(e[2] / length);
    row[4] = (float)(std::sqrt(g2) / length);
    row[5] = (float)std::log10(length);
    row[6] = (float)(-std::log10(tol));
  }
  return f;
}

void rankmlp_predict(hss_rankmlp_t r, const float* d_feats, int64_t n, int cap, int32_t* d_ranks);

bool construct(hss_matrix_t m, const double* d_points, int32_t dim, const hss_kernel& kern,
               const hss_construct_opts& o, const double* d_omega, int32_t s_avail, SamplePlan& sp) {
  hipStream_t st = m->ctx->stream;
  const int64_t N = m->n;
  const int L = m->L;
  const bool plain = o.mode == HSS_COMPRESS_PLAIN;
  KParams kp{kern.kind, kern.length, kern.sigma2, kern.nugget, kern.alpha, kern.eps};
  // ---- tree: node ranges from the sizes, the permutation on the device ----
  const std::vector<int64_t> leaf_lo = tree_leaf_lo(N, L);
  const int nleaves = 1 << L;
  m->nnodes = (2 << L) - 1;
  m->nodes.assign(m->nnodes, NodeDesc{});
  for (int i = 0; i < nleaves; ++i) {
    NodeDesc& nd = m->nodes[nleaves - 1 + i];
    nd.lo = leaf_lo[i];
    nd.npts = (int32_t)(leaf_lo[i + 1] - leaf_lo[i]);
    HSS_CHECK(nd.npts >= 1 && nd.npts <= kMaxBlock, HSS_ERR_UNSUPPORTED, "leaf sizes must be in [1, 1024]");
  }
  // provisional ranks: the leaf layout (D offsets) depends on the leaves only
  for (int k = 1; k < m->nnodes; ++k) m->nodes[k].r = 1;
  layout_representation(m);
  const bool want_boxes = sp.s_basis == 0;  // the rank model needs the leaves' boxes
  DevBuf lbox;
  lbox.ensure(want_boxes ? (int64_t)nleaves * 6 : 1);
  build_tree(st, d_points, N, dim, L, m->dperm, want_boxes ? lbox.p : nullptr);
  DevBuf Xs;
  Xs.ensure(N * dim);
  hipLaunchKernelGGL(k_points_soa, dim3(1024), dim3(256), 0, st, d_points, (const int64_t*)m->dperm, N, dim, Xs.p);
  HSS_HIP(hipGetLastError());
  {
    const LevelPlan& lp = m->levels[L];
    hipLaunchKernelGGL(k_leaf_blocks, dim3(64, lp.count), dim3(256), 0, st, m->dnodes, lp.first, kp,
                       (const double*)Xs.p, N, dim, m->dD);
    HSS_HIP(hipGetLastError());
  }
  if (L == 0) {
    HSS_HIP(hipStreamSynchronize(st));
    return true;
  }
  const int kfix = o.rank;
  int kcap = o.rank > 0 ? o.rank : (o.max_rank > 0 ? o.max_rank : 128);
  kcap = std::min(kcap, kMaxRank);
  if (sp.s_basis == 0) {
    // sample count from the learned rank model: largest predicted node rank + 8
    std::vector<double> hb((size_t)nleaves * 6);
    HSS_HIP(hipMemcpyAsync(hb.data(), lbox.p, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
    HSS_HIP(hipStreamSynchronize(st));
    const std::vector<float> f = node_features(hb, L, leaf_lo, kern.length > 0.0 ? kern.length : 1.0, o.tol);
    const int64_t cntf = (int64_t)f.size() / 7;
    float* dF = (float*)dev_alloc(sizeof(float) * f.size());
    int32_t* dR = (int32_t*)dev_alloc(sizeof(int32_t) * cntf);
    std::vector<int32_t> pr(cntf);
    try {
      HSS_HIP(hipMemcpyAsync(dF, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, st));
      rankmlp_predict(sp.model, dF, cntf, kcap, dR);
      HSS_HIP(hipMemcpyAsync(pr.data(), dR, sizeof(int32_t) * cntf, hipMemcpyDeviceToHost, st));
      HSS_HIP(hipStreamSynchronize(st));
    } catch (...) {
      dev_free(dF);
      dev_free(dR);
      throw;
    }
    dev_free(dF);
    dev_free(dR);
    sp.predicted_max = *std::max_element(pr.begin(), pr.end());
    sp.s_basis = std::max(1, std::min(s_avail - sp.probes, sp.predicted_max + 8));
    if (sp.s_basis >= s_avail - sp.probes) sp.abort_on_fail = false;  // already the last attempt
  }
  const int sb = sp.s_basis;
  const int s = sb + sp.probes;  // sample columns carried through the levels (basis samples, then the probe)
  kcap = std::min(kcap, sb);
  HSS_CHECK(kcap >= 1, HSS_ERR_INVALID_ARGUMENT, "sample count too small");

  DevBuf Om, PsiN, Zfull;
  Om.ensure(N * s);
  PsiN.ensure(N * s);
  Zfull.ensure(N * s);
  hipLaunchKernelGGL(k_gather_rows, dim3(2048), dim3(256), 0, st, d_omega, (int64_t)N, (const int64_t*)m->dperm, N,
                     sb, Om.p, (int64_t)N);
  HSS_HIP(hipGetLastError());
  if (sp.probes > 0) {  // the probe: the last columns of the caller's test matrix
    hipLaunchKernelGGL(k_gather_rows, dim3(2048), dim3(256), 0, st, d_omega + (int64_t)(s_avail - sp.probes) * N,
                       (int64_t)N, (const int64_t*)m->dperm, N, sp.probes, Om.p + (int64_t)sb * N, (int64_t)N);
    HSS_HIP(hipGetLastError());
  }
  sp.sample_bytes = 3 * (int64_t)sizeof(double) * N * s;
  DevArr<int32_t> dfail;

  std::vector<CNode> cur(nleaves);
  std::vector<const double*> zp(nleaves), php(nleaves);
  std::vector<int> ldz(nleaves);
  for (int i = 0; i < nleaves; ++i) {
    cur[i] = CNode{};
    cur[i].lo = leaf_lo[i];
    cur[i].npts = (int32_t)(leaf_lo[i + 1] - leaf_lo[i]);
    cur[i].n = cur[i].npts;
  }
  DevBuf Mb, Lb, Ib, Yb, Hb, Qb, Rb, Kb, Bb, Htmp, Rk, VRt, Wb, Sig, Zn, Phin, Mn, Tg, Sg;
  DevBuf WbigPrev, WbigCur, Bstore, Sstore, Zlvl, Philvl;
  std::vector<int64_t> wprev, wcur;
  std::vector<int> prevnodes_npts, prevnodes_k;
  std::vector<int64_t> bst_off(m->nnodes, -1), bst_len(m->nnodes, 0), sst_off(m->nnodes, -1), sst_len(m->nnodes, 0);
  std::vector<int32_t> rank(m->nnodes, 0);
  int64_t bst_used = 0, sst_used = 0;
  DevArr<CNode> dcur;
  DevArr<NodeDesc> dtn;
  DevArr<int32_t> dinfo;
  DevBuf ldscratch;

  auto stage = [&](DevBuf& store, int64_t& used, const double* src, int64_t len) -> int64_t {
    if (used + len > store.len) {
      DevBuf nb;
      nb.ensure(std::max<int64_t>(2 * store.len, used + len) + 1024);
      if (used > 0) HSS_HIP(hipMemcpyAsync(nb.p, store.p, sizeof(double) * used, hipMemcpyDeviceToDevice, st));
      HSS_HIP(hipStreamSynchronize(st));
      std::swap(nb.p, store.p);
      std::swap(nb.len, store.len);
    }
    HSS_HIP(hipMemcpyAsync(store.p + used, src, sizeof(double) * len, hipMemcpyDeviceToDevice, st));
    const int64_t off = used;
    used += len;
    return off;
  };

  for (int l = L; l >= 1; --l) {
    const int cnt = 1 << l;
    const int first = (1 << l) - 1;
    int64_t oM = 0, oY = 0, oH = 0, oR = 0;
    int nmax = 0;
    for (auto& c : cur) {
      c.offM = c.offL = c.offI = oM;
      oM += (int64_t)c.n * c.n;
      c.offY = oY;
      oY += (int64_t)c.n * s;
      c.offH = c.offQ = oH;
      oH += (int64_t)c.n * kcap;
      c.offR = oR;
      oR += (int64_t)kcap * s;
      nmax = std::max(nmax, c.n);
    }
    HSS_CHECK(nmax <= kMaxBlock, HSS_ERR_UNSUPPORTED, "diagonal block larger than 1024");
    Lb.ensure(oM);
    Ib.ensure(oM);
    Yb.ensure(oY);
    Hb.ensure(oH);
    Qb.ensure(oH);
    Rb.ensure(oR);
    // ---- Lc = chol(M_p) (SCALED only) ----
    if (plain) {
      // no scaling
    } else if (l == L) {
      for (int i = 0; i < cnt; ++i) {
        const NodeDesc& nd = m->nodes[first + i];
        HSS_HIP(hipMemcpyAsync(Lb.p + cur[i].offL, m->dD + nd.offD, sizeof(double) * cur[i].n * cur[i].n,
                               hipMemcpyDeviceToDevice, st));
      }
    } else {
      HSS_HIP(hipMemcpyAsync(Lb.p, Mb.p, sizeof(double) * oM, hipMemcpyDeviceToDevice, st));
    }
    if (!plain) {
      std::vector<NodeDesc> tn(cnt);
      for (int i = 0; i < cnt; ++i) {
        tn[i] = NodeDesc{};
        tn[i].n = cur[i].n;
        tn[i].m = cur[i].n;
        tn[i].offF = cur[i].offL;
      }
      dtn.upload(tn, st);
      std::vector<int32_t> zero(5, 0);  // status words + the flag of system 0
      dinfo.upload(zero, st);
      ldscratch.ensure(cnt + 1);
      launch_pchol_external(dtn.p, 0, cnt, nmax, Lb.p, dinfo.p, ldscratch.p, st);
      std::vector<int32_t> inf(4);
      HSS_HIP(hipMemcpyAsync(inf.data(), dinfo.p, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
      HSS_HIP(hipStreamSynchronize(st));
      HSS_CHECK(inf[0] == 0, HSS_ERR_NOT_SPD,
                "diagonal block of node " + std::to_string(first + inf[1]) + " (level " + std::to_string(l) +
                    ") is not positive definite");
    }
    dcur.upload(cur, st);
    if (!plain) {
      hipLaunchKernelGGL(k_trinv, dim3(cnt), dim3(256), 0, st, (const CNode*)dcur.p, Lb.p, Ib.p);
      HSS_HIP(hipGetLastError());
    }
    if (l == L) {
      // Psi = Lc^{-T} Omega (leaf rows; Omega itself for PLAIN), Z = A Psi - D Psi
      if (plain) {
        HSS_HIP(hipMemcpyAsync(PsiN.p, Om.p, sizeof(double) * N * s, hipMemcpyDeviceToDevice, st));
      } else {
        std::vector<GemmDesc> g;
        for (int i = 0; i < cnt; ++i)
          g.push_back({Ib.p + cur[i].offI, Om.p + cur[i].lo, nullptr, PsiN.p + cur[i].lo, cur[i].n, (int)s, cur[i].n,
                       cur[i].n, (int)N, 0, (int)N, 0, 0});
        run_gemm(std::move(g), true, false, 1.0, 0.0, st);
      }
      // Z = (A - blkdiag D) Psi: pairs within a leaf skipped in the product
      std::vector<int32_t> leafid(N);
      for (int i = 0; i < cnt; ++i)
        for (int64_t t = leaf_lo[i]; t < leaf_lo[i + 1]; ++t) leafid[t] = i;
      DevArr<int32_t> dleaf;
      dleaf.upload(leafid, st);
      std::vector<KGemmDesc> kg;
      const int64_t chunk = 1 << 16;
      for (int64_t r0 = 0; r0 < N; r0 += chunk)
        kg.push_back({r0, 0, (int32_t)std::min<int64_t>(chunk, N - r0), (int32_t)N, (int32_t)s, (int32_t)N,
                      (int32_t)N, PsiN.p, Zfull.p + r0});
      run_kgemm(kg, kp, Xs.p, N, dim, 0, st, dleaf.p);
      for (int i = 0; i < cnt; ++i) {
        zp[i] = Zfull.p + cur[i].lo;
        php[i] = PsiN.p + cur[i].lo;
        ldz[i] = (int)N;
      }
    }
    // ---- Y = Lc^{-1} Z (Y = Z for PLAIN), V = QRCP(Y)[:, :k] ----
    if (plain) {
      std::vector<Copy2D> cp;
      for (int i = 0; i < cnt; ++i) cp.push_back({zp[i], Yb.p + cur[i].offY, cur[i].n, (int)s, ldz[i], cur[i].n});
      run_copy2d(cp, st);
    } else {
      std::vector<GemmDesc> g;
      for (int i = 0; i < cnt; ++i)
        g.push_back({Ib.p + cur[i].offI, zp[i], nullptr, Yb.p + cur[i].offY, cur[i].n, (int)s, cur[i].n, cur[i].n,
                     ldz[i], 0, cur[i].n, 0, 0});
      run_gemm(std::move(g), false, false, 1.0, 0.0, st);
    }
    dcur.upload(cur, st);
    hipLaunchKernelGGL(k_qrcp, dim3(cnt), dim3(256), 0, st, dcur.p, Yb.p, Hb.p, Qb.p, Rb.p, sb, kfix, o.tol, kcap,
                       1, kcap);
    HSS_HIP(hipGetLastError());
    if (sp.probes > 0) {
      std::vector<int32_t> zf(cnt, 0);
      dfail.upload(zf, st);
      hipLaunchKernelGGL(k_judge, dim3(cnt), dim3(256), 0, st, (const CNode*)dcur.p, (const double*)Yb.p,
                         (const double*)Qb.p, sb, sp.probes, sp.judge_thr, dfail.p);
      HSS_HIP(hipGetLastError());
      std::vector<int32_t> hf(cnt);
      HSS_HIP(hipMemcpyAsync(hf.data(), dfail.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st));
      HSS_HIP(hipStreamSynchronize(st));
      int nf = 0;
      for (int32_t v : hf) nf += v;
      sp.judge_failures += nf;
      if (nf > 0 && sp.abort_on_fail) {
        sp.passed = false;
        return false;
      }
    }
    HSS_HIP(hipMemcpyAsync(cur.data(), dcur.p, sizeof(CNode) * cnt, hipMemcpyDeviceToHost, st));
    HSS_HIP(hipStreamSynchronize(st));
    // ---- K = Lc V = B R, Sigma = R R^T, W = Lc^{-T} V R^T ----
    std::vector<int64_t> offK(cnt), offKK(cnt);
    int64_t oK = 0, oKK = 0;
    for (int i = 0; i < cnt; ++i) {
      offK[i] = oK;
      oK += (int64_t)cur[i].n * cur[i].k;
      offKK[i] = oKK;
      oKK += (int64_t)cur[i].k * cur[i].k;
    }
    Kb.ensure(oK);
    Bb.ensure(oK);
    Htmp.ensure(oK);
    VRt.ensure(oK);
    Wb.ensure(oK);
    Rk.ensure(oKK);
    Sig.ensure(oKK);
    if (plain) {
      // the basis is V itself (orthonormal), and so is W
      std::vector<Copy2D> cp;
      for (int i = 0; i < cnt; ++i) {
        cp.push_back({Qb.p + cur[i].offQ, Bb.p + offK[i], cur[i].n, cur[i].k, cur[i].n, cur[i].n});
        cp.push_back({Qb.p + cur[i].offQ, Wb.p + offK[i], cur[i].n, cur[i].k, cur[i].n, cur[i].n});
      }
      run_copy2d(cp, st);
    }
    if (!plain) HSS_HIP(hipMemsetAsync(Rk.p, 0, sizeof(double) * std::max<int64_t>(oKK, 1), st));
    if (!plain) {
      std::vector<GemmDesc> g;
      for (int i = 0; i < cnt; ++i)
        g.push_back({Lb.p + cur[i].offL, Qb.p + cur[i].offQ, nullptr, Kb.p + offK[i], cur[i].n, cur[i].k, cur[i].n,
                     cur[i].n, cur[i].n, 0, cur[i].n, 0, 0});
      run_gemm(std::move(g), false, false, 1.0, 0.0, st);
    }
    if (!plain) {
      std::vector<int> ks;
      for (auto& c : cur) ks.push_back(c.k);
      std::sort(ks.begin(), ks.end());
      ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
      for (int kk : ks) {
        std::vector<CNode> grp;
        for (int i = 0; i < cnt; ++i)
          if (cur[i].k == kk) {
            CNode q = cur[i];
            q.offY = offK[i];
            q.offH = offK[i];
            q.offQ = offK[i];
            q.offR = offKK[i];
            grp.push_back(q);
          }
        DevArr<CNode> dg;
        dg.upload(grp, st);
        hipLaunchKernelGGL(k_qrcp, dim3((int)grp.size()), dim3(256), 0, st, dg.p, Kb.p, Htmp.p, Bb.p, Rk.p, kk, kk,
                           0.0, kk, 0, kk);
        HSS_HIP(hipGetLastError());
        HSS_HIP(hipStreamSynchronize(st));
      }
    }
    if (!plain) {
      std::vector<GemmDesc> g1, g2, g3;
      for (int i = 0; i < cnt; ++i) {
        const int n = cur[i].n, k = cur[i].k;
        // R is upper triangular: zero its strict lower part is implied by the QR writes
        g1.push_back({Rk.p + offKK[i], Rk.p + offKK[i], nullptr, Sig.p + offKK[i], k, k, k, k, k, 0, k, 0, 0});
        g2.push_back({Qb.p + cur[i].offQ, Rk.p + offKK[i], nullptr, VRt.p + offK[i], n, k, k, n, k, 0, n, 0, 0});
        g3.push_back({Ib.p + cur[i].offI, VRt.p + offK[i], nullptr, Wb.p + offK[i], n, k, n, n, n, 0, n, 0, 0});
      }
      run_gemm(std::move(g1), false, true, 1.0, 0.0, st);
      run_gemm(std::move(g2), false, true, 1.0, 0.0, st);
      run_gemm(std::move(g3), true, false, 1.0, 0.0, st);
    }
    for (int i = 0; i < cnt; ++i) {
      const int node = first + i;
      rank[node] = cur[i].k;
      bst_len[node] = (int64_t)cur[i].n * cur[i].k;
      bst_off[node] = stage(Bstore, bst_used, Bb.p + offK[i], bst_len[node]);
    }
    // ---- Wbig over the node's points ----
    wcur.assign(cnt, 0);
    {
      int64_t ow = 0;
      for (int i = 0; i < cnt; ++i) {
        wcur[i] = ow;
        ow += (int64_t)cur[i].npts * cur[i].k;
      }
      WbigCur.ensure(ow);
      if (l == L) {
        HSS_HIP(hipMemcpyAsync(WbigCur.p, Wb.p, sizeof(double) * ow, hipMemcpyDeviceToDevice, st));
      } else {
        std::vector<GemmDesc> g;
        for (int i = 0; i < cnt; ++i) {
          const int c1 = 2 * i, c2 = 2 * i + 1;
          const int np1 = prevnodes_npts[c1], np2 = prevnodes_npts[c2];
          const int r1 = prevnodes_k[c1], r2 = prevnodes_k[c2];
          const int n = cur[i].n, k = cur[i].k, np = cur[i].npts;
          (void)r2;
          g.push_back({WbigPrev.p + wprev[c1], Wb.p + offK[i], nullptr, WbigCur.p + wcur[i], np1, k, r1, np1, n, 0, np,
                       0, 0});
          g.push_back({WbigPrev.p + wprev[c2], Wb.p + offK[i] + r1, nullptr, WbigCur.p + wcur[i] + np1, np2, k,
                       prevnodes_k[c2], np2, n, 0, np, 0, 0});
        }
        run_gemm(std::move(g), false, false, 1.0, 0.0, st);
      }
    }
    // ---- couplings of siblings: S_g = Wbig_p1^T A[I_p1, I_p2] Wbig_p2 ----
    const int np = cnt / 2;
    std::vector<int64_t> offT(np), offS(np);
    {
      int64_t ot = 0, os = 0;
      for (int g = 0; g < np; ++g) {
        offT[g] = ot;
        ot += (int64_t)cur[2 * g].npts * cur[2 * g + 1].k;
        offS[g] = os;
        os += (int64_t)cur[2 * g].k * cur[2 * g + 1].k;
      }
      Tg.ensure(ot);
      Sg.ensure(os);
      std::vector<KGemmDesc> kg;
      for (int g = 0; g < np; ++g) {
        const CNode &a = cur[2 * g], &b = cur[2 * g + 1];
        kg.push_back({a.lo, b.lo, a.npts, b.npts, b.k, b.npts, a.npts, WbigCur.p + wcur[2 * g + 1], Tg.p + offT[g]});
      }
      run_kgemm(kg, kp, Xs.p, N, dim, 0, st);
      std::vector<GemmDesc> gs;
      for (int g = 0; g < np; ++g) {
        const CNode &a = cur[2 * g], &b = cur[2 * g + 1];
        gs.push_back({WbigCur.p + wcur[2 * g], Tg.p + offT[g], nullptr, Sg.p + offS[g], a.k, b.k, a.npts, a.npts,
                      a.npts, 0, a.k, 0, 0});
      }
      run_gemm(std::move(gs), true, false, 1.0, 0.0, st);
      for (int g = 0; g < np; ++g) {
        const int gnode = (1 << (l - 1)) - 1 + g;
        sst_len[gnode] = (int64_t)cur[2 * g].k * cur[2 * g + 1].k;
        sst_off[gnode] = stage(Sstore, sst_used, Sg.p + offS[g], sst_len[gnode]);
      }
    }
    if (l == 1) break;
    // ---- next level: Phi, Z, M of the parents ----
    std::vector<CNode> nxt(np);
    int64_t oZ = 0, oMn = 0;
    for (int g = 0; g < np; ++g) {
      nxt[g] = CNode{};
      nxt[g].lo = cur[2 * g].lo;
      nxt[g].npts = cur[2 * g].npts + cur[2 * g + 1].npts;
      nxt[g].n = cur[2 * g].k + cur[2 * g + 1].k;
      nxt[g].offZ = oZ;
      oZ += (int64_t)nxt[g].n * s;
      nxt[g].offM = oMn;
      oMn += (int64_t)nxt[g].n * nxt[g].n;
    }
    Zn.ensure(oZ);
    Phin.ensure(oZ);
    Mn.ensure(oMn);
    {
      std::vector<GemmDesc> gphi, gz;
      for (int g = 0; g < np; ++g)
        for (int c = 0; c < 2; ++c) {
          const int i = 2 * g + c;
          const int row = c == 0 ? 0 : cur[2 * g].k;
          const int n = cur[i].n, k = cur[i].k, ng = nxt[g].n;
          gphi.push_back({Bb.p + offK[i], php[i], nullptr, Phin.p + nxt[g].offZ + row, k, (int)s, n, n, ldz[i], 0, ng,
                          0, 0});
          gz.push_back({Wb.p + offK[i], zp[i], nullptr, Zn.p + nxt[g].offZ + row, k, (int)s, n, n, ldz[i], 0, ng, 0,
                        0});
        }
      run_gemm(std::move(gphi), true, false, 1.0, 0.0, st);
      run_gemm(std::move(gz), true, false, 1.0, 0.0, st);
      std::vector<GemmDesc> g1, g2;
      for (int g = 0; g < np; ++g) {
        const int r1 = cur[2 * g].k, r2 = cur[2 * g + 1].k, ng = nxt[g].n;
        double* Zg = Zn.p + nxt[g].offZ;
        const double* Pg = Phin.p + nxt[g].offZ;
        // rows of p1 -= S Phi'_p2 ; rows of p2 -= S^T Phi'_p1
        g1.push_back({Sg.p + offS[g], Pg + r1, Zg, Zg, r1, (int)s, r2, r1, ng, ng, ng, 0, 0});
        g2.push_back({Sg.p + offS[g], Pg, Zg + r1, Zg + r1, r2, (int)s, r1, r1, ng, ng, ng, 0, 0});
      }
      run_gemm(std::move(g1), false, false, -1.0, 1.0, st);
      run_gemm(std::move(g2), true, false, -1.0, 1.0, st);
    }
    if (!plain) {  // the parents' diagonal blocks [[Sigma_p1, S], [S^T, Sigma_p2]] (SCALED only)
      std::vector<int64_t> oSig(cnt), oSS(np);
      for (int i = 0; i < cnt; ++i) oSig[i] = offKK[i];
      for (int g = 0; g < np; ++g) oSS[g] = offS[g];
      DevArr<CNode> dpar, dkid;
      DevArr<int64_t> dos, dss;
      dpar.upload(nxt, st);
      dkid.upload(cur, st);
      dos.upload(oSig, st);
      dss.upload(oSS, st);
      hipLaunchKernelGGL(k_cmerge, dim3(np), dim3(256), 0, st, (const CNode*)dpar.p, (const CNode*)dkid.p,
                         (const double*)Sig.p, (const int64_t*)dos.p, (const double*)Sg.p, (const int64_t*)dss.p,
                         Mn.p);
      HSS_HIP(hipGetLastError());
      HSS_HIP(hipStreamSynchronize(st));
    }
    // rotate level state
    prevnodes_npts.assign(cnt, 0);
    prevnodes_k.assign(cnt, 0);
    for (int i = 0; i < cnt; ++i) {
      prevnodes_npts[i] = cur[i].npts;
      prevnodes_k[i] = cur[i].k;
    }
    std::swap(WbigPrev.p, WbigCur.p);
    std::swap(WbigPrev.len, WbigCur.len);
    wprev = wcur;
    std::swap(Mb.p, Mn.p);
    std::swap(Mb.len, Mn.len);
    // the parents' Z and Phi become the current level's (own buffers, ld = n)
    std::swap(Zlvl.p, Zn.p);
    std::swap(Zlvl.len, Zn.len);
    std::swap(Philvl.p, Phin.p);
    std::swap(Philvl.len, Phin.len);
    cur = nxt;
    zp.assign(np, nullptr);
    php.assign(np, nullptr);
    ldz.assign(np, 0);
    for (int g = 0; g < np; ++g) {
      zp[g] = Zlvl.p + nxt[g].offZ;
      php[g] = Philvl.p + nxt[g].offZ;
      ldz[g] = nxt[g].n;
    }
    // Mb holds the parents' blocks packed in order; offM recomputed at the top of the loop matches that packing
  }
  // ---- final layout with the ranks found ----
  for (int k = 1; k < m->nnodes; ++k) m->nodes[k].r = rank[k];
  dev_free(m->dB);
  dev_free(m->dS);
  m->dB = nullptr;
  m->dS = nullptr;
  layout_representation(m);
  std::vector<int64_t> so, doff, ln;
  for (int k = 1; k < m->nnodes; ++k) {
    so.push_back(bst_off[k]);
    doff.push_back(m->nodes[k].offB);
    ln.push_back(bst_len[k]);
  }
  {
    DevArr<int64_t> a, b, c;
    a.upload(so, st);
    b.upload(doff, st);
    c.upload(ln, st);
    hipLaunchKernelGGL(k_copy_blocks, dim3(64, (int)so.size()), dim3(256), 0, st, (const double*)Bstore.p,
                       (const int64_t*)a.p, m->dB, (const int64_t*)b.p, (const int64_t*)c.p);
    HSS_HIP(hipGetLastError());
    HSS_HIP(hipStreamSynchronize(st));
  }
  so.clear();
  doff.clear();
  ln.clear();
  for (int k = 0; k < nleaves - 1; ++k) {
    so.push_back(sst_off[k]);
    doff.push_back(m->nodes[k].offS);
    ln.push_back(sst_len[k]);
  }
  {
    DevArr<int64_t> a, b, c;
    a.upload(so, st);
    b.upload(doff, st);
    c.upload(ln, st);
    hipLaunchKernelGGL(k_copy_blocks, dim3(64, (int)so.size()), dim3(256), 0, st, (const double*)Sstore.p,
                       (const int64_t*)a.p, m->dS, (const int64_t*)b.p, (const int64_t*)c.p);
    HSS_HIP(hipGetLastError());
    HSS_HIP(hipStreamSynchronize(st));
  }
  return true;
}

}  // namespace hss

using namespace hss;

extern "C" hss_status hss_rank_features(hss_ctx_t ctx, const double* d_points, int64_t n, int32_t dim,
                                        int32_t leaf_size, double length, double tol, float* h_out,
                                        int64_t capacity, int64_t* needed) {
  try {
    HSS_CHECK(ctx && d_points && needed, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
    HSS_CHECK(n >= 1 && dim >= 1 && dim <= 3 && leaf_size >= 2, HSS_ERR_INVALID_ARGUMENT, "bad sizes");
    HSS_CHECK(length > 0.0 && tol > 0.0, HSS_ERR_INVALID_ARGUMENT, "need length > 0 and tol > 0");
    int L = 0;
    while (((int64_t)leaf_size << L) < n) ++L;
    HSS_CHECK(L <= 20, HSS_ERR_UNSUPPORTED, "too many levels");
    const int64_t cnt = ((int64_t)2 << L) - 2;
    *needed = cnt * 7;
    if (!h_out) return HSS_OK;
    HSS_CHECK(capacity >= cnt * 7, HSS_ERR_INVALID_ARGUMENT, "output too small");
    if (L == 0) return HSS_OK;
    CtxScope cs_(ctx);
    const std::vector<int64_t> leaf_lo = tree_leaf_lo(n, L);
    std::vector<double> hb((size_t)6 << L);
    {
      DevBuf perm, box;
      perm.ensure(n);  // int64 entries, same size as doubles
      box.ensure((int64_t)hb.size());
      build_tree(ctx->stream, d_points, n, dim, L, (int64_t*)perm.p, box.p);
      HSS_HIP(hipMemcpyAsync(hb.data(), box.p, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, ctx->stream));
      HSS_HIP(hipStreamSynchronize(ctx->stream));
    }
    const std::vector<float> f = node_features(hb, L, leaf_lo, length, tol);
    std::copy(f.begin(), f.end(), h_out);
    return HSS_OK;
  } catch (const hss::Error& e) {
    hss::set_error(e.msg);
    return e.st;
  } catch (...) {
    hss::set_error("unexpected internal exception");
    return HSS_ERR_DEVICE;
  }
}
