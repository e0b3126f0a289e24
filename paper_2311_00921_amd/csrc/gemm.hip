// Batched GEMM on the matrix cores (MFMA 16x16x4, FP64 and FP32) for the
// contraction steps of the HSS-ULV factorization: the diagonal product
// Q^T A Q in compact WY form (Eq. 7) and the products around it.
//
// One launch covers every node of a level: grid.y indexes the batch entry,
// grid.x the 64x64 output tiles of that entry. Each 256-thread workgroup
// stages 64x16 slices of op(A) and 16x64 slices of op(B) in LDS; each of its
// four waves owns a 32x32 quadrant of the tile as 2x2 MFMA accumulators.
#include "hss_internal.h"

namespace hss {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct AccT;
template <>
struct AccT<double> {
  typedef v4d type;
};
template <>
struct AccT<float> {
  typedef v4f type;
};

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int BM = 64, BN = 64, BK = 16;

// Row of the 16x16 MFMA output held by lane `lane` in accumulator slot v.
// FP64 16x16x4 interleaves rows across slots; FP32 16x16x4 stacks them.
__device__ __forceinline__ int mfma_row(double, int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int mfma_row(float, int lane, int v) { return 4 * (lane >> 4) + v; }

__device__ __forceinline__ int perm_index(int t, int dim, int r) {
  return r > 0 ? (t < r ? t + (dim - r) : t - r) : t;
}

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs, T alpha, T beta) {
  const GemmDesc d = descs[blockIdx.y];
  const int tilesM = (d.m + BM - 1) / BM;
  const int tilesN = (d.n + BN - 1) / BN;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int row0 = (blockIdx.x % tilesM) * BM;
  const int col0 = (blockIdx.x / tilesM) * BN;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const T* __restrict__ A = (const T*)d.A;
  const T* __restrict__ B = (const T*)d.B;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  typename AccT<T>::type acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int k0 = 0; k0 < d.k; k0 += BK) {
#pragma unroll
    for (int e0 = 0; e0 < BM * BK; e0 += 256) {
      const int e = e0 + tid;
      int r, kk;
      if (!TA) {
        r = e % BM;
        kk = e / BM;
      } else {
        kk = e % BK;
        r = e / BK;
      }
      const int gr = row0 + r, gk = k0 + kk;
      T v = 0;
      if (gr < d.m && gk < d.k)
        v = TA ? A[gk + (int64_t)gr * d.lda] : A[gr + (int64_t)gk * d.lda];
      As[kk][r] = v;
    }
#pragma unroll
    for (int e0 = 0; e0 < BN * BK; e0 += 256) {
      const int e = e0 + tid;
      int c, kk;
      if (!TB) {
        kk = e % BK;
        c = e / BK;
      } else {
        c = e % BN;
        kk = e / BN;
      }
      const int gc = col0 + c, gk = k0 + kk;
      T v = 0;
      if (gc < d.n && gk < d.k)
        v = TB ? B[gc + (int64_t)gk * d.ldb] : B[gk + (int64_t)gc * d.ldb];
      Bs[kk][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lk][wn + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

  T* __restrict__ C = (T*)d.C;
  const T* __restrict__ Cin = (const T*)d.Cin;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wm + 16 * i + mfma_row((T)0, lane, v);
        const int col = col0 + wn + 16 * j + lr;
        if (row < d.m && col < d.n) {
          const int prow = perm_index(row, d.m, d.perm_r);
          const int pcol = perm_index(col, d.n, d.perm_r);
          T val = alpha * acc[i][j][v];
          if (beta != (T)0) {
            const int irow = d.perm_in ? prow : row;
            const int icol = d.perm_in ? pcol : col;
            val += beta * Cin[irow + (int64_t)icol * d.ldcin];
          }
          C[prow + (int64_t)pcol * d.ldc] = val;
          if (d.C2) ((T*)d.C2)[prow + (int64_t)pcol * d.ldc] = val;
        }
      }
}

void gemm_upload(GemmBatch& b, hipStream_t s) {
  b.count = (int32_t)b.host.size();
  b.mmax = b.nmax = 0;
  for (auto& g : b.host) {
    b.mmax = std::max(b.mmax, g.m);
    b.nmax = std::max(b.nmax, g.n);
  }
  if (b.dev) dev_free(b.dev);
  b.dev = nullptr;
  if (b.count == 0) return;
  b.dev = (GemmDesc*)dev_alloc(sizeof(GemmDesc) * b.count);
  HSS_HIP(hipMemcpyAsync(b.dev, b.host.data(), sizeof(GemmDesc) * b.count, hipMemcpyHostToDevice, s));
}

void gemm_free(GemmBatch& b) {
  if (b.dev) dev_free(b.dev);
  b.dev = nullptr;
}

template <typename T>
static void launch(const GemmBatch& b, bool ta, bool tb, T alpha, T beta, hipStream_t s) {
  if (b.count == 0 || b.mmax == 0 || b.nmax == 0) return;
  const int tiles = ((b.mmax + BM - 1) / BM) * ((b.nmax + BN - 1) / BN);
  HSS_CHECK(b.count <= 65535, HSS_ERR_UNSUPPORTED, "too many GEMM batch entries in one launch");
  dim3 grid(tiles, b.count);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, false, false>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, true, false>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, false, true>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  HSS_HIP(hipGetLastError());
}

void gemm_launch_f64(const GemmBatch& b, bool ta, bool tb, double alpha, double beta, hipStream_t s) {
  launch<double>(b, ta, tb, alpha, beta, s);
}
void gemm_launch_f32(const GemmBatch& b, bool ta, bool tb, float alpha, float beta, hipStream_t s) {
  launch<float>(b, ta, tb, alpha, beta, s);
}

}  // namespace hss
