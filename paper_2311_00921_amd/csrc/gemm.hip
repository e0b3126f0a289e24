// Batched GEMM on the matrix cores (MFMA 16x16x4 FP64 and FP32, 16x16x16
// BF16) for the contraction steps of the HSS-ULV factorization: the diagonal
// product Q^T A Q in compact WY form (Eq. 7) and the products around it.
//
// One launch covers every node of a stage: grid.y indexes the batch entry,
// grid.x the BM x BN output tiles of that entry. Each 256-thread workgroup
// stages BM x BK slices of op(A) and BK x BN slices of op(B) in LDS; each of
// its four waves owns a (BM/2) x (BN/2) quadrant of the tile as a grid of
// 16x16 MFMA accumulators, computed transposed so that the stores of the
// column-major output coalesce. The tile shape is one of a few compiled variants,
// picked per batch by the autotuner (default 64 x 64).
#include "hss_internal.h"

namespace hss {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

typedef short v4s __attribute__((ext_vector_type(4)));

// BF16 compute types: operands rounded to BF16 (Bf16) or split into two BF16
// parts, x = hi + lo + O(2^-16 |x|) (Bf16x3), multiplied on the BF16 matrix
// cores with FP32 accumulation; Bf16x3 forms hi*hi + hi*lo + lo*hi, which
// leaves out only the lo*lo term.
struct Bf16 {};
struct Bf16x3 {};

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
template <>
struct AccT<Bf16> {
  typedef v4f type;
};
template <>
struct AccT<Bf16x3> {
  typedef v4f type;
};

template <typename TC>
constexpr int kBfParts = 0;  // BF16 parts per operand (0: not a BF16 type)
template <>
constexpr int kBfParts<Bf16> = 1;
template <>
constexpr int kBfParts<Bf16x3> = 2;

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// 16x16x16 BF16: each lane holds 4 consecutive k of its row (A) or column (B)
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// BF16 bits of x, rounded to nearest (through FP32)
__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ double bf16_value(uint16_t h) {
  return (double)__builtin_bit_cast(float, (uint32_t)h << 16);
}


// tile variants: {BM, BN, BK}; the deep-K ones (BK 32 and 64) halve or quarter
// the number of dependent global-load rounds, which is what bounds the small
// GEMMs of the stages with few nodes
// 64x96 and 96x96 fit the r = 96 panels of the workloads without ragged tiles
constexpr int kTileM[kGemmVariants] = {64, 32, 128, 64, 32, 64, 64, 96};
constexpr int kTileN[kGemmVariants] = {64, 32, 64, 128, 32, 64, 96, 96};
constexpr int kTileK[kGemmVariants] = {16, 16, 16, 16, 64, 32, 16, 16};

// Row of the 16x16 MFMA output held by lane `lane` in accumulator slot v.
// FP64 16x16x4 interleaves rows across slots; the FP32-accumulating ones
// (FP32 16x16x4, BF16 16x16x16) stack them.
__device__ __forceinline__ int mfma_row(double, int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int mfma_row(float, int lane, int v) { return 4 * (lane >> 4) + v; }
__device__ __forceinline__ int mfma_row(Bf16, int lane, int v) { return 4 * (lane >> 4) + v; }
__device__ __forceinline__ int mfma_row(Bf16x3, int lane, int v) { return 4 * (lane >> 4) + v; }

// LDS tiles of one K slice. FP64 / FP32: [k][row] of op(A) and [k][col] of
// op(B), one 16x16x4 operand per k row. BF16: [part][row][k] with 4 k of
// a row adjacent (one 8-byte read per lane and 16x16x16 operand); the row
// pitch BK + 4 keeps those reads 8-byte aligned and spreads the 16 rows
// that one read touches over the banks.
// (The one-element row padding of the FP64 / FP32 tiles measured best among 1 and 16.)
template <typename TC, int BM, int BN, int BK, int P = kBfParts<TC>>
struct GemmLds {
  TC A[BK][BM + 1];
  TC B[BK][BN + 1];
};
template <typename TC, int BM, int BN, int BK>
struct GemmLds<TC, BM, BN, BK, 1> {
  alignas(16) uint16_t A[1][BM][BK + 4];
  alignas(16) uint16_t B[1][BN][BK + 4];
};
template <typename TC, int BM, int BN, int BK>
struct GemmLds<TC, BM, BN, BK, 2> {
  alignas(16) uint16_t A[2][BM][BK + 4];
  alignas(16) uint16_t B[2][BN][BK + 4];
};

// Rounds x into the BF16 part(s) at A[.][r][k] of an LDS tile
template <int P, int R, int K>
__device__ __forceinline__ void stage_bf16(uint16_t (&A)[P][R][K], int r, int k, double x) {
  const uint16_t hi = bf16_bits((float)x);
  A[0][r][k] = hi;
  if constexpr (P == 2) A[1][r][k] = bf16_bits((float)(x - bf16_value(hi)));  // x - hi is exact in FP64
}

__device__ __forceinline__ int perm_index(int t, int dim, int r) {
  return r > 0 ? (t < r ? t + (dim - r) : t - r) : t;
}

// Workgroups are dealt to the 8 XCDs round-robin by linear id, and each XCD
// has its own L2. The logical (tile, entry) of a workgroup is chosen so that
// consecutive workgroups of one XCD take consecutive tiles of the same batch
// entry: the panels that the tiles of an entry share are then read from that
// XCD's L2 instead of once per tile from HBM.
__device__ __forceinline__ void xcd_tile(int& tile, int& entry) {
  const int gx = gridDim.x;
  const int total = gx * gridDim.y;
  const int lin = blockIdx.x + blockIdx.y * gx;
  const int q = (total % 8 == 0) ? (lin % 8) * (total / 8) + lin / 8 : lin;
  tile = q % gx;
  entry = q / gx;
}

// T is the storage type of A, B, Cin and C; TC the compute type: the operands
// are rounded to TC as they are staged into LDS, the matrix cores multiply and
// accumulate in TC, and alpha * (product) + beta * Cin is formed in T.
// Waves per SIMD the compiler must leave room for: the 96 x 96 tile would
// otherwise take 244 registers and run two waves per SIMD (three measured 15%
// faster on the leaf rank-2r update).
template <int TileElems>
constexpr int kMinWaves = TileElems >= 96 * 96 ? 3 : 1;

template <typename T, typename TC, bool TA, bool TB, int BM, int BN, int BK>
__global__ __launch_bounds__(256, kMinWaves<BM * BN>) void k_gemm(const GemmDesc* __restrict__ descs, T alpha,
                                                                  T beta) {
  constexpr int IM = BM / 32, JN = BN / 32;  // 16x16 accumulators per wave
  int tile, entry;
  xcd_tile(tile, entry);
  const GemmDesc d = descs[entry];
  const int tilesM = (d.m + BM - 1) / BM;
  const int tilesN = (d.n + BN - 1) / BN;
  if (tile >= tilesM * tilesN) return;
  const int row0 = (tile % tilesM) * BM;
  const int col0 = (tile / tilesM) * BN;
  if (d.lower_only) {
    // output position of index t is t + (dim - r) for t < r, t - r otherwise (r = perm_r, square)
    const int r = d.perm_r, mm = d.m - r;
    const int r1 = min(row0 + BM, d.m) - 1, c1 = min(col0 + BN, d.n) - 1;
    int maxp = -1;
    if (row0 < r) maxp = max(maxp, min(r1, r - 1) + mm);
    if (r1 >= r) maxp = max(maxp, r1 - r);
    const int minp = (c1 >= r) ? max(col0, r) - r : col0 + mm;
    if (maxp < minp) return;  // every element of the tile lies strictly above the diagonal
  }
  constexpr int NP = kBfParts<TC>;
  static_assert(NP == 0 || BK % 16 == 0, "a BF16 K slice holds whole 16x16x16 steps");
  __shared__ GemmLds<TC, BM, BN, BK> lds;
  constexpr int QA = BM * BK / 256, QB = BN * BK / 256;  // elements per thread and K slice
  const T* __restrict__ A = (const T*)d.A;
  const T* __restrict__ B = (const T*)d.B;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid >> 1) * (BM / 2), wn = (wid & 1) * (BN / 2);
  const int lr = lane & 15, lk = lane >> 4;
  // interior tiles (the whole tile inside the output and no partial K slice)
  // load without bounds checks, by pointers stepped once per K slice
  const bool interior = row0 + BM <= d.m && col0 + BN <= d.n && d.k % BK == 0;
  int ar[QA], ak[QA], bc[QB], bk[QB];
  const T* pa[QA];
  const T* pb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int e = q * 256 + tid;
    if (!TA) {
      ar[q] = e % BM;
      ak[q] = e / BM;
    } else {
      ak[q] = e % BK;
      ar[q] = e / BK;
    }
    pa[q] = TA ? A + ak[q] + (int64_t)(row0 + ar[q]) * d.lda : A + (row0 + ar[q]) + (int64_t)ak[q] * d.lda;
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int e = q * 256 + tid;
    if (!TB) {
      bk[q] = e % BK;
      bc[q] = e / BK;
    } else {
      bc[q] = e % BN;
      bk[q] = e / BN;
    }
    pb[q] = TB ? B + (col0 + bc[q]) + (int64_t)bk[q] * d.ldb : B + bk[q] + (int64_t)(col0 + bc[q]) * d.ldb;
  }
  const int64_t sa = TA ? BK : (int64_t)BK * d.lda;
  const int64_t sb = TB ? (int64_t)BK * d.ldb : BK;
  typename AccT<TC>::type acc[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
  T ra[QA], rb[QB];
  auto load = [&](int k0) {
    if (d.kswap > 0) {
      // rotated k index of op(B): the addresses are formed per slice
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        int kr = k0 + bk[q] + d.kswap;
        if (kr >= d.k) kr -= d.k;
        pb[q] = TB ? B + (col0 + bc[q]) + (int64_t)kr * d.ldb : B + kr + (int64_t)(col0 + bc[q]) * d.ldb;
      }
    }
    if (interior) {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        ra[q] = *pa[q];
        pa[q] += sa;
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        rb[q] = *pb[q];
        pb[q] += sb;
      }
    } else {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        ra[q] = (row0 + ar[q] < d.m && k0 + ak[q] < d.k) ? *pa[q] : (T)0;
        pa[q] += sa;
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        rb[q] = (col0 + bc[q] < d.n && k0 + bk[q] < d.k) ? *pb[q] : (T)0;
        pb[q] += sb;
      }
    }
  };
  // software pipeline: the next K slice is fetched into registers while the
  // matrix cores consume the current one from LDS
  if (d.k > 0) load(0);
  for (int k0 = 0; k0 < d.k; k0 += BK) {
    if constexpr (NP == 0) {
#pragma unroll
      for (int q = 0; q < QA; ++q) lds.A[ak[q]][ar[q]] = (TC)ra[q];
#pragma unroll
      for (int q = 0; q < QB; ++q) lds.B[bk[q]][bc[q]] = (TC)rb[q];
    } else {
#pragma unroll
      for (int q = 0; q < QA; ++q) stage_bf16(lds.A, ar[q], ak[q], (double)ra[q]);
#pragma unroll
      for (int q = 0; q < QB; ++q) stage_bf16(lds.B, bc[q], bk[q], (double)rb[q]);
    }
    __syncthreads();
    if (k0 + BK < d.k) load(k0 + BK);
    if constexpr (NP == 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        TC a[IM], b[JN];
#pragma unroll
        for (int i = 0; i < IM; ++i) a[i] = lds.A[kk + lk][wm + 16 * i + lr];
#pragma unroll
        for (int j = 0; j < JN; ++j) b[j] = lds.B[kk + lk][wn + 16 * j + lr];
        // operands swapped: the accumulator holds the transposed 16 x 16 tile,
        // so that lanes run along the output's rows (column-major stores coalesce)
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j) acc[i][j] = mfma16(b[j], a[i], acc[i][j]);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        v4s a[NP][IM], b[NP][JN];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
          for (int i = 0; i < IM; ++i) a[p][i] = *(const v4s*)&lds.A[p][wm + 16 * i + lr][kk + 4 * lk];
#pragma unroll
          for (int j = 0; j < JN; ++j) b[p][j] = *(const v4s*)&lds.B[p][wn + 16 * j + lr][kk + 4 * lk];
        }
        // swapped as above; the small cross terms first
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j) {
            if constexpr (NP == 2) {
              acc[i][j] = mfma16(b[1][j], a[0][i], acc[i][j]);
              acc[i][j] = mfma16(b[0][j], a[1][i], acc[i][j]);
            }
            acc[i][j] = mfma16(b[0][j], a[0][i], acc[i][j]);
          }
      }
    }
    __syncthreads();
  }

  T* __restrict__ C = (T*)d.C;
  const T* __restrict__ Cin = (const T*)d.Cin;
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wm + 16 * i + lr;
        const int col = col0 + wn + 16 * j + mfma_row(TC{}, lane, v);
        if (row < d.m && col < d.n) {
          const int prow = perm_index(row, d.m, d.perm_r);
          const int pcol = perm_index(col, d.n, d.perm_r);
          T val = alpha * (T)acc[i][j][v];
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

thread_local TuneRec* g_tune = nullptr;

static hipEvent_t tune_event(TuneRec* t) {
  if (t->used == t->pool.size()) {
    hipEvent_t e;
    HSS_HIP(hipEventCreate(&e));
    t->pool.push_back(e);
  }
  return t->pool[t->used++];
}

GemmTimer::GemmTimer(const GemmBatch& g, hipStream_t st) {
  if (!g_tune) return;
  t = g_tune;
  s = st;
  hipEvent_t a = tune_event(t);
  b = tune_event(t);
  HSS_HIP(hipEventRecord(a, s));
  t->recs.push_back({&g, a, b});
}

GemmTimer::~GemmTimer() {
  if (t) (void)hipEventRecord(b, s);
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

template <typename T, typename TC, int BM, int BN, int BK>
static void launch_tile(const GemmBatch& b, bool ta, bool tb, T alpha, T beta, hipStream_t s) {
  const int tiles = ((b.mmax + BM - 1) / BM) * ((b.nmax + BN - 1) / BN);
  dim3 grid(tiles, b.count);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, TC, false, false, BM, BN, BK>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, TC, true, false, BM, BN, BK>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, TC, false, true, BM, BN, BK>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  else
    hipLaunchKernelGGL((k_gemm<T, TC, true, true, BM, BN, BK>), grid, dim3(256), 0, s, b.dev, alpha, beta);
  HSS_HIP(hipGetLastError());
}

template <typename T, typename TC>
static void launch(const GemmBatch& b, bool ta, bool tb, T alpha, T beta, hipStream_t s) {
  if (b.count == 0 || b.mmax == 0 || b.nmax == 0) return;
  HSS_CHECK(b.count <= 65535, HSS_ERR_UNSUPPORTED, "too many GEMM batch entries in one launch");
  GemmTimer t(b, s);
#define HSS_TILE(v) launch_tile<T, TC, kTileM[v], kTileN[v], kTileK[v]>(b, ta, tb, alpha, beta, s)
  switch (b.variant) {
    case 1: HSS_TILE(1); break;
    case 2: HSS_TILE(2); break;
    case 3: HSS_TILE(3); break;
    case 4: HSS_TILE(4); break;
    case 5: HSS_TILE(5); break;
    case 6: HSS_TILE(6); break;
    case 7: HSS_TILE(7); break;
    default: HSS_TILE(0); break;
  }
#undef HSS_TILE
}

void gemm_launch_f64(const GemmBatch& b, bool ta, bool tb, double alpha, double beta, hipStream_t s) {
  switch (b.compute) {
    case HSS_P_FP32: launch<double, float>(b, ta, tb, alpha, beta, s); break;
    case HSS_P_BF16: launch<double, Bf16>(b, ta, tb, alpha, beta, s); break;
    case HSS_P_BF16X3: launch<double, Bf16x3>(b, ta, tb, alpha, beta, s); break;
    default: launch<double, double>(b, ta, tb, alpha, beta, s); break;
  }
}
void gemm_launch_f32(const GemmBatch& b, bool ta, bool tb, float alpha, float beta, hipStream_t s) {
  launch<float, float>(b, ta, tb, alpha, beta, s);
}

}  // namespace hss
