// BLR^2-ULV (Sec. 3.1, Alg. 1) of an HSS matrix viewed at its leaf level.
//
// The leaf blocks with their shared bases U_i form a weakly admissible BLR^2
// matrix: the block between leaves i and j is U_i S_ij U_j^T, where S_ij is the
// coupling of their lowest common ancestor expressed in the leaves' own bases
// through the transfer matrices below it (the nested basis of Eq. 6).
//
//   1. Diagonal product and partial Cholesky of every leaf (Eq. 7, 10-12): the
//      leaf stage of the HSS-ULV, same kernels.
//   2. Permutation of every leaf's skeleton rows to the end (Eq. 13): the K x K
//      skeleton matrix (K = sum of the leaf ranks), Sg Sigma_i Sg on its
//      diagonal blocks and Phi_c1 S Phi_c2^T between the leaves under the two
//      children of each node, Phi_c being the product of the transfer matrices
//      from c down to its leaves (Phi = E one level above the leaves).
//   3. Dense Cholesky of the skeleton matrix: right-looking, 64-column panels
//      in outer blocks of four; each diagonal block is factored and inverted by
//      one wave in registers, the panel below is multiplied by that inverse in
//      place (rows independent), and the lower triangle right of the panel is
//      updated by the FP64 MFMA GEMM: inside the outer block per panel, after
//      it with the block's full depth, the part beyond the next block on a
//      second stream while the next block is factored (a lookahead of one
//      block).
//   Solve (Eq. 14): the leaf forward sweep, the two dense triangular solves
//   (panel by panel, with the inverted diagonal blocks), the leaf backward sweep.
//
// The skeleton matrix takes K^2 doubles and its Cholesky K^3 / 3 flops: the
// variant exists to show what the nested basis of the HSS-ULV saves, and is
// limited to K <= 65536 (32 GiB).
#include <algorithm>
#include <cmath>

#include "hss_internal.h"

namespace hss {

constexpr int DNB = 64;                // panel width of the skeleton Cholesky
constexpr int DOB = 4;                 // panels per outer block (trailing updates of depth 4 DNB)
constexpr int64_t kBlr2MaxK = 65536;   // skeleton rows
constexpr int kSolveCols = 16;         // right-hand sides per dense-solve pass

struct Blr2State {
  bool valid = false;
  int64_t K = 0;
  int npanel = 0;
  std::vector<int64_t> offK;   // per node: first skeleton row of its leftmost leaf
  std::vector<int64_t> rows;   // per node: skeleton rows below it (sum of its leaves' ranks)
  int64_t* doffK = nullptr;    // device copy of offK
  double* dK = nullptr;        // K x K, lower triangle: the skeleton matrix, then its Cholesky factor
  double* dLinv = nullptr;     // npanel blocks of DNB x DNB: inverses of the factor's diagonal blocks
  double* dPhi = nullptr;      // Phi of the nodes two or more levels above the leaves
  double* dG = nullptr;        // per coupling above the leaves' parents: Phi_c2 S^T
  double* dpanel = nullptr;    // per panel: sum of the log pivots
  int32_t* dinfo = nullptr;    // [0] failed, [1] first failing skeleton row
  double* dlog = nullptr;      // [0] log-determinant
  std::vector<int64_t> offPhi, offG;  // per node
  std::vector<GemmBatch> phi;  // per tree level, deepest first
  std::vector<GemmBatch> g1, g2;  // per tree level of the coupling's node: G = Phi_c2 S^T, block = G Phi_c1^T
  // Cholesky updates, launched as single-entry views: inside an outer block, each
  // panel's update of the block's later columns (all rows below); after the
  // block, the update of depth DOB * DNB of the next block's columns (tnext) and
  // of the rest of the trailing matrix (trest, on the second stream)
  GemmBatch inblk, tnext, trest;
  std::vector<int> inblk_of, tnext_of, trest_of;  // per panel / per outer block: entry index or -1
  hipEvent_t ev_block = nullptr;  // an outer block's panels are factored
  hipEvent_t ev_rest = nullptr;   // the rest of the trailing matrix is updated
  double* dZ = nullptr;        // solve: K x kSolveCols each
  double* dY = nullptr;
  double* dW = nullptr;
  double logdet = 0.0;
  float factor_ms = 0.f;
};

namespace {

// Copies the merged block of each node of the leaves' parents' stage into the
// skeleton matrix at its leftmost leaf's skeleton row (the block is n x n with
// n the sum of its two leaves' ranks, so it lands on the diagonal).
__global__ __launch_bounds__(256) void k_blr2_diag(const NodeDesc* __restrict__ nodes, int first,
                                                   const double* __restrict__ Mb, const int64_t* __restrict__ offK,
                                                   double* __restrict__ Kmat, int64_t K) {
  const int p = first + blockIdx.x;
  const NodeDesc nd = nodes[p];
  const int n = nd.n;
  const double* M = Mb + nd.offM;
  double* dst = Kmat + offK[p] * (K + 1);
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 256) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i >= j) dst[i + j * K] = M[e];
  }
}

// Value of v held by lane l (l wave-uniform), through scalar registers.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Cholesky of the diagonal block (k0, k0) of order jb <= 64, then its inverse,
// by one workgroup of four waves, the block in LDS (rows and columns past jb
// padded with the identity, so every step runs unmasked).
//   Factor, blocked by 16 columns: wave 0 factors a panel with lane i holding
//   row i's 16 panel entries in registers (the pivot from lane j, each later
//   panel column c taking L(c, j) from lane c), then the four waves update the
//   lower triangle right of the panel from LDS. A step of the serial chain
//   touches at most 16 columns.
//   Inverse X = L^{-1} by columns, forward substitution L x = e_j with four
//   threads per column (thread part p sums the terms q = p, p + 4, ...; two
//   shuffles complete each sum); L and X are read from LDS, and x_i is written
//   there by the thread of part i mod 4 (the four threads of a column share a
//   wave, whose LDS accesses stay in order).
// Writes L back (lower triangle), L^{-1} into Linv (64 x 64, zero above the
// diagonal and past jb), the sum of log pivots into *pld. A non-positive pivot
// is recorded (the first failing row over all panels) and replaced by 1.
__global__ __launch_bounds__(256) void k_dchol_diag(double* __restrict__ A, int64_t lda, int64_t k0, int jb,
                                                    double* __restrict__ Linv, double* __restrict__ pld,
                                                    int32_t* __restrict__ info) {
  constexpr int PW = 16;               // panel width
  __shared__ double Ls[DNB][DNB + 1];  // Ls[row][col]: the block, then L (zero above the diagonal)
  __shared__ double Xs[DNB][DNB + 1];  // Xs[row][col] = Linv(row, col)
  __shared__ double rdg[DNB];          // 1 / L(i, i)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double* Ab = A + k0 + k0 * lda;
  {
    double v[DNB / 4];
#pragma unroll
    for (int u = 0; u < DNB / 4; ++u) {
      const int c = wv + 4 * u;
      v[u] = (lane < jb && c < jb && lane >= c) ? Ab[lane + c * lda] : (lane == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < DNB / 4; ++u) {
      Ls[lane][wv + 4 * u] = v[u];
      Xs[lane][wv + 4 * u] = 0.0;
    }
  }
  __syncthreads();
  int bad = -1;       // wave 0
  double mine = 1.0;  // wave 0: lane i's pivot
#pragma unroll 1
  for (int j0 = 0; j0 < DNB; j0 += PW) {
    if (wv == 0) {
      const int i = lane;
      double a[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) a[c] = Ls[i][j0 + c];
#pragma unroll
      for (int k = 0; k < PW; ++k) {
        double d = lane_value(a[k], j0 + k);
        if (!(d > 0.0)) {
          if (bad < 0) bad = j0 + k;
          d = 1.0;
        }
        const double piv = sqrt(d);
        const double rs = 1.0 / piv;
        const bool me = i == j0 + k;
        a[k] = me ? piv : a[k] * rs;
        mine = me ? piv : mine;
        if (me) rdg[i] = rs;
#pragma unroll
        for (int c = k + 1; c < PW; ++c) a[c] -= a[k] * lane_value(a[k], j0 + c);
      }
      if (i >= j0)
#pragma unroll
        for (int c = 0; c < PW; ++c) Ls[i][j0 + c] = (j0 + c <= i) ? a[c] : 0.0;
    }
    __syncthreads();
    // lower triangle right of the panel: Ls[r][c] -= sum_k L(r, j0 + k) L(c, j0 + k)
    const int n2 = DNB - j0 - PW;
    for (int e = t; e < n2 * n2; e += 256) {
      const int rr = j0 + PW + e % n2, cc = j0 + PW + e / n2;
      if (rr >= cc) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < PW; ++k) sum += Ls[rr][j0 + k] * Ls[cc][j0 + k];
        Ls[rr][cc] -= sum;
      }
    }
    __syncthreads();
  }
  if (wv == 0) {
    if (bad >= 0 && lane == 0) {
      atomicMin(&info[1], (int32_t)(k0 + bad));
      atomicExch(&info[0], 1);
    }
    double lg = lane < jb ? log(mine) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lg += __shfl_xor(lg, o, 64);
    if (lane == 0) *pld = 2.0 * lg;
  }
  {
    const int j = t >> 2, p = t & 3;
#pragma unroll 1
    for (int i = j; i < DNB; ++i) {  // x_i = 0 above the diagonal (Xs starts at zero)
      double sum = 0.0;
#pragma unroll
      for (int u = 0; u < DNB / 4; ++u) sum += Ls[i][p + 4 * u] * Xs[p + 4 * u][j];  // L(i, q) = 0 for q >= i
      sum += __shfl_xor(sum, 1, 4);
      sum += __shfl_xor(sum, 2, 4);
      if ((i & 3) == p) Xs[i][j] = ((i == j ? 1.0 : 0.0) - sum) * rdg[i];
      __builtin_amdgcn_wave_barrier();  // the column's other threads read x_i at the next step
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < DNB / 4; ++u) {
    const int c = wv + 4 * u;
    if (lane < jb && c < jb && c <= lane) Ab[lane + c * lda] = Ls[lane][c];
    Linv[lane + c * DNB] = (lane < jb && c < jb) ? Xs[lane][c] : 0.0;
  }
}

// The panel below the diagonal block: rows k0 + jb + 64 b .. of columns
// k0 .. k0 + jb, multiplied in place by L_kk^{-T} (L21 = A21 L11^{-T}).
__global__ __launch_bounds__(256) void k_dtrsm_rows(double* __restrict__ A, int64_t lda, int64_t K, int64_t k0,
                                                    int jb, const double* __restrict__ Linv) {
  __shared__ double sa[DNB][DNB + 1];  // sa[col][row]
  __shared__ double sl[DNB][DNB + 1];  // sl[col][row] = Linv(row, col)
  const int t = threadIdx.x;
  const int64_t r0 = k0 + jb + (int64_t)blockIdx.x * DNB;
  const int nr = (int)std::min<int64_t>(DNB, K - r0);
  double* P = A + r0 + k0 * lda;
  for (int e = t; e < DNB * DNB; e += 256) {
    const int i = e % DNB, j = e / DNB;
    sa[j][i] = (i < nr && j < jb) ? P[i + j * lda] : 0.0;
    sl[j][i] = Linv[i + j * DNB];
  }
  __syncthreads();
  // out(i, c) = sum_{q <= c} A21(i, q) Linv(c, q)
  double out[DNB * DNB / 256];
#pragma unroll
  for (int u = 0; u < DNB * DNB / 256; ++u) {
    const int e = t + 256 * u, i = e % DNB, c = e / DNB;
    double s = 0.0;
    for (int q = 0; q <= c; ++q) s += sa[q][i] * sl[q][c];
    out[u] = s;
  }
#pragma unroll
  for (int u = 0; u < DNB * DNB / 256; ++u) {
    const int e = t + 256 * u, i = e % DNB, c = e / DNB;
    if (i < nr && c < jb) P[i + c * lda] = out[u];
  }
}

// Forward solve with the skeleton factor, panel k: y_k = Linv_k z_k (every
// workgroup forms it from an LDS copy of Linv_k; workgroup 0 stores it in Y),
// then z_i -= L(i, panel) y_k for the 64 rows of the workgroup below the panel:
// thread (row r, group g) accumulates the 4 right-hand sides 4g .. 4g + 3.
__global__ __launch_bounds__(256) void k_dtrsv_fwd(const double* __restrict__ A, int64_t lda, int64_t K, int64_t k0,
                                                   int jb, const double* __restrict__ Linv, double* __restrict__ Z,
                                                   double* __restrict__ Y, int nc) {
  constexpr int CG = kSolveCols / 4;
  static_assert(CG * 64 == 256, "four column groups of four right-hand sides");
  __shared__ double lq[DNB][DNB + 1];  // lq[q][i] = Linv(i, q)
  __shared__ double zk[DNB][kSolveCols];
  __shared__ double yk[DNB][kSolveCols];
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  for (int e = t; e < DNB * DNB; e += 256) lq[e / DNB][e % DNB] = Linv[e];
  for (int e = t; e < DNB * kSolveCols; e += 256) {
    const int i = e % DNB, c = e / DNB;
    zk[i][c] = (i < jb && c < nc) ? Z[k0 + i + c * K] : 0.0;
  }
  __syncthreads();
  {
    double y[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int q = 0; q < DNB; ++q) {  // Linv is zero above its diagonal and past jb
      const double l = lq[q][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] += l * zk[q][4 * g + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) yk[r][4 * g + c] = y[c];
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = t; e < DNB * kSolveCols; e += 256) {
      const int i = e % DNB, c = e / DNB;
      if (i < jb && c < nc) Y[k0 + i + c * K] = yk[i][c];
    }
  const int64_t row = k0 + jb + (int64_t)blockIdx.x * 64 + r;
  if (row >= K) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const double* L = A + row + k0 * lda;
#pragma unroll 16
  for (int q = 0; q < DNB; ++q) {
    const double l = q < jb ? L[q * lda] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += l * yk[q][4 * g + c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (4 * g + c < nc) Z[row + (4 * g + c) * K] -= acc[c];
}

// Backward solve with the skeleton factor, panel k: w_k = Linv_k^T y_k (every
// workgroup forms it from an LDS copy of Linv_k; workgroup 0 stores it in W),
// then y_j -= L(panel, j)^T w_k for the 64 rows j < k0 of the workgroup, one
// column of L per 4-lane group (lane s reads the panel rows s, s + 4, ...).
__global__ __launch_bounds__(256) void k_dtrsv_bwd(const double* __restrict__ A, int64_t lda, int64_t K, int64_t k0,
                                                   int jb, const double* __restrict__ Linv, double* __restrict__ Y,
                                                   double* __restrict__ W, int nc) {
  static_assert(kSolveCols == 16, "four lanes of four right-hand sides per column of L");
  __shared__ double lt[DNB][DNB + 1];  // lt[q][i] = Linv(q, i)
  __shared__ double yk[DNB][kSolveCols];
  __shared__ double wk[DNB][kSolveCols + 1];
  const int t = threadIdx.x;
  for (int e = t; e < DNB * DNB; e += 256) lt[e % DNB][e / DNB] = Linv[e];
  for (int e = t; e < DNB * kSolveCols; e += 256) {
    const int i = e % DNB, c = e / DNB;
    yk[i][c] = (i < jb && c < nc) ? Y[k0 + i + c * K] : 0.0;
  }
  __syncthreads();
  {
    const int r = t & 63, g = t >> 6;
    double w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int q = 0; q < DNB; ++q) {  // Linv is zero above its diagonal and past jb
      const double l = lt[q][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] += l * yk[q][4 * g + c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) wk[r][4 * g + c] = w[c];
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = t; e < DNB * kSolveCols; e += 256) {
      const int i = e % DNB, c = e / DNB;
      if (i < jb && c < nc) W[k0 + i + c * K] = wk[i][c];
    }
  const int sub = t & 3;
  const int64_t j = (int64_t)blockIdx.x * 64 + (t >> 2);
  if (j >= k0) return;
  double acc[kSolveCols];
#pragma unroll
  for (int c = 0; c < kSolveCols; ++c) acc[c] = 0.0;
  const double* L = A + k0 + j * lda;
#pragma unroll
  for (int u = 0; u < DNB / 4; ++u) {
    const int q = sub + 4 * u;
    const double l = q < jb ? L[q] : 0.0;
#pragma unroll
    for (int c = 0; c < kSolveCols; ++c) acc[c] += l * wk[q][c];
  }
#pragma unroll
  for (int c = 0; c < kSolveCols; ++c) {
    acc[c] += __shfl_xor(acc[c], 1, 4);
    acc[c] += __shfl_xor(acc[c], 2, 4);
  }
  // lane s of the group stores right-hand sides 4 s .. 4 s + 3
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const double v = sub == 0 ? acc[cc] : sub == 1 ? acc[4 + cc] : sub == 2 ? acc[8 + cc] : acc[12 + cc];
    const int c = 4 * sub + cc;
    if (c < nc) Y[j + c * K] -= v;
  }
}

// Skeleton vector <-> the per-node vector slots of the leaves' parents (the
// slot of node p holds n_p rows per right-hand side, n_p = sum of its two
// leaves' ranks, in the order of the merged block).
__global__ __launch_bounds__(256) void k_blr2_gather(const NodeDesc* __restrict__ nodes, int first,
                                                     const int64_t* __restrict__ offK, const double* __restrict__ vec,
                                                     int64_t nrhs, int64_t c0, int nc, double* __restrict__ Z,
                                                     int64_t K, int to_slots) {
  const int p = first + blockIdx.x;
  const NodeDesc nd = nodes[p];
  const int n = nd.n;
  double* slot = (double*)vec + nd.offVec * nrhs;
  for (int e = threadIdx.x; e < n * nc; e += 256) {
    const int i = e % n, c = e / n;
    double* zp = Z + offK[p] + i + (int64_t)c * K;
    double* sp = slot + i + (c0 + c) * n;
    if (to_slots)
      *sp = *zp;
    else
      *zp = *sp;
  }
}

__global__ void k_blr2_logdet(const double* __restrict__ node_ld, int nnodes, const double* __restrict__ panel_ld,
                              int npanel, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nnodes; i += 256) s += node_ld[i];
  for (int i = threadIdx.x; i < npanel; i += 256) s += panel_ld[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_blr2_clear(int32_t* info) {
  info[0] = 0;
  info[1] = 0x7fffffff;
}

// The nodes of stage si (a contiguous range of node indices).
struct Range {
  int first, count;
};

// Checks the tree shape BLR^2 needs: one system, at least one level, every
// leaf in the first stage with its parent in the second.
void check_shape(hss_matrix_t m) {
  HSS_CHECK(m->nsys == 1, HSS_ERR_UNSUPPORTED, "BLR^2-ULV: one system only (not a batch)");
  HSS_CHECK(m->stages.size() >= 2, HSS_ERR_UNSUPPORTED, "BLR^2-ULV: the tree needs at least one level");
  const LevelPlan& l0 = m->stages[0];
  const LevelPlan& l1 = m->stages[1];
  int leaves = 0;
  for (const NodeDesc& d : m->nodes) leaves += d.c1 < 0 ? 1 : 0;
  HSS_CHECK(l0.leaf && l0.count == leaves && l0.root_first == l0.first + l0.count, HSS_ERR_UNSUPPORTED,
            "BLR^2-ULV: every leaf must sit on the deepest level");
  for (int p = l1.first; p < l1.first + l1.count; ++p) {
    const NodeDesc& d = m->nodes[p];
    HSS_CHECK(d.c1 >= 0 && m->nodes[d.c1].c1 < 0 && m->nodes[d.c2].c1 < 0, HSS_ERR_UNSUPPORTED,
              "BLR^2-ULV: the second stage must hold the leaves' parents");
  }
}

// Skeleton row offsets: the leaves in point order, each with its rank; a node's
// range is its leaves' (children's ranges are contiguous, first child first).
void skeleton_offsets(hss_matrix_t m, Blr2State& st) {
  const int nn = m->nnodes;
  st.offK.assign(nn, 0);
  st.rows.assign(nn, 0);
  std::vector<int> leaves;
  for (int k = 0; k < nn; ++k)
    if (m->nodes[k].c1 < 0) leaves.push_back(k);
  std::sort(leaves.begin(), leaves.end(), [&](int a, int b) { return m->nodes[a].lo < m->nodes[b].lo; });
  int64_t o = 0;
  for (int k : leaves) {
    st.offK[k] = o;
    st.rows[k] = m->nodes[k].r;
    o += m->nodes[k].r;
  }
  st.K = o;
  // parents after children: deepest levels first
  std::vector<int> order(nn);
  for (int k = 0; k < nn; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return m->nodes[a].level > m->nodes[b].level; });
  for (int k : order) {
    const NodeDesc& d = m->nodes[k];
    if (d.c1 < 0) continue;
    HSS_CHECK(st.offK[d.c1] + st.rows[d.c1] == st.offK[d.c2], HSS_ERR_UNSUPPORTED,
              "BLR^2-ULV: a node's leaves are not contiguous in point order");
    st.offK[k] = st.offK[d.c1];
    st.rows[k] = st.rows[d.c1] + st.rows[d.c2];
  }
}

void alloc_state(hss_matrix_t m, Blr2State& st) {
  hipStream_t s = m->ctx->stream;
  skeleton_offsets(m, st);
  const int64_t K = st.K;
  HSS_CHECK(K >= 1, HSS_ERR_UNSUPPORTED, "BLR^2-ULV: no skeleton rows");
  HSS_CHECK(K <= kBlr2MaxK, HSS_ERR_UNSUPPORTED,
            "BLR^2-ULV: the skeleton matrix would have " + std::to_string(K) + " rows, above the limit of " +
                std::to_string(kBlr2MaxK));
  st.npanel = (int)((K + DNB - 1) / DNB);
  const int nn = m->nnodes;
  const int L = m->L;
  // Phi of the nodes whose level is at most L - 2 (excluding the root) and G of
  // every coupling node at level <= L - 2
  st.offPhi.assign(nn, -1);
  st.offG.assign(nn, -1);
  int64_t lenPhi = 0, lenG = 0;
  for (int k = 0; k < nn; ++k) {
    const NodeDesc& d = m->nodes[k];
    if (d.parent >= 0 && d.level <= L - 2) {
      st.offPhi[k] = lenPhi;
      lenPhi += st.rows[k] * d.r;
    }
    if (d.c1 >= 0 && d.level <= L - 2) {
      st.offG[k] = lenG;
      lenG += st.rows[d.c2] * m->nodes[d.c1].r;
    }
  }
  st.dK = (double*)dev_alloc(sizeof(double) * K * K);
  HSS_HIP(hipMemsetAsync(st.dK, 0, sizeof(double) * K * K, s));
  st.dLinv = (double*)dev_alloc(sizeof(double) * (int64_t)st.npanel * DNB * DNB);
  st.dPhi = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(lenPhi, 1));
  st.dG = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(lenG, 1));
  st.dpanel = (double*)dev_alloc(sizeof(double) * st.npanel);
  st.dinfo = (int32_t*)dev_alloc(sizeof(int32_t) * 2);
  st.dlog = (double*)dev_alloc(sizeof(double));
  st.dZ = (double*)dev_alloc(sizeof(double) * K * kSolveCols * 3);
  st.dY = st.dZ + K * kSolveCols;
  st.dW = st.dY + K * kSolveCols;
  // the node offsets on the device (read by the copy kernels)
  st.doffK = (int64_t*)dev_alloc(sizeof(int64_t) * nn);
  HSS_HIP(hipMemcpyAsync(st.doffK, st.offK.data(), sizeof(int64_t) * nn, hipMemcpyHostToDevice, s));
  const double* B = m->dB;
  const double* S = m->dS;
  // Phi_c = [Phi_c1 E_c[:r1, :]; Phi_c2 E_c[r1:, :]], levels L - 2 .. 1; the
  // leaves' parents (level L - 1) use E itself
  auto phi_of = [&](int c, int& ld) -> const double* {
    const NodeDesc& d = m->nodes[c];
    if (d.level == L - 1) {
      ld = d.n;
      return B + d.offB;
    }
    ld = (int)st.rows[c];
    return st.dPhi + st.offPhi[c];
  };
  st.phi.assign(std::max(L - 1, 0), GemmBatch{});
  st.g1.assign(std::max(L - 1, 0), GemmBatch{});
  st.g2.assign(std::max(L - 1, 0), GemmBatch{});
  for (int k = 0; k < nn; ++k) {
    const NodeDesc& d = m->nodes[k];
    if (d.c1 < 0) continue;
    if (d.parent >= 0 && d.level <= L - 2) {
      const int r1 = m->nodes[d.c1].r;
      int ld1 = 0, ld2 = 0;
      const double* P1 = phi_of(d.c1, ld1);
      const double* P2 = phi_of(d.c2, ld2);
      double* P = st.dPhi + st.offPhi[k];
      const int rows1 = (int)st.rows[d.c1], rows2 = (int)st.rows[d.c2], rows = (int)st.rows[k];
      const double* E = B + d.offB;
      auto& g = st.phi[L - 2 - d.level];
      g.host.push_back({P1, E, nullptr, P, rows1, d.r, r1, ld1, d.n, 0, rows, 0, 0});
      g.host.push_back({P2, E + r1, nullptr, P + rows1, rows2, d.r, m->nodes[d.c2].r, ld2, d.n, 0, rows, 0, 0});
    }
    if (d.level <= L - 2) {
      const int r1 = m->nodes[d.c1].r, r2 = m->nodes[d.c2].r;
      int ld1 = 0, ld2 = 0;
      const double* P1 = phi_of(d.c1, ld1);
      const double* P2 = phi_of(d.c2, ld2);
      const int rows1 = (int)st.rows[d.c1], rows2 = (int)st.rows[d.c2];
      double* G = st.dG + st.offG[k];
      // G = Phi_c2 S^T (S is r1 x r2), then the block (c2 rows, c1 columns) = G Phi_c1^T
      st.g1[L - 2 - d.level].host.push_back({P2, S + d.offS, nullptr, G, rows2, r1, r2, ld2, r1, 0, rows2, 0, 0});
      double* C = st.dK + st.offK[d.c2] + st.offK[d.c1] * K;
      st.g2[L - 2 - d.level].host.push_back({G, P1, nullptr, C, rows2, rows1, r1, rows2, ld1, 0, (int)K, 0, 0});
    }
  }
  for (auto& g : st.phi) gemm_upload(g, s);
  for (auto& g : st.g1) gemm_upload(g, s);
  for (auto& g : st.g2) gemm_upload(g, s);
  // updates of the Cholesky, A22 -= L21 L21^T (lower triangle): within an outer
  // block of DOB panels, panel k updates the block's columns right of it over all
  // rows below; after the block, the trailing matrix is updated with depth the
  // block's width in two parts, the next block's columns and the rest
  st.inblk_of.assign(st.npanel, -1);
  const int nblock = (st.npanel + DOB - 1) / DOB;
  st.tnext_of.assign(nblock, -1);
  st.trest_of.assign(nblock, -1);
  for (int k = 0; k < st.npanel; ++k) {
    const int64_t k0 = (int64_t)k * DNB;
    const int jb = (int)std::min<int64_t>(DNB, K - k0);
    const int64_t bend = std::min<int64_t>((int64_t)(k / DOB + 1) * DOB * DNB, K);  // end of this panel's block
    const int64_t cols = bend - k0 - jb, rows = K - k0 - jb;
    if (cols <= 0 || rows <= 0) continue;
    const double* Lp = st.dK + (k0 + jb) + k0 * K;
    double* C = st.dK + (k0 + jb) * (K + 1);
    st.inblk_of[k] = (int)st.inblk.host.size();
    st.inblk.host.push_back({Lp, Lp, C, C, (int)rows, (int)cols, jb, (int)K, (int)K, (int)K, (int)K, 0, 0, nullptr, 1});
  }
  for (int q = 0; q < nblock; ++q) {
    const int64_t b0 = (int64_t)q * DOB * DNB, bend = std::min<int64_t>(b0 + DOB * DNB, K);
    const int64_t rem = K - bend;
    if (rem <= 0) continue;
    const int64_t w = std::min<int64_t>(DOB * DNB, rem);  // the next block's width
    const int kd = (int)(bend - b0);
    const double* Lp = st.dK + bend + b0 * K;
    double* C = st.dK + bend * (K + 1);
    st.tnext_of[q] = (int)st.tnext.host.size();
    st.tnext.host.push_back({Lp, Lp, C, C, (int)rem, (int)w, kd, (int)K, (int)K, (int)K, (int)K, 0, 0, nullptr, 1});
    const int64_t rr = rem - w;
    if (rr <= 0) continue;
    const double* Lr = Lp + w;
    double* Cr = C + w * (K + 1);
    st.trest_of[q] = (int)st.trest.host.size();
    st.trest.host.push_back({Lr, Lr, Cr, Cr, (int)rr, (int)rr, kd, (int)K, (int)K, (int)K, (int)K, 0, 0, nullptr, 1});
  }
  gemm_upload(st.inblk, s);
  gemm_upload(st.tnext, s);
  gemm_upload(st.trest, s);
  HSS_HIP(hipEventCreateWithFlags(&st.ev_block, hipEventDisableTiming));
  HSS_HIP(hipEventCreateWithFlags(&st.ev_rest, hipEventDisableTiming));
}

void free_state(Blr2State* st) {
  if (!st) return;
  for (auto& g : st->phi) gemm_free(g);
  for (auto& g : st->g1) gemm_free(g);
  for (auto& g : st->g2) gemm_free(g);
  gemm_free(st->inblk);
  gemm_free(st->tnext);
  gemm_free(st->trest);
  if (st->ev_block) (void)hipEventDestroy(st->ev_block);
  if (st->ev_rest) (void)hipEventDestroy(st->ev_rest);
  void* ptrs[] = {st->dK, st->dLinv, st->dPhi, st->dG, st->dpanel, st->dinfo, st->dlog, st->dZ, st->doffK};
  for (void* p : ptrs)
    if (p) dev_free(p);
  delete st;
}

// A single entry of a uploaded batch, launched alone.
GemmBatch entry_view(const GemmBatch& b, int k, int variant) {
  GemmBatch v;
  v.dev = b.dev + k;
  v.count = 1;
  v.mmax = b.host[k].m;
  v.nmax = b.host[k].n;
  v.variant = variant;
  return v;
}

void factor_blr2(hss_matrix_t m) {
  hss_ctx_t cx = m->ctx;
  hipStream_t s = cx->stream;
  check_shape(m);
  if (!m->blr2) {
    m->blr2 = new Blr2State();
    try {
      alloc_state(m, *m->blr2);
    } catch (...) {
      free_state(m->blr2);
      m->blr2 = nullptr;
      throw;
    }
  }
  Blr2State& st = *m->blr2;
  st.valid = false;
  m->state = 0;  // the leaf buffers are shared with the HSS-ULV factorization
  HSS_HIP(hipEventRecord(cx->ev0, s));
  // 1. the leaf stage and the leaves' parents' merged blocks
  factor_leaf_stage_fp64(m);
  hipLaunchKernelGGL(k_blr2_clear, dim3(1), dim3(1), 0, s, st.dinfo);
  HSS_HIP(hipGetLastError());
  // 2. the skeleton matrix: diagonal blocks, then the couplings of every
  // level above the leaves' parents
  {
    const LevelPlan& lp = m->stages[1];
    Prof pf(cx, "blr2_diag", lp.level);
    hipLaunchKernelGGL(k_blr2_diag, dim3(lp.count), dim3(256), 0, s, m->dnodes, lp.first, (const double*)m->dM,
                       (const int64_t*)st.doffK, st.dK, st.K);
    HSS_HIP(hipGetLastError());
  }
  for (auto& g : st.phi) {
    Prof pf(cx, "blr2_phi", -1);
    gemm_launch_f64(g, false, false, 1.0, 0.0, s);
  }
  for (size_t q = 0; q < st.g1.size(); ++q) {
    Prof pf(cx, "blr2_couplings", -1);
    gemm_launch_f64(st.g1[q], false, true, 1.0, 0.0, s);
    gemm_launch_f64(st.g2[q], false, true, 1.0, 0.0, s);
  }
  // 3. dense Cholesky of the skeleton matrix, with a lookahead of one outer
  // block: after block q, the next block's columns are updated on the first
  // stream and its panels factored there, while the rest of the trailing
  // matrix is updated on the second stream (the two write disjoint columns;
  // the next block's own trailing update waits for that rest update)
  if (!cx->aux_stream) HSS_HIP(hipStreamCreateWithFlags(&cx->aux_stream, hipStreamNonBlocking));
  hipStream_t a = cx->aux_stream;
  bool rest_pending = false;
  const int64_t K = st.K;
  for (int k = 0; k < st.npanel; ++k) {
    const int64_t k0 = (int64_t)k * DNB;
    const int jb = (int)std::min<int64_t>(DNB, K - k0);
    const int64_t rem = K - k0 - jb;
    double* Li = st.dLinv + (int64_t)k * DNB * DNB;
    Prof pf(cx, "blr2_cholesky", -1);
    hipLaunchKernelGGL(k_dchol_diag, dim3(1), dim3(256), 0, s, st.dK, K, k0, jb, Li, st.dpanel + k, st.dinfo);
    HSS_HIP(hipGetLastError());
    if (rem <= 0) continue;
    hipLaunchKernelGGL(k_dtrsm_rows, dim3((unsigned)((rem + DNB - 1) / DNB)), dim3(256), 0, s, st.dK, K, K, k0, jb,
                       (const double*)Li);
    HSS_HIP(hipGetLastError());
    if (st.inblk_of[k] >= 0) gemm_launch_f64(entry_view(st.inblk, st.inblk_of[k], 0), false, true, -1.0, 1.0, s);
    if ((k + 1) % DOB == 0 || k + 1 == st.npanel) {
      const int q = k / DOB;
      if (st.trest_of[q] >= 0) {
        HSS_HIP(hipEventRecord(st.ev_block, s));
        HSS_HIP(hipStreamWaitEvent(a, st.ev_block, 0));
      }
      if (rest_pending) {  // the previous rest update wrote this update's columns too
        HSS_HIP(hipStreamWaitEvent(s, st.ev_rest, 0));
        rest_pending = false;
      }
      if (st.tnext_of[q] >= 0) gemm_launch_f64(entry_view(st.tnext, st.tnext_of[q], 0), false, true, -1.0, 1.0, s);
      if (st.trest_of[q] >= 0) {
        gemm_launch_f64(entry_view(st.trest, st.trest_of[q], 7), false, true, -1.0, 1.0, a);
        HSS_HIP(hipEventRecord(st.ev_rest, a));
        rest_pending = true;
      }
    }
  }
  if (rest_pending) HSS_HIP(hipStreamWaitEvent(s, st.ev_rest, 0));
  hipLaunchKernelGGL(k_blr2_logdet, dim3(1), dim3(256), 0, s, (const double*)m->dlogdet, m->nnodes,
                     (const double*)st.dpanel, st.npanel, st.dlog);
  HSS_HIP(hipGetLastError());
  HSS_HIP(hipEventRecord(cx->ev1, s));
  int32_t leaf_info[4] = {0, 0, 0, 0};
  int32_t skel_info[2] = {0, 0};
  HSS_HIP(hipMemcpyAsync(leaf_info, m->dinfo, sizeof(leaf_info), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipMemcpyAsync(skel_info, st.dinfo, sizeof(skel_info), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipMemcpyAsync(&st.logdet, st.dlog, sizeof(double), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipStreamSynchronize(s));
  HSS_HIP(hipEventElapsedTime(&st.factor_ms, cx->ev0, cx->ev1));
  if (leaf_info[0] != 0)
    throw Error{HSS_ERR_NOT_SPD, "BLR^2-ULV: non-positive pivot at leaf node " + std::to_string(leaf_info[1]) +
                                     ", pivot " + std::to_string(leaf_info[2])};
  if (skel_info[0] != 0)
    throw Error{HSS_ERR_NOT_SPD,
                "BLR^2-ULV: non-positive pivot in the skeleton matrix at row " + std::to_string(skel_info[1])};
  st.valid = true;
}

void solve_blr2(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  Blr2State& st = *m->blr2;
  hss_ctx_t cx = m->ctx;
  hipStream_t s = cx->stream;
  ensure_vec_ws(m, nrhs);
  const int rc = solve_chunk();
  const LevelPlan& lp = m->stages[1];
  const int64_t K = st.K;
  for (int64_t c0 = 0; c0 < nrhs; c0 += rc) {
    Prof pf(cx, "blr2_leaf_forward", -1);
    solve_leaf_sweep(m, true, b, nullptr, nrhs, c0, (int)std::min<int64_t>(rc, nrhs - c0), ld);
  }
  for (int64_t c0 = 0; c0 < nrhs; c0 += kSolveCols) {
    const int nc = (int)std::min<int64_t>(kSolveCols, nrhs - c0);
    Prof pf(cx, "blr2_skeleton_solve", -1);
    hipLaunchKernelGGL(k_blr2_gather, dim3(lp.count), dim3(256), 0, s, m->dnodes, lp.first, (const int64_t*)st.doffK,
                       (const double*)m->dvec, nrhs, c0, nc, st.dZ, K, 0);
    HSS_HIP(hipGetLastError());
    for (int k = 0; k < st.npanel; ++k) {
      const int64_t k0 = (int64_t)k * DNB;
      const int jb = (int)std::min<int64_t>(DNB, K - k0);
      const int64_t rem = K - k0 - jb;
      const unsigned g = (unsigned)std::max<int64_t>(1, (rem + 63) / 64);
      hipLaunchKernelGGL(k_dtrsv_fwd, dim3(g), dim3(256), 0, s, (const double*)st.dK, K, K, k0, jb,
                         (const double*)(st.dLinv + (int64_t)k * DNB * DNB), st.dZ, st.dY, nc);
      HSS_HIP(hipGetLastError());
    }
    for (int k = st.npanel - 1; k >= 0; --k) {
      const int64_t k0 = (int64_t)k * DNB;
      const int jb = (int)std::min<int64_t>(DNB, K - k0);
      const unsigned g = (unsigned)std::max<int64_t>(1, (k0 + 63) / 64);
      hipLaunchKernelGGL(k_dtrsv_bwd, dim3(g), dim3(256), 0, s, (const double*)st.dK, K, K, k0, jb,
                         (const double*)(st.dLinv + (int64_t)k * DNB * DNB), st.dY, st.dW, nc);
      HSS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_blr2_gather, dim3(lp.count), dim3(256), 0, s, m->dnodes, lp.first, (const int64_t*)st.doffK,
                       (const double*)m->dvec, nrhs, c0, nc, st.dW, K, 1);
    HSS_HIP(hipGetLastError());
  }
  for (int64_t c0 = 0; c0 < nrhs; c0 += rc) {
    Prof pf(cx, "blr2_leaf_backward", -1);
    solve_leaf_sweep(m, false, nullptr, x, nrhs, c0, (int)std::min<int64_t>(rc, nrhs - c0), ld);
  }
}

}  // namespace

void blr2_free(hss_matrix_t m) {
  if (!m || !m->blr2) return;
  free_state(m->blr2);
  m->blr2 = nullptr;
}

void blr2_invalidate(hss_matrix_t m) {
  if (m && m->blr2) m->blr2->valid = false;
}

}  // namespace hss

using namespace hss;

#define BLR2_API_BEGIN try {
#define BLR2_API_END                                 \
  }                                                  \
  catch (const Error& e) {                           \
    set_error(e.msg);                                \
    return e.st;                                     \
  }                                                  \
  catch (const std::bad_alloc&) {                    \
    set_error("host allocation failed");             \
    return HSS_ERR_OUT_OF_MEMORY;                    \
  }                                                  \
  catch (...) {                                      \
    set_error("unexpected internal exception");      \
    return HSS_ERR_DEVICE;                           \
  }                                                  \
  return HSS_OK;

extern "C" {

hss_status hss_blr2_factor(hss_ctx_t ctx, hss_matrix_t m) {
  BLR2_API_BEGIN
  CtxScope cs_(ctx);
  HSS_CHECK(ctx && m, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->ctx == ctx, HSS_ERR_INVALID_ARGUMENT, "matrix belongs to another context");
  factor_blr2(m);
  BLR2_API_END
}

hss_status hss_blr2_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x, int64_t nrhs, int64_t ld) {
  BLR2_API_BEGIN
  CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && d_b && d_x, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->ctx == ctx, HSS_ERR_INVALID_ARGUMENT, "matrix belongs to another context");
  HSS_CHECK(nrhs >= 1 && ld >= m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld >= n");
  HSS_CHECK(m->blr2 && m->blr2->valid, HSS_ERR_BAD_STATE, "matrix has no BLR^2-ULV factorization");
  solve_blr2(m, d_b, d_x, nrhs, ld);
  BLR2_API_END
}

hss_status hss_blr2_logdet(hss_ctx_t ctx, hss_matrix_t m, double* h_out) {
  BLR2_API_BEGIN
  HSS_CHECK(ctx && m && h_out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->blr2 && m->blr2->valid, HSS_ERR_BAD_STATE, "matrix has no BLR^2-ULV factorization");
  *h_out = m->blr2->logdet;
  BLR2_API_END
}

hss_status hss_blr2_stats(hss_matrix_t m, int64_t* skeleton_rows, float* factor_ms) {
  BLR2_API_BEGIN
  HSS_CHECK(m && skeleton_rows, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  if (m->blr2) {
    *skeleton_rows = m->blr2->K;
    if (factor_ms) *factor_ms = m->blr2->valid ? m->blr2->factor_ms : 0.f;
  } else {
    Blr2State tmp;
    check_shape(m);
    skeleton_offsets(m, tmp);
    *skeleton_rows = tmp.K;
    if (factor_ms) *factor_ms = 0.f;
  }
  BLR2_API_END
}

}  // extern "C"
