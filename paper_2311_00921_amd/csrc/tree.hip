// Cluster tree on the GPU: recursive coordinate bisection of the points.
//
// At every node the points are ordered by (coordinate on the longest side of
// their bounding box, lowest axis on ties; original index on equal
// coordinates) and the first ceil(s/2) go to the left child. That key is a
// total order, so above the last level only the membership of the two halves
// matters: each level finds, per node, the ceil(s/2)-th smallest key by an
// exact radix select (8-bit digits of the 64-bit order-preserving coordinate,
// then of the 40-bit index) and partitions the node's points by comparison
// with it. At the last level every node is sorted in LDS (bitonic network),
// which fixes the order of the points inside each leaf. Bounding boxes come
// from wave-reduced 64-bit atomics on order-preserving keys (min and max are
// exact). The node ranges follow from the sizes alone and are computed on the
// host; no point leaves the device.
#include <algorithm>

#include "hss_internal.h"

namespace hss {

namespace {

constexpr int TB_NT = 256;
constexpr int TB_CHUNK = 4096;     // points per workgroup in the per-node passes
constexpr int TB_SORT = 2 * kMaxBlock;  // largest node the last-level sort takes (two largest leaves)
constexpr int TB_IDX_BITS = 40;    // point indices below 2^40

// Order-preserving map of a double to uint64 (-0 taken as +0, so that equal
// coordinates compare equal).
__device__ __forceinline__ uint64_t okey(double v) {
  if (v == 0.0) v = 0.0;
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double okey_inv(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

struct Seg {
  int64_t lo, hi;  // points [lo, hi) of the node in the current order
};

__global__ void k_iota(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = i;
}

// per node and axis: [0..2] min keys, [3..5] max keys
__global__ void k_box_init(uint64_t* __restrict__ box, int nseg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nseg * 6) box[i] = (i % 6) < 3 ? ~0ull : 0ull;
}

// Workgroup (c, s) covers points [lo_s + c * TB_CHUNK, ...) of node s.
__global__ __launch_bounds__(TB_NT) void k_box(const Seg* __restrict__ seg, const double* __restrict__ X, int dim,
                                               const int64_t* __restrict__ perm, uint64_t* __restrict__ box) {
  const Seg sg = seg[blockIdx.y];
  const int64_t b0 = sg.lo + (int64_t)blockIdx.x * TB_CHUNK;
  if (b0 >= sg.hi) return;
  const int64_t b1 = min(sg.hi, b0 + TB_CHUNK);
  uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
  for (int64_t t = b0 + threadIdx.x; t < b1; t += TB_NT) {
    const double* x = X + perm[t] * dim;
    for (int a = 0; a < dim; ++a) {
      const uint64_t k = okey(x[a]);
      mn[a] = min(mn[a], k);
      mx[a] = max(mx[a], k);
    }
  }
  for (int a = 0; a < dim; ++a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = min(mn[a], (uint64_t)__shfl_xor((unsigned long long)mn[a], o, 64));
      mx[a] = max(mx[a], (uint64_t)__shfl_xor((unsigned long long)mx[a], o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin((unsigned long long*)&box[blockIdx.y * 6 + a], (unsigned long long)mn[a]);
      atomicMax((unsigned long long*)&box[blockIdx.y * 6 + 3 + a], (unsigned long long)mx[a]);
    }
  }
}

// Per node: the split axis (longest side, lowest axis on ties, the side being
// max - min in FP64), and the radix-select state: rank k = ceil(s/2) of the
// last left point, empty prefix.
__global__ void k_axis(const Seg* __restrict__ seg, int nseg, const uint64_t* __restrict__ box, int dim,
                       int32_t* __restrict__ axis, int64_t* __restrict__ krem, uint64_t* __restrict__ pre) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int ax = 0;
  double best = okey_inv(box[s * 6 + 3]) - okey_inv(box[s * 6]);
  for (int a = 1; a < dim; ++a) {
    const double e = okey_inv(box[s * 6 + 3 + a]) - okey_inv(box[s * 6 + a]);
    if (e > best) {
      best = e;
      ax = a;
    }
  }
  axis[s] = ax;
  const int64_t n = seg[s].hi - seg[s].lo;
  krem[s] = (n + 1) / 2;
  pre[2 * s] = 0;
  pre[2 * s + 1] = 0;
}

// Digit j of the 104-bit key (coordinate key, then index), and whether the
// key's higher digits equal the prefix found so far.
__device__ __forceinline__ bool digit_of(uint64_t kc, uint64_t ki, int j, const uint64_t* pre, int& d) {
  if (j < 8) {
    const int sh = 56 - 8 * j;
    if (j > 0 && (kc >> (sh + 8)) != (pre[0] >> (sh + 8))) return false;
    d = (int)((kc >> sh) & 255);
    return true;
  }
  if (kc != pre[0]) return false;
  const int sh = TB_IDX_BITS - 8 - 8 * (j - 8);
  if (j > 8 && (ki >> (sh + 8)) != (pre[1] >> (sh + 8))) return false;
  d = (int)((ki >> sh) & 255);
  return true;
}

__global__ __launch_bounds__(TB_NT) void k_hist(const Seg* __restrict__ seg, const double* __restrict__ X, int dim,
                                                const int64_t* __restrict__ perm, const int32_t* __restrict__ axis,
                                                const uint64_t* __restrict__ pre, int j, int32_t* __restrict__ hist) {
  __shared__ int32_t h[256];
  const int s = blockIdx.y;
  const Seg sg = seg[s];
  const int64_t b0 = sg.lo + (int64_t)blockIdx.x * TB_CHUNK;
  if (b0 >= sg.hi) return;
  const int64_t b1 = min(sg.hi, b0 + TB_CHUNK);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int ax = axis[s];
  const uint64_t p[2] = {pre[2 * s], pre[2 * s + 1]};
  for (int64_t t = b0 + threadIdx.x; t < b1; t += TB_NT) {
    const int64_t id = perm[t];
    int d;
    if (digit_of(okey(X[id * dim + ax]), (uint64_t)id, j, p, d)) atomicAdd(&h[d], 1);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[s * 256 + threadIdx.x], h[threadIdx.x]);
}

// One thread per node: the digit holding the krem-th key of the current
// bucket; the node's bins are cleared for the next digit.
__global__ void k_select(int nseg, int j, int32_t* __restrict__ hist, int64_t* __restrict__ krem,
                         uint64_t* __restrict__ pre) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int64_t k = krem[s];
  int d = 0;
  for (; d < 256; ++d) {
    const int64_t c = hist[s * 256 + d];
    if (k <= c) break;
    k -= c;
  }
  d = min(d, 255);
  krem[s] = k;
  if (j < 8)
    pre[2 * s] |= (uint64_t)d << (56 - 8 * j);
  else
    pre[2 * s + 1] |= (uint64_t)d << (TB_IDX_BITS - 8 - 8 * (j - 8));
  for (int e = 0; e < 256; ++e) hist[s * 256 + e] = 0;
}

// Points with keys up to the selected one go to the left child, the others to
// the right child (order inside each half is immaterial: the next level orders
// by its own total key).
__global__ __launch_bounds__(TB_NT) void k_split(const Seg* __restrict__ seg, const double* __restrict__ X, int dim,
                                                 const int64_t* __restrict__ perm, const int32_t* __restrict__ axis,
                                                 const uint64_t* __restrict__ pre, int64_t* __restrict__ cnt,
                                                 int64_t* __restrict__ out) {
  const int s = blockIdx.y;
  const Seg sg = seg[s];
  const int64_t b0 = sg.lo + (int64_t)blockIdx.x * TB_CHUNK;
  if (b0 >= sg.hi) return;
  const int64_t b1 = min(sg.hi, b0 + TB_CHUNK);
  const int ax = axis[s];
  const uint64_t pc = pre[2 * s], pi = pre[2 * s + 1];
  const int64_t mid = sg.lo + (sg.hi - sg.lo + 1) / 2;
  for (int64_t t = b0 + threadIdx.x; t < b1; t += TB_NT) {
    const int64_t id = perm[t];
    const uint64_t kc = okey(X[id * dim + ax]);
    const bool left = kc < pc || (kc == pc && (uint64_t)id <= pi);
    const int64_t pos = left ? sg.lo + atomicAdd((unsigned long long*)&cnt[2 * s], 1ull)
                             : mid + atomicAdd((unsigned long long*)&cnt[2 * s + 1], 1ull);
    out[pos] = id;
  }
}

__global__ void k_zero64(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Last level: each node (at most TB_SORT points) sorted by its key in LDS.
__global__ __launch_bounds__(512) void k_sort_nodes(const Seg* __restrict__ seg, const double* __restrict__ X, int dim,
                                                    const int32_t* __restrict__ axis, int64_t* __restrict__ perm) {
  __shared__ uint64_t kc[TB_SORT];
  __shared__ uint64_t ki[TB_SORT];
  const int s = blockIdx.x;
  const Seg sg = seg[s];
  const int n = (int)(sg.hi - sg.lo);
  int P = 1;
  while (P < n) P <<= 1;
  const int ax = axis[s];
  for (int t = threadIdx.x; t < P; t += 512) {
    if (t < n) {
      const int64_t id = perm[sg.lo + t];
      kc[t] = okey(X[id * dim + ax]);
      ki[t] = (uint64_t)id;
    } else {
      kc[t] = ~0ull;
      ki[t] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = threadIdx.x; t < P; t += 512) {
        const int u = t ^ jj;
        if (u > t) {
          const bool up = (t & k) == 0;
          const bool gt = kc[t] > kc[u] || (kc[t] == kc[u] && ki[t] > ki[u]);
          if (gt == up) {
            const uint64_t a = kc[t], b = ki[t];
            kc[t] = kc[u];
            ki[t] = ki[u];
            kc[u] = a;
            ki[u] = b;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < n; t += 512) perm[sg.lo + t] = (int64_t)ki[t];
}

// Per leaf: FP64 bounding box (lo[3], hi[3]; zero beyond dim).
__global__ void k_box_decode(const uint64_t* __restrict__ box, int nseg, int dim, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  for (int a = 0; a < 3; ++a) {
    out[s * 6 + a] = a < dim ? okey_inv(box[s * 6 + a]) : 0.0;
    out[s * 6 + 3 + a] = a < dim ? okey_inv(box[s * 6 + 3 + a]) : 0.0;
  }
}

template <typename T>
struct DevArr {
  T* p = nullptr;
  explicit DevArr(int64_t n) { p = (T*)dev_alloc(sizeof(T) * std::max<int64_t>(n, 1)); }
  ~DevArr() {
    if (p) dev_free(p);
  }
  DevArr(const DevArr&) = delete;
  DevArr& operator=(const DevArr&) = delete;
};

int64_t max_len(const std::vector<Seg>& v) {
  int64_t m = 0;
  for (const Seg& s : v) m = std::max(m, s.hi - s.lo);
  return m;
}

}  // namespace

// Node ranges of every level from the point count alone (left child takes
// ceil(s/2)); the last entry of leaf_lo is n.
static std::vector<std::vector<Seg>> tree_ranges(int64_t n, int L) {
  std::vector<std::vector<Seg>> lv(L + 1);
  lv[0] = {{0, n}};
  for (int l = 0; l < L; ++l)
    for (const Seg& s : lv[l]) {
      const int64_t mid = s.lo + (s.hi - s.lo + 1) / 2;
      lv[l + 1].push_back({s.lo, mid});
      lv[l + 1].push_back({mid, s.hi});
    }
  return lv;
}

std::vector<int64_t> tree_leaf_lo(int64_t n, int L) {
  const std::vector<std::vector<Seg>> lv = tree_ranges(n, L);
  std::vector<int64_t> leaf_lo;
  for (const Seg& s : lv[L]) leaf_lo.push_back(s.lo);
  leaf_lo.push_back(n);
  return leaf_lo;
}

void build_tree(hipStream_t st, const double* d_points, int64_t n, int dim, int L, int64_t* d_perm,
                double* d_leafbox) {
  HSS_CHECK(n >= 1 && dim >= 1 && dim <= 3 && L >= 0 && L <= 20, HSS_ERR_INVALID_ARGUMENT, "tree: bad sizes");
  HSS_CHECK(n < ((int64_t)1 << TB_IDX_BITS), HSS_ERR_UNSUPPORTED, "tree: too many points");
  const std::vector<std::vector<Seg>> lv = tree_ranges(n, L);
  if (L > 0)
    HSS_CHECK(max_len(lv[L - 1]) <= TB_SORT, HSS_ERR_UNSUPPORTED,
              "tree: nodes above the leaves hold more than " + std::to_string(TB_SORT) + " points");
  const int nmax = 1 << L;  // nodes of the deepest level
  DevArr<int64_t> tmp(n);
  DevArr<Seg> dseg(nmax);
  DevArr<uint64_t> box((int64_t)nmax * 6);
  DevArr<int32_t> axis(nmax);
  DevArr<int64_t> krem(nmax);
  DevArr<uint64_t> pre((int64_t)nmax * 2);
  DevArr<int32_t> hist((int64_t)(nmax > 1 ? nmax / 2 : 1) * 256);
  DevArr<int64_t> cnt((int64_t)nmax * 2);
  int64_t* cur = d_perm;
  int64_t* nxt = tmp.p;
  hipLaunchKernelGGL(k_iota, dim3(1024), dim3(256), 0, st, cur, n);
  HSS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_zero64, dim3(64), dim3(256), 0, st, (int64_t*)hist.p,
                     (int64_t)(nmax > 1 ? nmax / 2 : 1) * 128);
  HSS_HIP(hipGetLastError());
  auto boxes = [&](const std::vector<Seg>& segs) {
    const int ns = (int)segs.size();
    HSS_HIP(hipMemcpyAsync(dseg.p, segs.data(), sizeof(Seg) * ns, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_box_init, dim3((ns * 6 + 255) / 256), dim3(256), 0, st, box.p, ns);
    const unsigned chunks = (unsigned)((max_len(segs) + TB_CHUNK - 1) / TB_CHUNK);
    hipLaunchKernelGGL(k_box, dim3(chunks, ns), dim3(TB_NT), 0, st, (const Seg*)dseg.p, d_points, dim,
                       (const int64_t*)cur, box.p);
    HSS_HIP(hipGetLastError());
  };
  for (int l = 0; l < L; ++l) {
    const std::vector<Seg>& segs = lv[l];
    const int ns = (int)segs.size();
    boxes(segs);
    hipLaunchKernelGGL(k_axis, dim3((ns + 255) / 256), dim3(256), 0, st, (const Seg*)dseg.p, ns,
                       (const uint64_t*)box.p, dim, axis.p, krem.p, pre.p);
    HSS_HIP(hipGetLastError());
    if (l == L - 1) {
      hipLaunchKernelGGL(k_sort_nodes, dim3(ns), dim3(512), 0, st, (const Seg*)dseg.p, d_points, dim,
                         (const int32_t*)axis.p, cur);
      HSS_HIP(hipGetLastError());
      break;
    }
    const unsigned chunks = (unsigned)((max_len(segs) + TB_CHUNK - 1) / TB_CHUNK);
    for (int j = 0; j < 8 + TB_IDX_BITS / 8; ++j) {
      hipLaunchKernelGGL(k_hist, dim3(chunks, ns), dim3(TB_NT), 0, st, (const Seg*)dseg.p, d_points, dim,
                         (const int64_t*)cur, (const int32_t*)axis.p, (const uint64_t*)pre.p, j, hist.p);
      hipLaunchKernelGGL(k_select, dim3((ns + 255) / 256), dim3(256), 0, st, ns, j, hist.p, krem.p, pre.p);
      HSS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_zero64, dim3(64), dim3(256), 0, st, cnt.p, (int64_t)ns * 2);
    hipLaunchKernelGGL(k_split, dim3(chunks, ns), dim3(TB_NT), 0, st, (const Seg*)dseg.p, d_points, dim,
                       (const int64_t*)cur, (const int32_t*)axis.p, (const uint64_t*)pre.p, cnt.p, nxt);
    HSS_HIP(hipGetLastError());
    std::swap(cur, nxt);
  }
  if (cur != d_perm) HSS_HIP(hipMemcpyAsync(d_perm, cur, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
  if (d_leafbox) {
    boxes(lv[L]);
    hipLaunchKernelGGL(k_box_decode, dim3(((1 << L) + 255) / 256), dim3(256), 0, st, (const uint64_t*)box.p,
                       1 << L, dim, d_leafbox);
    HSS_HIP(hipGetLastError());
  }
  // the temporaries are released when this returns: wait for the kernels
  HSS_HIP(hipStreamSynchronize(st));
}

}  // namespace hss
