// C ABI of libhss.so: argument validation, the matrix state machine, the
// device layout of the HSS representation, import and export.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>

#include "hss_internal.h"

namespace hss {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// Device memory: from the allocator of the context whose call is running on
// this thread (CtxScope), else hipMalloc. Every block remembers the allocator
// it came from, so that it goes back to it whenever it is freed.
thread_local hss_ctx_t g_alloc_ctx = nullptr;

namespace {
std::mutex g_blocks_mu;
std::unordered_map<void*, hss_allocator> g_blocks;  // blocks from a caller's allocator
}  // namespace

void* dev_alloc(size_t bytes) {
  const size_t nb = bytes == 0 ? 8 : bytes;
  void* p = nullptr;
  if (g_alloc_ctx && g_alloc_ctx->allocator.alloc) {
    const hss_allocator a = g_alloc_ctx->allocator;
    p = a.alloc(nb, a.user);
    if (!p) throw Error{HSS_ERR_OUT_OF_MEMORY, "the caller's allocator returned no block of " + std::to_string(nb) +
                                                   " bytes"};
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    g_blocks[p] = a;
    return p;
  }
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{HSS_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  hss_allocator a{};
  bool custom = false;
  {
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    auto it = g_blocks.find(p);
    if (it != g_blocks.end()) {
      a = it->second;
      custom = true;
      g_blocks.erase(it);
    }
  }
  if (custom) {
    // the caller's allocator may hand the block out again at once, on any
    // stream: no work of ours may still use it
    (void)hipDeviceSynchronize();
    a.free(p, a.user);
  } else {
    (void)hipFree(p);
  }
}

static hipEvent_t pool_event(hss_ctx_t c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    HSS_HIP(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

Prof::Prof(hss_ctx_t c, const char* name, int level) : ctx(c) {
  if (!ctx || !ctx->prof) return;
  ProfRec r{name, level, pool_event(ctx), pool_event(ctx)};
  HSS_HIP(hipEventRecord(r.a, ctx->stream));
  idx = ctx->prof_recs.size();
  ctx->prof_recs.push_back(r);
}

Prof::~Prof() {
  if (idx == (size_t)-1) return;
  (void)hipEventRecord(ctx->prof_recs[idx].b, ctx->stream);
}

static int level_of(int k) {
  int l = 0;
  while ((2 << l) - 1 <= k) ++l;
  return l;
}

// Block sizes, offsets and child rows of every node, given the links, leaf
// point ranges and ranks (any node order). Allocates nothing.
void assign_offsets(hss_matrix_t m) {
  auto& nd = m->nodes;
  const int nn = (int)nd.size();
  // children before parents: leaves have their size; internal nodes need the children's ranks
  for (int k = 0; k < nn; ++k)
    if (nd[k].c1 < 0) nd[k].n = nd[k].npts;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int k = 0; k < nn; ++k)
      if (nd[k].c1 >= 0) {
        const int want = nd[nd[k].c1].r + nd[nd[k].c2].r;
        if (nd[k].n != want) {
          nd[k].n = want;
          changed = true;
        }
      }
  }
  int64_t oD = 0, oB = 0, oS = 0, oF = 0, oM = 0, oV = 0, oT = 0, oSg = 0, oW = 0, oX = 0, oVec = 0, oR = 0;
  m->max_rank = 0;
  for (int k = 0; k < nn; ++k) {
    NodeDesc& d = nd[k];
    const bool leaf = d.c1 < 0;
    const bool root = d.parent < 0;
    if (root) d.r = 0;
    d.m = d.n - d.r;
    HSS_CHECK(d.r >= 0 && d.r <= d.n, HSS_ERR_INVALID_ARGUMENT,
              "node " + std::to_string(k) + ": rank exceeds block size");
    HSS_CHECK(root || d.r >= 1, HSS_ERR_INVALID_ARGUMENT, "node " + std::to_string(k) + ": rank must be >= 1");
    m->max_rank = std::max(m->max_rank, d.r);
    d.offD = leaf ? oD : -1;
    if (leaf) oD += (int64_t)d.n * d.n;
    d.offB = root ? -1 : oB;
    if (!root) oB += (int64_t)d.n * d.r;
    d.offS = leaf ? -1 : oS;
    if (!leaf) oS += (int64_t)nd[d.c1].r * nd[d.c2].r;
    d.offF = oF;
    oF += (int64_t)d.n * d.n;
    d.offM = leaf ? -1 : oM;
    if (!leaf) oM += (int64_t)d.n * d.n;
    // V sits at the right of an n x 2r slot: the two-sided update reads [Z V] as
    // one n x 2r operand (and [V Z] as the same operand with its columns rotated)
    d.offV = oV + (int64_t)d.n * d.r;
    oV += 2 * (int64_t)d.n * d.r;
    d.offT = oT;
    oT += (int64_t)d.r * d.r;
    d.offSg = oSg;
    oSg += d.r;
    d.offW = oW;
    oW += 2 * (int64_t)d.n * d.r;
    d.offX = oX;
    oX += 2 * (int64_t)d.r * d.r;
    d.offVec = oVec;
    oVec += d.n;
    d.offR = oR;
    oR += d.r;
    d.child_row = 0;
  }
  for (int k = 0; k < nn; ++k)
    if (nd[k].c1 >= 0) {
      nd[nd[k].c1].child_row = 0;
      nd[nd[k].c2].child_row = nd[nd[k].c1].r;
    }
  m->lenD = oD;
  m->lenB = oB;
  m->lenS = oS;
  m->lenF = oF;
  m->lenM = oM;
  m->lenV = oV;
  m->lenT = oT;
  m->lenSg = oSg;
  m->lenW = oW;
  m->lenX = oX;
  m->sum_n = oVec;
  m->sum_r = oR;
}

// Per-stage extents, the explicit-inverse choice and the Li / L_SR slots; uploads the node table.
void finish_stages(hss_matrix_t m) {
  auto& nd = m->nodes;
  const int nn = (int)nd.size();
  m->offLi.assign(nn, 0);
  m->offS2.assign(nn, 0);
  int64_t oLi = 0, oS2 = 0;
  for (auto& lp : m->stages) {
    lp.nmax = lp.rmax = lp.mmax = 0;
    lp.root_first = lp.first + lp.count;
    for (int k = lp.first; k < lp.first + lp.count; ++k) {
      lp.nmax = std::max(lp.nmax, nd[k].n);
      lp.rmax = std::max(lp.rmax, nd[k].r);
      lp.mmax = std::max(lp.mmax, nd[k].m);
      if (nd[k].parent < 0 && lp.root_first == lp.first + lp.count) lp.root_first = k;
    }
    lp.leaf = (nd[lp.first].c1 < 0) ? 1 : 0;
    lp.inv = (lp.mmax <= 96 && lp.mmax >= 1) ? 1 : 0;
    lp.root_split = (!lp.inv && lp.root_first == lp.first && lp.nmax > 96 && lp.nmax <= 192) ? 1 : 0;
    if (lp.root_split) {
      // inverses of the two diagonal blocks, h x h then (n - h) x (n - h)
      for (int k = lp.first; k < lp.first + lp.count; ++k) {
        const int h = root_split_h(nd[k].n), h2 = nd[k].n - h;
        m->offLi[k] = oLi;
        oLi += (int64_t)h * h + (int64_t)h2 * h2;
      }
      continue;
    }
    if (!lp.inv) continue;
    for (int k = lp.first; k < lp.first + lp.count; ++k) {
      m->offLi[k] = oLi;
      oLi += (int64_t)nd[k].m * nd[k].m;
      m->offS2[k] = oS2;
      oS2 += (int64_t)nd[k].r * nd[k].m;
    }
  }
  m->lenLi = oLi;
  m->lenS2 = oS2;
  m->inv_used64.assign(m->stages.size(), 0);
  if (m->dOffLi) dev_free(m->dOffLi);
  if (m->dOffS2) dev_free(m->dOffS2);
  m->dOffLi = (int64_t*)dev_alloc(sizeof(int64_t) * nn);
  m->dOffS2 = (int64_t*)dev_alloc(sizeof(int64_t) * nn);
  HSS_HIP(hipMemcpyAsync(m->dOffLi, m->offLi.data(), sizeof(int64_t) * nn, hipMemcpyHostToDevice, m->ctx->stream));
  HSS_HIP(hipMemcpyAsync(m->dOffS2, m->offS2.data(), sizeof(int64_t) * nn, hipMemcpyHostToDevice, m->ctx->stream));
  if (m->dnodes) dev_free(m->dnodes);
  m->dnodes = (NodeDesc*)dev_alloc(sizeof(NodeDesc) * nn);
  HSS_HIP(hipMemcpyAsync(m->dnodes, nd.data(), sizeof(NodeDesc) * nn, hipMemcpyHostToDevice, m->ctx->stream));
}

// Single tree in heap order (node k has children 2k+1, 2k+2): links, offsets,
// one stage per level (leaves first); allocates the representation buffers.
void layout_representation(hss_matrix_t m) {
  const int L = m->L;
  const int nn = m->nnodes;
  auto& nd = m->nodes;
  for (int k = (1 << L) - 2; k >= 0; --k) {
    nd[k].lo = nd[2 * k + 1].lo;
    nd[k].npts = nd[2 * k + 1].npts + nd[2 * k + 2].npts;
  }
  for (int k = 0; k < nn; ++k) {
    nd[k].level = level_of(k);
    nd[k].parent = k > 0 ? (k - 1) / 2 : -1;
    const bool leaf = nd[k].level == L;
    nd[k].c1 = leaf ? -1 : 2 * k + 1;
    nd[k].c2 = leaf ? -1 : 2 * k + 2;
    nd[k].sys = 0;
  }
  nd[0].r = 0;
  assign_offsets(m);
  m->levels.clear();
  m->stages.clear();
  for (int l = 0; l <= L; ++l) {
    LevelPlan lp{};
    lp.level = l;
    lp.first = (1 << l) - 1;
    lp.count = 1 << l;
    m->levels.push_back(lp);
  }
  for (int l = L; l >= 0; --l) m->stages.push_back(m->levels[l]);
  finish_stages(m);
  for (auto& st : m->stages) m->levels[st.level] = st;
  m->nsys = 1;
  m->sys_lo.assign(1, 0);
  m->sys_root.assign(1, 0);
  if (!m->dD) m->dD = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenD, 1));
  if (!m->dB) m->dB = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenB, 1));
  if (!m->dS) m->dS = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenS, 1));
  if (!m->dperm) m->dperm = (int64_t*)dev_alloc(sizeof(int64_t) * m->n);
}

static void destroy_matrix(hss_matrix_t m) {
  if (!m) return;
  if (m->ctx) (void)hipStreamSynchronize(m->ctx->stream);
  drop_graphs(m);
  blr2_free(m);
  free_factor(m);
  void* ptrs[] = {m->dnodes, m->dD, m->dB, m->dS, m->dperm, m->dvec, m->dxt, m->dyt, m->dtmp,
                  m->dOffLi, m->dOffS2};
  for (void* p : ptrs)
    if (p) dev_free(p);
  delete m;
}

}  // namespace hss

using namespace hss;

#define HSS_API_BEGIN try {
#define HSS_API_END                                 \
  }                                                 \
  catch (const hss::Error& e) {                     \
    hss::set_error(e.msg);                          \
    return e.st;                                    \
  }                                                 \
  catch (const std::bad_alloc&) {                   \
    hss::set_error("host allocation failed");       \
    return HSS_ERR_OUT_OF_MEMORY;                   \
  }                                                 \
  catch (...) {                                     \
    hss::set_error("unexpected internal exception"); \
    return HSS_ERR_DEVICE;                          \
  }                                                 \
  return HSS_OK;

extern "C" {

const char* hss_status_string(hss_status s) {
  switch (s) {
    case HSS_OK: return "ok";
    case HSS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case HSS_ERR_NOT_SPD: return "matrix not positive definite";
    case HSS_ERR_OUT_OF_MEMORY: return "out of memory";
    case HSS_ERR_DEVICE: return "device error";
    case HSS_ERR_BAD_STATE: return "bad state";
    case HSS_ERR_NOT_CONVERGED: return "not converged";
    case HSS_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* hss_last_error(void) { return g_last_error.c_str(); }

hss_status hss_ctx_create(int32_t device, void* hip_stream, const hss_allocator* allocator, hss_ctx_t* out) {
  HSS_API_BEGIN
  HSS_CHECK(out != nullptr, HSS_ERR_INVALID_ARGUMENT, "out is NULL");
  HSS_CHECK(!allocator || (allocator->alloc && allocator->free) || (!allocator->alloc && !allocator->free),
            HSS_ERR_INVALID_ARGUMENT, "an allocator needs both alloc and free");
  int count = 0;
  HSS_HIP(hipGetDeviceCount(&count));
  HSS_CHECK(device >= 0 && device < count, HSS_ERR_INVALID_ARGUMENT, "device index out of range");
  HSS_HIP(hipSetDevice(device));
  noalloc_init(device);  // the static scratch array of the no-allocation solve, on this device
  hss_ctx_t c = new hss_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (allocator) c->allocator = *allocator;
  HSS_HIP(hipEventCreate(&c->ev0));
  HSS_HIP(hipEventCreate(&c->ev1));
  *out = c;
  HSS_API_END
}

hss_status hss_ctx_destroy(hss_ctx_t ctx) {
  HSS_API_BEGIN
  if (!ctx) return HSS_OK;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_trail) (void)hipEventDestroy(ctx->ev_trail);
  delete ctx;
  HSS_API_END
}

hss_status hss_ctx_set_stream(hss_ctx_t ctx, void* hip_stream) {
  HSS_API_BEGIN
  HSS_CHECK(ctx != nullptr, HSS_ERR_INVALID_ARGUMENT, "ctx is NULL");
  ctx->stream = (hipStream_t)hip_stream;
  HSS_API_END
}

hss_status hss_profile_enable(hss_ctx_t ctx, int32_t on) {
  HSS_API_BEGIN
  HSS_CHECK(ctx != nullptr, HSS_ERR_INVALID_ARGUMENT, "ctx is NULL");
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  ctx->prof = on != 0;
  ctx->prof_recs.clear();
  ctx->ev_used = 0;
  HSS_API_END
}

hss_status hss_profile_read(hss_ctx_t ctx, char* buf, int64_t capacity, int64_t* needed) {
  HSS_API_BEGIN
  HSS_CHECK(ctx != nullptr, HSS_ERR_INVALID_ARGUMENT, "ctx is NULL");
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  // aggregate by (name, level): launches and total milliseconds
  struct Agg {
    std::string name;
    int level;
    int64_t count;
    double ms;
  };
  std::vector<Agg> agg;
  for (auto& r : ctx->prof_recs) {
    float ms = 0.f;
    HSS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    bool found = false;
    for (auto& a : agg)
      if (a.name == r.name && a.level == r.level) {
        a.count++;
        a.ms += ms;
        found = true;
        break;
      }
    if (!found) agg.push_back({r.name, r.level, 1, (double)ms});
  }
  std::string out;
  for (auto& a : agg)
    out += a.name + " " + std::to_string(a.level) + " " + std::to_string(a.count) + " " + std::to_string(a.ms) + "\n";
  if (needed) *needed = (int64_t)out.size() + 1;
  if (buf && capacity > 0) {
    const size_t n = std::min<size_t>(out.size(), (size_t)capacity - 1);
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  HSS_API_END
}

hss_status hss_import(hss_ctx_t ctx, const hss_desc* d, hss_matrix_t* out) {
  hss::CtxScope cs_(ctx);
  hss_matrix_t m = nullptr;
  HSS_API_BEGIN
  HSS_CHECK(ctx && d && out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(d->n >= 1, HSS_ERR_INVALID_ARGUMENT, "n must be >= 1");
  HSS_CHECK(d->levels >= 0 && d->levels <= 24, HSS_ERR_INVALID_ARGUMENT, "levels out of range");
  HSS_CHECK(d->leaf_lo && d->D, HSS_ERR_INVALID_ARGUMENT, "leaf_lo and D are required");
  const int L = d->levels;
  HSS_CHECK(L == 0 || (d->rank && d->U && d->S), HSS_ERR_INVALID_ARGUMENT, "rank, U and S are required");
  HSS_CHECK(L <= 1 || d->E, HSS_ERR_INVALID_ARGUMENT, "E is required for levels >= 2");
  m = new hss_matrix_s();
  m->ctx = ctx;
  m->n = d->n;
  m->L = L;
  m->nnodes = (2 << L) - 1;
  m->nodes.assign(m->nnodes, NodeDesc{});
  const int nleaves = 1 << L;
  HSS_CHECK(d->leaf_lo[0] == 0 && d->leaf_lo[nleaves] == d->n, HSS_ERR_INVALID_ARGUMENT,
            "leaf boundaries must span [0, n)");
  for (int i = 0; i < nleaves; ++i) {
    NodeDesc& nd = m->nodes[nleaves - 1 + i];
    nd.lo = d->leaf_lo[i];
    nd.npts = (int32_t)(d->leaf_lo[i + 1] - d->leaf_lo[i]);
    HSS_CHECK(nd.npts >= 1 && nd.npts <= kMaxBlock, HSS_ERR_INVALID_ARGUMENT, "leaf sizes must be in [1, 1024]");
  }
  for (int k = 1; k < m->nnodes; ++k) m->nodes[k].r = d->rank[k];
  layout_representation(m);
  for (int k = 1; k < m->nnodes; ++k)
    HSS_CHECK(m->nodes[k].n <= kMaxBlock && m->nodes[k].r <= kMaxRank, HSS_ERR_UNSUPPORTED,
              "blocks above 1024 rows or ranks above 512 are not supported");
  HSS_CHECK(m->nodes[0].n <= kMaxBlock, HSS_ERR_UNSUPPORTED, "root block above 1024 rows");
  hipStream_t s = ctx->stream;
  HSS_HIP(hipMemcpyAsync(m->dD, d->D, sizeof(double) * m->lenD, hipMemcpyHostToDevice, s));
  if (L > 0) {
    // dB = [E of nodes 1..2^L-2 | U of the leaves] in heap order
    int64_t lenE = 0;
    for (int k = 1; k < nleaves - 1; ++k) lenE += (int64_t)m->nodes[k].n * m->nodes[k].r;
    if (lenE > 0) HSS_HIP(hipMemcpyAsync(m->dB, d->E, sizeof(double) * lenE, hipMemcpyHostToDevice, s));
    HSS_HIP(hipMemcpyAsync(m->dB + lenE, d->U, sizeof(double) * (m->lenB - lenE), hipMemcpyHostToDevice, s));
    HSS_HIP(hipMemcpyAsync(m->dS, d->S, sizeof(double) * m->lenS, hipMemcpyHostToDevice, s));
  }
  std::vector<int64_t> perm(m->n);
  if (d->perm) {
    std::vector<char> seen(m->n, 0);
    for (int64_t i = 0; i < m->n; ++i) {
      HSS_CHECK(d->perm[i] >= 0 && d->perm[i] < m->n && !seen[d->perm[i]], HSS_ERR_INVALID_ARGUMENT,
                "perm is not a permutation");
      seen[d->perm[i]] = 1;
      perm[i] = d->perm[i];
    }
  } else {
    for (int64_t i = 0; i < m->n; ++i) perm[i] = i;
  }
  HSS_HIP(hipMemcpyAsync(m->dperm, perm.data(), sizeof(int64_t) * m->n, hipMemcpyHostToDevice, s));
  HSS_HIP(hipStreamSynchronize(s));
  *out = m;
  m = nullptr;
  return HSS_OK;
  }
  catch (const hss::Error& e) {
    hss::set_error(e.msg);
    destroy_matrix(m);
    return e.st;
  }
  catch (...) {
    hss::set_error("unexpected internal exception");
    destroy_matrix(m);
    return HSS_ERR_DEVICE;
  }
}

hss_status hss_construct(hss_ctx_t ctx, const double* d_points, int64_t n, int32_t dim, const hss_kernel* kernel,
                         const hss_construct_opts* opts, const double* d_omega, int32_t s, hss_matrix_t* out) {
  hss::CtxScope cs_(ctx);
  hss_matrix_t m = nullptr;
  try {
    HSS_CHECK(ctx && d_points && kernel && opts && out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
    HSS_CHECK(n >= 1, HSS_ERR_INVALID_ARGUMENT, "n must be >= 1");
    HSS_CHECK(dim >= 1 && dim <= 3, HSS_ERR_INVALID_ARGUMENT, "dim must be 1, 2 or 3");
    HSS_CHECK(opts->leaf_size >= 2 && opts->leaf_size <= kMaxBlock, HSS_ERR_INVALID_ARGUMENT,
              "leaf_size must be in [2, 1024]");
    HSS_CHECK(opts->rank >= 0 && opts->rank <= kMaxRank, HSS_ERR_INVALID_ARGUMENT, "rank must be in [0, 512]");
    HSS_CHECK(opts->rank > 0 || opts->tol > 0.0, HSS_ERR_INVALID_ARGUMENT, "adaptive rank needs tol > 0");
    HSS_CHECK(opts->max_rank >= 0, HSS_ERR_INVALID_ARGUMENT, "max_rank must be >= 0");
    HSS_CHECK(opts->mode == HSS_COMPRESS_SCALED || opts->mode == HSS_COMPRESS_PLAIN, HSS_ERR_INVALID_ARGUMENT,
              "unknown compression mode");
    HSS_CHECK(kernel->kind >= 0 && kernel->kind <= 4, HSS_ERR_INVALID_ARGUMENT, "unknown kernel");
    HSS_CHECK(kernel->kind >= HSS_K_LAPLACE2D || kernel->length > 0.0, HSS_ERR_INVALID_ARGUMENT,
              "kernel length must be > 0");
    HSS_CHECK(kernel->nugget >= 0.0, HSS_ERR_INVALID_ARGUMENT, "nugget must be >= 0");
    int L = 0;
    while (((int64_t)opts->leaf_size << L) < n) ++L;
    HSS_CHECK(opts->levels == 0 || opts->levels == L, HSS_ERR_INVALID_ARGUMENT,
              "levels must equal ceil(log2(N / leaf_size)) = " + std::to_string(L));
    HSS_CHECK(L <= 20, HSS_ERR_UNSUPPORTED, "too many levels");
    HSS_CHECK(L == 0 || (d_omega && s >= 1 && s <= kMaxSamples), HSS_ERR_INVALID_ARGUMENT,
              "need a test matrix with 1..512 columns");
    HSS_CHECK(L == 0 || opts->rank == 0 || s >= opts->rank, HSS_ERR_INVALID_ARGUMENT, "need s >= rank");
    const bool sized = opts->rank == 0 && (opts->rank_model != nullptr || opts->sample_start > 0);
    HSS_CHECK(opts->sample_start >= 0 && opts->probes >= 0 && opts->probes <= 64 && opts->judge_factor >= 0.0,
              HSS_ERR_INVALID_ARGUMENT, "bad sample sizing options");
    SamplePlan sp;
    if (sized && L > 0) {
      sp.model = opts->rank_model;
      sp.probes = opts->probes > 0 ? opts->probes : 8;
      HSS_CHECK(s >= sp.probes + 1, HSS_ERR_INVALID_ARGUMENT, "need s > probes for the judge");
      sp.s_basis = opts->rank_model ? 0 : std::min(opts->sample_start, s - sp.probes);
      sp.judge_thr = (opts->judge_factor > 0.0 ? opts->judge_factor : 10.0) * opts->tol;
    } else {
      sp.s_basis = s;
    }
    hss_construct_stats st{};
    for (;;) {
      m = new hss_matrix_s();
      m->ctx = ctx;
      m->n = n;
      m->L = L;
      const int smax = s - sp.probes;
      sp.abort_on_fail = sized && (sp.s_basis == 0 || sp.s_basis < smax);
      sp.passed = true;
      st.attempts += 1;
      const bool ok = construct(m, d_points, dim, *kernel, *opts, d_omega, s, sp);
      if (ok || sp.s_basis >= smax) break;
      destroy_matrix(m);  // restart with twice the samples
      m = nullptr;
      sp.s_basis = std::min(2 * sp.s_basis, smax);
    }
    st.samples = L > 0 ? sp.s_basis : 0;
    st.probes = sp.probes;
    st.judge_failures = sp.judge_failures;
    st.predicted_max = sp.predicted_max;
    st.max_rank = m->max_rank;
    st.sample_bytes = sp.sample_bytes;
    m->cstats = st;
    *out = m;
    return HSS_OK;
  } catch (const hss::Error& e) {
    hss::set_error(e.msg);
    destroy_matrix(m);
    return e.st;
  } catch (...) {
    hss::set_error("unexpected internal exception");
    destroy_matrix(m);
    return HSS_ERR_DEVICE;
  }
}

hss_status hss_get_construct_stats(hss_matrix_t m, hss_construct_stats* out) {
  HSS_API_BEGIN
  HSS_CHECK(m && out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = m->cstats;
  HSS_API_END
}

hss_status hss_export_sizes(hss_matrix_t m, int64_t sizes[7]) {
  HSS_API_BEGIN
  HSS_CHECK(m && sizes, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->nsys == 1, HSS_ERR_UNSUPPORTED, "a batch cannot be exported; export its systems");
  sizes[0] = (1 << m->L) + 1;
  sizes[1] = m->nnodes;
  sizes[2] = m->lenD;
  int64_t lenE = 0;
  for (int k = 1; k < (1 << m->L) - 1; ++k) lenE += (int64_t)m->nodes[k].n * m->nodes[k].r;
  sizes[3] = m->lenB - lenE;
  sizes[4] = lenE;
  sizes[5] = m->lenS;
  sizes[6] = m->n;
  HSS_API_END
}

hss_status hss_export(hss_ctx_t ctx, hss_matrix_t m, hss_desc_out* o) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && o, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->nsys == 1, HSS_ERR_UNSUPPORTED, "a batch cannot be exported; export its systems");
  hipStream_t s = ctx->stream;
  const int nleaves = 1 << m->L;
  if (o->leaf_lo) {
    for (int i = 0; i < nleaves; ++i) o->leaf_lo[i] = m->nodes[nleaves - 1 + i].lo;
    o->leaf_lo[nleaves] = m->n;
  }
  if (o->rank)
    for (int k = 0; k < m->nnodes; ++k) o->rank[k] = m->nodes[k].r;
  int64_t lenE = 0;
  for (int k = 1; k < nleaves - 1; ++k) lenE += (int64_t)m->nodes[k].n * m->nodes[k].r;
  if (o->D) HSS_HIP(hipMemcpyAsync(o->D, m->dD, sizeof(double) * m->lenD, hipMemcpyDeviceToHost, s));
  if (m->L > 0) {
    if (o->E && lenE > 0) HSS_HIP(hipMemcpyAsync(o->E, m->dB, sizeof(double) * lenE, hipMemcpyDeviceToHost, s));
    if (o->U)
      HSS_HIP(hipMemcpyAsync(o->U, m->dB + lenE, sizeof(double) * (m->lenB - lenE), hipMemcpyDeviceToHost, s));
    if (o->S) HSS_HIP(hipMemcpyAsync(o->S, m->dS, sizeof(double) * m->lenS, hipMemcpyDeviceToHost, s));
  }
  if (o->perm) HSS_HIP(hipMemcpyAsync(o->perm, m->dperm, sizeof(int64_t) * m->n, hipMemcpyDeviceToHost, s));
  HSS_HIP(hipStreamSynchronize(s));
  HSS_API_END
}

// Runs a factorization (run() enqueues it on the context stream), then reads
// the pivot status: FACTORED, or FAILED with the failing node and NOT_SPD.
static void factor_checked(hss_ctx_t ctx, hss_matrix_t m, int prec, const std::function<void()>& run) {
  hipStream_t s = ctx->stream;
  m->state = 0;
  blr2_invalidate(m);
  m->failed_level = m->failed_node = m->failed_pivot = m->failed_system = -1;
  HSS_HIP(hipEventRecord(ctx->ev0, s));
  run();
  HSS_HIP(hipEventRecord(ctx->ev1, s));
  int32_t info[4] = {0, 0, 0, 0};
  HSS_HIP(hipMemcpyAsync(info, m->dinfo, sizeof(info), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  HSS_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  m->factor_ms = ms;
  m->precision = prec;
  if (info[0] != 0) {
    m->state = 2;
    m->failed_node = info[1];
    m->failed_level = m->nodes[info[1]].level;
    m->failed_system = m->nodes[info[1]].sys;
    m->failed_pivot = info[2];
    throw Error{HSS_ERR_NOT_SPD, "non-positive pivot at level " + std::to_string(m->failed_level) + ", node " +
                                     std::to_string(info[1]) + ", pivot " + std::to_string(info[2]) +
                                     (m->nsys > 1 ? ", system " + std::to_string(m->failed_system) : "")};
  }
  m->state = 1;
}

hss_status hss_ulv_factor(hss_ctx_t ctx, hss_matrix_t m, const hss_factor_opts* opts) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  const int prec = opts ? opts->precision : HSS_P_FP64;
  HSS_CHECK(prec >= HSS_P_FP64 && prec <= HSS_P_BF16X3, HSS_ERR_INVALID_ARGUMENT, "unknown precision");
  factor_checked(ctx, m, prec, [&] { factor_run(m, prec); });
  HSS_API_END
}

hss_status hss_ulv_factor_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x, int64_t nrhs,
                                int64_t ld) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && d_b && d_x, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(nrhs >= 1 && ld >= m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld >= n");
  factor_checked(ctx, m, HSS_P_FP64, [&] {
    if (ctx->prof) {
      // per-launch profiling times every launch on the context stream: no overlap
      factor_fp64(m);
      solve_fp64(m, d_b, d_x, nrhs, ld);
    } else {
      factor_solve_fp64(m, d_b, d_x, nrhs, ld);
    }
  });
  HSS_API_END
}

hss_status hss_ulv_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x, int64_t nrhs, int64_t ld) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && d_b && d_x, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(nrhs >= 1 && ld >= m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld >= n");
  HSS_CHECK(m->state == 1, HSS_ERR_BAD_STATE, "matrix is not factored");
  hipStream_t s = ctx->stream;
  HSS_HIP(hipEventRecord(ctx->ev0, s));
  solve_run(m, d_b, d_x, nrhs, ld);
  HSS_HIP(hipEventRecord(ctx->ev1, s));
  HSS_API_END
}

hss_status hss_matvec(hss_ctx_t ctx, hss_matrix_t m, const double* d_x, double* d_y, int64_t nrhs, int64_t ld) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && d_x && d_y, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(nrhs >= 1 && ld >= m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld >= n");
  HSS_CHECK(d_x != d_y, HSS_ERR_INVALID_ARGUMENT, "x and y must not alias");
  matvec_fp64(m, d_x, d_y, nrhs, ld);
  HSS_API_END
}

hss_status hss_logdet(hss_ctx_t ctx, hss_matrix_t m, double* h_out) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && h_out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(m->state == 1, HSS_ERR_BAD_STATE, "matrix is not factored");
  *h_out = read_logdet(m);
  HSS_API_END
}

hss_status hss_get_info(hss_matrix_t m, hss_info* o) {
  HSS_API_BEGIN
  HSS_CHECK(m && o, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memset(o, 0, sizeof(*o));
  o->n = m->n;
  o->levels = m->L;
  o->factored = m->state == 1;
  o->precision = m->precision;
  o->max_rank = m->max_rank;
  o->failed_level = m->failed_level;
  o->failed_node = m->failed_node;
  o->failed_pivot = m->failed_pivot;
  o->bytes_representation = 8 * (m->lenD + m->lenB + m->lenS);
  o->bytes_factor = 8 * (m->lenF + m->lenV + m->lenT + m->lenSg);
  o->factor_ms = m->factor_ms;
  o->solve_ms = m->solve_ms;
  o->systems = m->nsys;
  o->failed_system = m->failed_system;
  o->promoted_nodes = m->promoted;
  HSS_API_END
}

hss_status hss_get_ranks(hss_matrix_t m, int32_t* h_out, int64_t capacity, int64_t* needed) {
  HSS_API_BEGIN
  HSS_CHECK(m && needed, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  *needed = m->nnodes;
  if (!h_out) return HSS_OK;
  HSS_CHECK(capacity >= m->nnodes, HSS_ERR_INVALID_ARGUMENT, "output too small");
  for (int k = 0; k < m->nnodes; ++k) h_out[k] = m->nodes[k].r;
  HSS_API_END
}

hss_status hss_get_permutation(hss_ctx_t ctx, hss_matrix_t m, int64_t* d_perm) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && d_perm, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_HIP(hipMemcpyAsync(d_perm, m->dperm, sizeof(int64_t) * m->n, hipMemcpyDeviceToDevice, ctx->stream));
  HSS_API_END
}

hss_status hss_debug_node_block(hss_ctx_t ctx, hss_matrix_t m, int32_t node, int32_t what, double* h_out,
                                int64_t capacity) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && h_out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(node >= 0 && node < m->nnodes, HSS_ERR_INVALID_ARGUMENT, "node out of range");
  HSS_CHECK(m->state == 1, HSS_ERR_BAD_STATE, "matrix is not factored");
  const NodeDesc& nd = m->nodes[node];
  hipStream_t s = ctx->stream;
  if (what == 0) {
    HSS_CHECK(node > 0, HSS_ERR_INVALID_ARGUMENT, "the root has no Schur complement");
    HSS_CHECK(capacity >= (int64_t)nd.r * nd.r, HSS_ERR_INVALID_ARGUMENT, "capacity too small");
    std::vector<double> F((size_t)nd.n * nd.n), sg(nd.r);
    HSS_HIP(hipMemcpyAsync(F.data(), m->dF + nd.offF, sizeof(double) * F.size(), hipMemcpyDeviceToHost, s));
    HSS_HIP(hipMemcpyAsync(sg.data(), m->dSg + nd.offSg, sizeof(double) * nd.r, hipMemcpyDeviceToHost, s));
    HSS_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < nd.r; ++j)
      for (int i = 0; i < nd.r; ++i) {
        const int a = std::max(i, j), b = std::min(i, j);
        h_out[i + (int64_t)j * nd.r] = sg[i] * sg[j] * F[(nd.m + a) + (int64_t)(nd.m + b) * nd.n];
      }
  } else if (what == 1) {
    HSS_CHECK(nd.c1 >= 0, HSS_ERR_INVALID_ARGUMENT, "leaves have no merged block");
    HSS_CHECK(capacity >= (int64_t)nd.n * nd.n, HSS_ERR_INVALID_ARGUMENT, "capacity too small");
    HSS_HIP(hipMemcpyAsync(h_out, m->dM + nd.offM, sizeof(double) * nd.n * nd.n, hipMemcpyDeviceToHost, s));
    HSS_HIP(hipStreamSynchronize(s));
  } else if (what >= 2 && what <= 5) {
    // raw factor data: 2 = V (n x r), 3 = T (r x r), 4 = F block (n x n, [R;S] order), 5 = signs (r)
    const int64_t len = what == 2 ? (int64_t)nd.n * nd.r : what == 3 ? (int64_t)nd.r * nd.r
                        : what == 4 ? (int64_t)nd.n * nd.n : nd.r;
    const double* src = what == 2 ? m->dV + nd.offV : what == 3 ? m->dT + nd.offT
                        : what == 4 ? m->dF + nd.offF : m->dSg + nd.offSg;
    HSS_CHECK(capacity >= len, HSS_ERR_INVALID_ARGUMENT, "capacity too small");
    HSS_HIP(hipMemcpyAsync(h_out, src, sizeof(double) * len, hipMemcpyDeviceToHost, s));
    HSS_HIP(hipStreamSynchronize(s));
  } else {
    throw Error{HSS_ERR_INVALID_ARGUMENT, "unknown block kind"};
  }
  HSS_API_END
}

hss_status hss_matrix_destroy(hss_matrix_t m) {
  HSS_API_BEGIN
  destroy_matrix(m);
  HSS_API_END
}

}  // extern "C"
