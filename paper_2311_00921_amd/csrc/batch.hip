// Batches of independent HSS systems, HIP-graph replay of the factorization
// and the solve, and the autotuner of the batched GEMM tile shapes.
//
// A batch is one hss_matrix_t holding a forest: the trees of all systems, with
// their nodes regrouped into stages by height above the leaves. Every step of
// Alg. 2 and of the solve (Eq. 17) is then one launch per stage for all
// systems, whatever their sizes and depths; a system whose tree is shallower
// simply has its root in a lower stage. Vectors of a batch are the systems'
// vectors stacked in order.
#include <algorithm>
#include <array>
#include <map>

#include "hss_internal.h"

namespace hss {

struct CopyDesc {
  const double* src;
  double* dst;
  int64_t len;
};

__global__ void k_copy_many(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.len; i += (int64_t)gridDim.x * blockDim.x)
    d.dst[i] = d.src[i];
}

struct PermDesc {
  const int64_t* src;
  int64_t* dst;
  int64_t len;
  int64_t add;
};

__global__ void k_copy_perm(const PermDesc* __restrict__ descs) {
  const PermDesc d = descs[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.len; i += (int64_t)gridDim.x * blockDim.x)
    d.dst[i] = d.src[i] + d.add;
}

template <typename D, typename K>
static void run_descs(const std::vector<D>& h, K kern, int64_t maxlen, hipStream_t s) {
  if (h.empty() || maxlen <= 0) return;
  D* dd = (D*)dev_alloc(sizeof(D) * h.size());
  HSS_HIP(hipMemcpyAsync(dd, h.data(), sizeof(D) * h.size(), hipMemcpyHostToDevice, s));
  for (size_t c0 = 0; c0 < h.size(); c0 += 65535) {
    const int cnt = (int)std::min<size_t>(65535, h.size() - c0);
    const int bx = (int)std::min<int64_t>((maxlen + 255) / 256, 64);
    hipLaunchKernelGGL(kern, dim3(bx, cnt), dim3(256), 0, s, (const D*)(dd + c0));
    HSS_HIP(hipGetLastError());
  }
  HSS_HIP(hipStreamSynchronize(s));
  dev_free(dd);
}

// Builds the forest of `mats` (single trees in heap order) into m: node table,
// stages by height (within a stage the non-roots first, each system's nodes
// together, siblings adjacent), offsets, and copies of D, U/E, S and perm.
static void layout_forest(hss_matrix_t m, const std::vector<hss_matrix_t>& mats) {
  hipStream_t s = m->ctx->stream;
  const int ns = (int)mats.size();
  m->nsys = ns;
  m->sys_lo.assign(ns, 0);
  m->sys_root.assign(ns, 0);
  int64_t ntot = 0;
  int H = 0, nn = 0;
  for (int k = 0; k < ns; ++k) {
    HSS_CHECK(mats[k]->nsys == 1, HSS_ERR_INVALID_ARGUMENT, "a batch cannot contain another batch");
    m->sys_lo[k] = ntot;
    ntot += mats[k]->n;
    H = std::max(H, mats[k]->L);
    nn += mats[k]->nnodes;
  }
  m->n = ntot;
  m->L = H;
  m->nnodes = nn;
  // new index of every (system, heap node)
  std::vector<std::vector<int>> idx(ns);
  for (int k = 0; k < ns; ++k) idx[k].assign(mats[k]->nnodes, -1);
  m->stages.clear();
  int next = 0;
  for (int h = 0; h <= H; ++h) {
    LevelPlan lp{};
    lp.level = h;
    lp.first = next;
    for (int pass = 0; pass < 2; ++pass)  // non-roots, then roots
      for (int k = 0; k < ns; ++k) {
        const int L = mats[k]->L, l = L - h;
        if (l < 0) continue;
        if ((l == 0) != (pass == 1)) continue;
        for (int j = (1 << l) - 1; j < (2 << l) - 1; ++j) idx[k][j] = next++;
      }
    lp.count = next - lp.first;
    if (lp.count > 0) m->stages.push_back(lp);
  }
  m->nodes.assign(nn, NodeDesc{});
  for (int k = 0; k < ns; ++k) {
    const hss_matrix_t a = mats[k];
    for (int j = 0; j < a->nnodes; ++j) {
      const NodeDesc& o = a->nodes[j];
      NodeDesc& d = m->nodes[idx[k][j]];
      d.lo = o.lo + m->sys_lo[k];
      d.npts = o.npts;
      d.n = o.n;
      d.r = o.r;
      d.level = o.level;
      d.parent = o.parent >= 0 ? idx[k][o.parent] : -1;
      d.c1 = o.c1 >= 0 ? idx[k][o.c1] : -1;
      d.c2 = o.c2 >= 0 ? idx[k][o.c2] : -1;
      d.sys = k;
    }
    m->sys_root[k] = idx[k][0];
  }
  assign_offsets(m);
  finish_stages(m);
  m->levels = m->stages;  // labels only: index = height
  m->dD = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenD, 1));
  m->dB = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenB, 1));
  m->dS = (double*)dev_alloc(sizeof(double) * std::max<int64_t>(m->lenS, 1));
  m->dperm = (int64_t*)dev_alloc(sizeof(int64_t) * std::max<int64_t>(m->n, 1));
  std::vector<CopyDesc> cp;
  int64_t maxlen = 0;
  auto add = [&](const double* src, double* dst, int64_t len) {
    if (len <= 0) return;
    cp.push_back({src, dst, len});
    maxlen = std::max(maxlen, len);
  };
  for (int k = 0; k < ns; ++k) {
    const hss_matrix_t a = mats[k];
    for (int j = 0; j < a->nnodes; ++j) {
      const NodeDesc& o = a->nodes[j];
      const NodeDesc& d = m->nodes[idx[k][j]];
      HSS_CHECK(o.n == d.n && o.r == d.r, HSS_ERR_DEVICE, "inconsistent node sizes in batch layout");
      if (o.c1 < 0) add(a->dD + o.offD, m->dD + d.offD, (int64_t)o.n * o.n);
      if (o.parent >= 0) add(a->dB + o.offB, m->dB + d.offB, (int64_t)o.n * o.r);
      if (o.c1 >= 0) add(a->dS + o.offS, m->dS + d.offS, (int64_t)a->nodes[o.c1].r * a->nodes[o.c2].r);
    }
  }
  run_descs(cp, k_copy_many, maxlen, s);
  std::vector<PermDesc> pp;
  int64_t pmax = 0;
  for (int k = 0; k < ns; ++k) {
    pp.push_back({mats[k]->dperm, m->dperm + m->sys_lo[k], mats[k]->n, m->sys_lo[k]});
    pmax = std::max(pmax, mats[k]->n);
  }
  run_descs(pp, k_copy_perm, pmax, s);
}

// ---------------------------------------------------------------------------
// HIP graphs
// ---------------------------------------------------------------------------

// Records the launches that fn() enqueues on the context stream into a graph
// (on a private non-blocking stream, so the caller's stream may be the null
// stream) and instantiates it. Nothing executes during the recording.
template <class F>
static hipGraphExec_t record_graph(hss_matrix_t m, F fn) {
  hss_ctx_t c = m->ctx;
  if (!c->cap_stream) HSS_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  HSS_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap_stream;
  hipGraph_t g = nullptr;
  try {
    fn();
  } catch (...) {
    c->stream = user;
    if (hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    throw;
  }
  c->stream = user;
  HSS_HIP(hipStreamEndCapture(c->cap_stream, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HSS_HIP(e);
  return ex;
}

void drop_graphs(hss_matrix_t m) {
  for (auto& g : m->gexec_factor)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  if (m->gexec_solve) (void)hipGraphExecDestroy(m->gexec_solve);
  m->gexec_solve = nullptr;
  m->solve_key = hss_matrix_s::SolveKey{};
}

static void factor_direct(hss_matrix_t m, int precision) {
  if (precision == HSS_P_FP64)
    factor_fp64(m);
  else
    factor_mixed(m, precision);
}

void factor_run(hss_matrix_t m, int precision) {
  // the mixed factorization reads a failure count back between stages, so it
  // is never recorded into a graph
  if (!m->use_graph || m->ctx->prof || g_tune || precision != HSS_P_FP64) {
    factor_direct(m, precision);
    return;
  }
  prepare_factor(m, precision);  // allocations and descriptor uploads happen outside the recording
  hipGraphExec_t& ex = m->gexec_factor[precision == HSS_P_FP64 ? 0 : 1];
  if (!ex) ex = record_graph(m, [&] { factor_direct(m, precision); });
  HSS_HIP(hipGraphLaunch(ex, m->ctx->stream));
}

// Both precisions leave FP64 factors: the solve is the same.
static void solve_direct(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  solve_fp64(m, b, x, nrhs, ld);
}

void solve_run(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  if (!m->use_graph || m->ctx->prof) {
    solve_direct(m, b, x, nrhs, ld);
    return;
  }
  ensure_vec_ws(m, nrhs);
  hss_matrix_s::SolveKey key;
  key.prec = m->precision;
  key.b = b;
  key.x = x;
  key.nrhs = nrhs;
  key.ld = ld;
  key.ws = m->dvec;
  if (!m->gexec_solve || !(m->solve_key == key)) {
    if (m->gexec_solve) (void)hipGraphExecDestroy(m->gexec_solve);
    m->gexec_solve = nullptr;
    m->gexec_solve = record_graph(m, [&] { solve_direct(m, b, x, nrhs, ld); });
    m->solve_key = key;
  }
  HSS_HIP(hipGraphLaunch(m->gexec_solve, m->ctx->stream));
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

// Runs the factorization once untimed, then `reps` times with every GEMM batch
// on each tile variant in turn, timing each batched launch with events; keeps
// the fastest variant per batch. Every run is a complete factorization.
static void autotune(hss_matrix_t m, int precision, int reps, std::vector<float>* report) {
  prepare_factor(m, precision);
  auto& plan = precision == HSS_P_FP64 ? m->gemm_plan : m->gemm_plan32;
  hipStream_t s = m->ctx->stream;
  drop_graphs(m);
  const bool prof = m->ctx->prof;
  m->ctx->prof = false;
  TuneRec rec;
  std::map<const GemmBatch*, std::array<double, kGemmVariants>> tm;
  struct Guard {
    TuneRec* rec;
    hss_ctx_t ctx;
    bool prof;
    ~Guard() {
      g_tune = nullptr;
      ctx->prof = prof;
      for (hipEvent_t e : rec->pool) (void)hipEventDestroy(e);
    }
  } guard{&rec, m->ctx, prof};
  factor_direct(m, precision);  // warm-up
  g_tune = &rec;
  // the shapes take turns within each repetition, and each batch keeps its
  // best time over the repetitions: drift and interference from the second
  // stream then bias no shape
  for (int it = 0; it < reps; ++it) {
    for (int v = 0; v < kGemmVariants; ++v) {
      for (auto& st : plan)
        for (auto& g : st) g.variant = v;
      rec.recs.clear();
      rec.used = 0;
      factor_direct(m, precision);
      HSS_HIP(hipStreamSynchronize(s));
      std::map<const GemmBatch*, double> once;  // per factorization (a batch may launch more than once)
      for (auto& r : rec.recs) {
        float ms = 0.f;
        HSS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        once[r.batch] += ms;
      }
      for (auto& kv : once) {
        auto ins = tm.try_emplace(kv.first);
        if (ins.second) ins.first->second.fill(1e30);
        double& slot = ins.first->second[v];
        slot = std::min(slot, kv.second);
      }
    }
  }
  g_tune = nullptr;
  float total[kGemmVariants + 1] = {0};
  for (auto& st : plan)
    for (auto& g : st) {
      auto it = tm.find(&g);
      if (it == tm.end()) {
        g.variant = 0;
        continue;
      }
      int best = 0;
      for (int v = 0; v < kGemmVariants; ++v) {
        total[v] += (float)it->second[v];
        if (it->second[v] < it->second[best]) best = v;
      }
      total[kGemmVariants] += (float)it->second[best];
      g.variant = best;
    }
  if (report) report->assign(total, total + kGemmVariants + 1);
  m->state = 0;  // tuning runs leave no usable factorization state behind
  blr2_invalidate(m);
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
  catch (const std::exception& e) {                 \
    hss::set_error(e.what());                       \
    return HSS_ERR_DEVICE;                          \
  }                                                 \
  return HSS_OK;

extern "C" {

hss_status hss_batch_create(hss_ctx_t ctx, int32_t count, const hss_matrix_t* mats, hss_matrix_t* out) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && mats && out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(count >= 1, HSS_ERR_INVALID_ARGUMENT, "count must be >= 1");
  std::vector<hss_matrix_t> v(mats, mats + count);
  for (auto a : v) HSS_CHECK(a != nullptr, HSS_ERR_INVALID_ARGUMENT, "NULL matrix in batch");
  HSS_HIP(hipSetDevice(ctx->device));
  hss_matrix_t m = new hss_matrix_s();
  m->ctx = ctx;
  try {
    layout_forest(m, v);
  } catch (...) {
    hss_matrix_destroy(m);
    throw;
  }
  *out = m;
  HSS_API_END
}

hss_status hss_construct_batched(hss_ctx_t ctx, int32_t count, const double* const* d_points, const int64_t* n,
                                 int32_t dim, const hss_kernel* kernels, const hss_construct_opts* opts,
                                 const double* const* d_omega, const int32_t* s, hss_matrix_t* out) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && d_points && n && kernels && opts && d_omega && s && out, HSS_ERR_INVALID_ARGUMENT,
            "NULL argument");
  HSS_CHECK(count >= 1, HSS_ERR_INVALID_ARGUMENT, "count must be >= 1");
  std::vector<hss_matrix_t> v(count, nullptr);
  hss_status st = HSS_OK;
  for (int k = 0; k < count && st == HSS_OK; ++k)
    st = hss_construct(ctx, d_points[k], n[k], dim, &kernels[k], &opts[k], d_omega[k], s[k], &v[k]);
  if (st == HSS_OK) st = hss_batch_create(ctx, count, v.data(), out);
  const std::string err = st == HSS_OK ? std::string() : std::string(hss_last_error());
  for (auto a : v)
    if (a) hss_matrix_destroy(a);
  if (st != HSS_OK) {
    set_error(err);
    return st;
  }
  HSS_API_END
}

hss_status hss_batch_query(hss_ctx_t ctx, hss_matrix_t m, int32_t count, int64_t* h_offsets, int32_t* h_failed,
                           double* h_logdet) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(count == m->nsys, HSS_ERR_INVALID_ARGUMENT, "count must equal the number of systems");
  if (h_offsets) {
    for (int k = 0; k < count; ++k) h_offsets[k] = m->sys_lo[k];
    h_offsets[count] = m->n;
  }
  if (!h_failed && !h_logdet) return HSS_OK;
  HSS_CHECK(m->state != 0 && m->dinfo && m->dlogdet, HSS_ERR_BAD_STATE, "matrix has not been factored");
  hipStream_t s = ctx->stream;
  std::vector<int32_t> info(4 + m->nsys);
  std::vector<double> ld(m->nnodes + 1);
  HSS_HIP(hipMemcpyAsync(info.data(), m->dinfo, sizeof(int32_t) * info.size(), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipMemcpyAsync(ld.data(), m->dlogdet, sizeof(double) * ld.size(), hipMemcpyDeviceToHost, s));
  HSS_HIP(hipStreamSynchronize(s));
  if (h_failed)
    for (int k = 0; k < count; ++k) h_failed[k] = info[4 + k];
  if (h_logdet) {
    for (int k = 0; k < count; ++k) h_logdet[k] = 0.0;
    for (int j = 0; j < m->nnodes; ++j) h_logdet[m->nodes[j].sys] += ld[j];
  }
  HSS_API_END
}

hss_status hss_use_graphs(hss_ctx_t ctx, hss_matrix_t m, int32_t on) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  drop_graphs(m);
  m->use_graph = on != 0;
  HSS_API_END
}

hss_status hss_autotune(hss_ctx_t ctx, hss_matrix_t m, int32_t precision, int32_t reps, float* h_report) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(precision >= HSS_P_FP64 && precision <= HSS_P_BF16X3, HSS_ERR_INVALID_ARGUMENT, "unknown precision");
  HSS_CHECK(reps >= 1 && reps <= 100, HSS_ERR_INVALID_ARGUMENT, "reps must be in [1, 100]");
  std::vector<float> rep;
  autotune(m, precision, reps, &rep);
  if (h_report)
    for (size_t i = 0; i < rep.size(); ++i) h_report[i] = rep[i];
  HSS_API_END
}

hss_status hss_gemm_variants(hss_matrix_t m, int32_t precision, int32_t* h_out, int64_t capacity, int64_t* needed) {
  HSS_API_BEGIN
  HSS_CHECK(m && needed, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  const auto& plan = precision == HSS_P_FP64 ? m->gemm_plan : m->gemm_plan32;
  int64_t k = 0;
  for (auto& st : plan)
    for (auto& g : st) {
      if (h_out && k < capacity) h_out[k] = g.variant;
      ++k;
    }
  *needed = k;
  HSS_API_END
}

hss_status hss_set_gemm_variants(hss_ctx_t ctx, hss_matrix_t m, int32_t precision, const int32_t* h_variants,
                                 int64_t count) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && m && h_variants, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(precision >= HSS_P_FP64 && precision <= HSS_P_BF16X3, HSS_ERR_INVALID_ARGUMENT, "unknown precision");
  prepare_factor(m, precision);
  auto& plan = precision == HSS_P_FP64 ? m->gemm_plan : m->gemm_plan32;
  int64_t k = 0;
  for (auto& st : plan) k += (int64_t)st.size();
  HSS_CHECK(count == k, HSS_ERR_INVALID_ARGUMENT, "count must equal the number of GEMM batches");
  for (int64_t i = 0; i < count; ++i)
    HSS_CHECK(h_variants[i] >= 0 && h_variants[i] < kGemmVariants, HSS_ERR_INVALID_ARGUMENT, "unknown tile shape");
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  drop_graphs(m);
  k = 0;
  for (auto& st : plan)
    for (auto& g : st) g.variant = h_variants[k++];
  HSS_API_END
}

}  // extern "C"
