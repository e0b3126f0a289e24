// Internal definitions shared by the HIP translation units of libhss.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "hss.h"

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------

namespace hss {

void set_error(const std::string& msg);

struct Error {
  hss_status st;
  std::string msg;
};

#define HSS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::hss::Error{HSS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HSS_CHECK(cond, code, msg)                  \
  do {                                              \
    if (!(cond)) throw ::hss::Error{(code), (msg)}; \
  } while (0)

// ---------------------------------------------------------------------------
// per-node descriptor; every stage is a contiguous range of node indices and
// the tree links are explicit, so one object can hold a forest of trees
// ---------------------------------------------------------------------------

struct NodeDesc {
  int64_t lo;     // first tree position of the node's points
  int64_t offD;   // leaf: dense block D (n x n), else -1
  int64_t offB;   // basis (n x r): U at a leaf, E above; -1 at the root
  int64_t offS;   // coupling of the children (r_c1 x r_c2); -1 at a leaf
  int64_t offF;   // factor block (n x n) in [R;S] order
  int64_t offM;   // merged diagonal block (n x n), upper nodes only
  int64_t offV;   // Householder vectors (n x r)
  int64_t offT;   // triangular factor T of the compact WY form (r x r)
  int64_t offSg;  // signs of the S coordinates (r)
  int64_t offW;   // level scratch for W and Z (n x r each, 2 n r)
  int64_t offX;   // level scratch for r x r products (2 r r)
  int64_t offVec; // per-node vector slot (n rows) in solve workspaces
  int64_t offR;   // per-node rank slot (r rows) in matvec workspaces
  int32_t npts;   // points below the node
  int32_t n;      // size of the node's diagonal block in the ULV sweep
  int32_t r;      // basis rank (0 at the root)
  int32_t m;      // n - r (redundant rows eliminated at this node)
  int32_t level;
  int32_t child_row;  // row offset of this node's skeleton part in the parent's block
  int32_t parent;     // index of the parent node, -1 at a root
  int32_t c1, c2;     // indices of the children, -1 at a leaf
  int32_t sys;        // system (tree) the node belongs to
};

// A stage is a contiguous range of nodes processed by one launch of each step:
// one tree level for a single matrix (leaves first), one height above the
// leaves for a forest of several matrices. Roots of a stage come last.
struct LevelPlan {
  int32_t level;       // tree level (single matrix) or height (forest), for labels
  int32_t first;       // first node index of the stage
  int32_t count;       // nodes in the stage
  int32_t nmax, rmax, mmax;
  int32_t leaf;        // 1 for the stage of the leaves
  int32_t inv;         // 1 if the LDS Cholesky + explicit inverse path is used
  int32_t root_first;  // first root of the stage (first + count if none)
  int32_t root_split;  // 1 if the stage holds only roots with 96 < n <= 192: each is
                       // factored as two LDS blocks of h = (n + 1) / 2 and n - h
                       // (leading block with its S rows, then the trailing Schur
                       // complement), both with explicit inverses
};

// Split point of a root factored in two LDS blocks (LevelPlan::root_split).
__host__ __device__ inline int root_split_h(int n) { return (n + 1) / 2; }

// Size limits: rows of a diagonal block (a leaf, or two children's skeletons
// merged), the rank of a node, and the sample columns of a construction.
constexpr int kMaxBlock = 1024;
constexpr int kMaxRank = 512;
constexpr int kMaxSamples = 512;

// Batched GEMM entry: C = alpha * op(A) op(B) + beta * Cin, optional symmetric
// permutation of the output from [S;R] to [R;S] order (perm_r = r > 0).
struct GemmDesc {
  const void* A;
  const void* B;
  const void* Cin;
  void* C;
  int32_t m, n, k;
  int32_t lda, ldb, ldcin, ldc;
  int32_t perm_r;  // 0: plain store; r > 0: index t -> (t < r ? t + (dim - r) : t - r)
  int32_t perm_in; // 1: Cin is read at the permuted position too (in-place update)
  void* C2;        // optional second output (same values, same layout as C)
  int32_t lower_only;  // 1: square output; skip tiles lying entirely above the diagonal after the permutation
  int32_t kswap;       // > 0: op(B)'s k index is rotated, k -> (k + kswap) mod k (B = [X Y] read as [Y X])
};

constexpr int kGemmVariants = 8;  // compiled tile shapes of the batched GEMM

struct GemmBatch {
  std::vector<GemmDesc> host;
  GemmDesc* dev = nullptr;
  int32_t count = 0;
  int32_t mmax = 0, nmax = 0;
  int32_t variant = 0;  // tile shape, set by the autotuner
  int32_t compute = HSS_P_FP64;  // hss_precision of the products (storage stays FP64)
};

// Autotuning: while a recorder is installed on the calling thread, every
// batched GEMM launch is bracketed by two HIP events.
struct TuneRec {
  struct Rec {
    const GemmBatch* batch;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};
extern thread_local TuneRec* g_tune;

struct GemmTimer {
  TuneRec* t = nullptr;
  hipEvent_t b = nullptr;
  hipStream_t s = nullptr;
  GemmTimer(const GemmBatch& g, hipStream_t st);
  ~GemmTimer();
};

}  // namespace hss

// ---------------------------------------------------------------------------
// context and matrix objects
// ---------------------------------------------------------------------------

namespace hss {
struct Blr2State;  // BLR^2-ULV factors of a matrix (blr2.hip)
struct ProfRec {
  const char* name;
  int32_t level;
  hipEvent_t a, b;
};
}  // namespace hss

struct hss_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hss_allocator allocator{nullptr, nullptr, nullptr};  // the caller's device allocator (alloc NULL: hipMalloc)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // per-launch event profiling (off unless enabled)
  bool prof = false;
  std::vector<hss::ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  hipStream_t cap_stream = nullptr;  // non-blocking stream used only to record graphs
  hipStream_t aux_stream = nullptr;  // second stream for work off the critical path
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_trail = nullptr;  // fused factor + solve: a stage factored / the forward sweep done
};

struct hss_matrix_s {
  hss_ctx_t ctx = nullptr;
  int64_t n = 0;
  int32_t L = 0;
  int32_t nnodes = 0;
  int32_t state = 0;  // 0 constructed, 1 factored, 2 failed
  int32_t precision = 0;
  int32_t failed_level = -1, failed_node = -1, failed_pivot = -1, failed_system = -1;

  std::vector<hss::NodeDesc> nodes;  // host copy
  hss::NodeDesc* dnodes = nullptr;   // device copy
  std::vector<hss::LevelPlan> levels;  // single matrix: indexed by tree level
  std::vector<hss::LevelPlan> stages;  // processing order, leaves first
  int32_t nsys = 1;                    // systems in the matrix (a forest for batches)
  std::vector<int64_t> sys_lo;         // first global row of each system
  std::vector<int32_t> sys_root;       // root node of each system

  // representation (device)
  double* dD = nullptr;
  double* dB = nullptr;
  double* dS = nullptr;
  int64_t* dperm = nullptr;  // tree position -> caller index
  int64_t lenD = 0, lenB = 0, lenS = 0;

  // factor (device)
  double* dF = nullptr;
  double* dM = nullptr;
  double* dV = nullptr;
  double* dT = nullptr;
  double* dSg = nullptr;
  double* dW = nullptr;
  double* dX = nullptr;
  // explicit L_RR^{-1} (levels whose m <= 96) and the L_SR scratch of those levels
  std::vector<int64_t> offLi, offS2;
  int64_t* dOffLi = nullptr;
  int64_t* dOffS2 = nullptr;
  double* dLi = nullptr;
  double* dS2 = nullptr;
  int64_t lenLi = 0, lenS2 = 0;
  int32_t* dinfo = nullptr;  // [0] status, [1] node, [2] pivot
  double* dlogdet = nullptr; // per node partial sums
  int64_t lenF = 0, lenM = 0, lenV = 0, lenT = 0, lenSg = 0, lenW = 0, lenX = 0;
  bool factor_ready = false;
  std::vector<std::vector<hss::GemmBatch>> gemm_plan;  // per stage, per step
  std::vector<char> inv_used64;  // per stage: 1 explicit inverse factor, 2 split root, 0 neither
  // called once the kernels of factor stage si are enqueued (fused factor + solve)
  std::function<void(int)> after_stage;

  // mixed precision: the same FP64 buffers and GEMM batches, with the leaf
  // stage's products computed on FP32 or BF16 matrix cores (own tile
  // choices, shared by the three low precisions)
  bool mixed_ready = false;
  int32_t promoted = 0;  // leaves of the last mixed factorization redone in FP64
  int32_t mixed_prec = HSS_P_FP32;  // precision of the leaf products of the mixed factorization
  bool mixed_all64[4] = {};  // per hss_precision: found unsuitable for this matrix, mixed runs FP64
  double* dpmin = nullptr;   // per node: smallest pivot of its last partial Cholesky
  std::vector<double> leaf_scale;  // per node (leaves): |D|_inf, the rounding error scale
  std::vector<char> fp64_leaf;     // per node: leaf redone in FP64 by the last mixed factorization
  std::vector<std::vector<hss::GemmBatch>> gemm_plan32;

  // BLR^2-ULV factorization of the leaf level (Alg. 1); nullptr until used
  hss::Blr2State* blr2 = nullptr;

  // solve / matvec workspaces (device), sized for ws_nrhs columns
  double* dvec = nullptr;   // per-node vectors, sum(n) x nrhs
  double* dxt = nullptr;    // matvec up-sweep, sum(r) x nrhs
  double* dyt = nullptr;    // matvec down-sweep, sum(r) x nrhs
  int64_t ws_nrhs = 0;
  int64_t sum_n = 0, sum_r = 0;
  double* dtmp = nullptr;   // refinement temporaries (4 x N x nrhs)
  int64_t tmp_len = 0;

  double factor_ms = 0.0, solve_ms = 0.0;
  int32_t max_rank = 0;
  hss_construct_stats cstats{};

  // HIP graphs of the factorization (per precision) and of the last solve
  bool use_graph = false;
  hipGraphExec_t gexec_factor[2] = {nullptr, nullptr};
  hipGraphExec_t gexec_solve = nullptr;
  struct SolveKey {
    int prec = -1;
    const double* b = nullptr;
    double* x = nullptr;
    int64_t nrhs = 0, ld = 0;
    const void* ws = nullptr;  // the per-node vector workspace the recording used
    bool operator==(const SolveKey& o) const {
      return prec == o.prec && b == o.b && x == o.x && nrhs == o.nrhs && ld == o.ld && ws == o.ws;
    }
  } solve_key;
};

namespace hss {

// Brackets the launches issued in its scope with two events on the context
// stream when profiling is enabled.
struct Prof {
  hss_ctx_t ctx;
  size_t idx = (size_t)-1;
  Prof(hss_ctx_t c, const char* name, int level);
  ~Prof();
};

// allocation helpers (throw on failure): the allocator of the context set by
// the innermost CtxScope on this thread, else hipMalloc
void* dev_alloc(size_t bytes);
void dev_free(void* p);
extern thread_local hss_ctx_t g_alloc_ctx;
struct CtxScope {
  hss_ctx_t prev;
  explicit CtxScope(hss_ctx_t c) : prev(g_alloc_ctx) { g_alloc_ctx = c; }
  ~CtxScope() { g_alloc_ctx = prev; }
  CtxScope(const CtxScope&) = delete;
  CtxScope& operator=(const CtxScope&) = delete;
};

// Sample sizing of one construction attempt (construct.hip).
struct SamplePlan {
  hss_rankmlp_t model = nullptr;  // chooses s_basis when it is 0
  int s_basis = 0;                // sample columns for the bases
  int probes = 0;                 // probe columns for the judge (0: no judge)
  double judge_thr = 0.0;         // fail a node when its probe residual exceeds this
  bool abort_on_fail = false;     // stop at the first level with a failed node
  // outputs
  int judge_failures = 0;
  int predicted_max = 0;
  int64_t sample_bytes = 0;
  bool passed = true;
};
bool construct(hss_matrix_t m, const double* d_points, int32_t dim, const hss_kernel& kern,
               const hss_construct_opts& o, const double* d_omega, int32_t s_avail, SamplePlan& sp);

// representation setup (capi.hip)
void layout_representation(hss_matrix_t m);
void assign_offsets(hss_matrix_t m);
void finish_stages(hss_matrix_t m);

// gemm.hip
void gemm_upload(GemmBatch& b, hipStream_t s);
void gemm_free(GemmBatch& b);
void gemm_launch_f64(const GemmBatch& b, bool ta, bool tb, double alpha, double beta, hipStream_t s);
void gemm_launch_f32(const GemmBatch& b, bool ta, bool tb, float alpha, float beta, hipStream_t s);

// factor.hip
void factor_fp64(hss_matrix_t m);
void factor_mixed(hss_matrix_t m, int precision);
double read_logdet(hss_matrix_t m);
void factor_leaf_stage_fp64(hss_matrix_t m);
void free_factor(hss_matrix_t m);

void prepare_factor(hss_matrix_t m, int precision);
void factor_solve_fp64(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld);

// batch.hip: forest layout, graph replay, autotuning
void factor_run(hss_matrix_t m, int precision);
void solve_run(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld);
void drop_graphs(hss_matrix_t m);

// solve.hip
void ensure_vec_ws(hss_matrix_t m, int64_t nrhs);
void solve_fp64(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld);
void solve_fp64_ws(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld, double* vec);
void solve_leaf_sweep(hss_matrix_t m, bool forward, const double* b, double* x, int64_t nrhs, int64_t c0, int nc,
                      int64_t ld);
int solve_chunk();

// blr2.hip: releases the BLR^2-ULV factors of a matrix; marks them stale (any
// other factorization overwrites the leaf factors they share)
void blr2_free(hss_matrix_t m);
void blr2_invalidate(hss_matrix_t m);

// noalloc.hip: resolves the static scratch array's address on the current device
void noalloc_init(int device);
void matvec_fp64(hss_matrix_t m, const double* x, double* y, int64_t nrhs, int64_t ld);

// tree.hip: node ranges of the bisection tree from the point count (leaf i
// owns [leaf_lo[i], leaf_lo[i+1])), and the tree itself on the device: d_perm
// (n entries) receives tree position -> caller's index, d_leafbox (nullable,
// 2^L x 6: lo[3], hi[3], zero beyond dim) the leaves' bounding boxes.
// Synchronizes the stream.
std::vector<int64_t> tree_leaf_lo(int64_t n, int L);
void build_tree(hipStream_t st, const double* d_points, int64_t n, int dim, int L, int64_t* d_perm,
                double* d_leafbox);

// construct.hip


}  // namespace hss
