/*
 * hss.h - C ABI of the MI355X HSS-ULV library (libhss.so).
 *
 * The library builds a Hierarchically Semi-Separable (HSS) approximation of an
 * SPD kernel matrix on a point set, factors it with the HSS-ULV algorithm and
 * solves with the ULV forward/backward sweeps (Deshmukh, Ma, Yokota, Bosilca,
 * "O(N) distributed direct factorization of structured dense matrices using
 * runtime systems", ICPP 2023: Sec. 2 construction and notation, Sec. 3.2
 * Alg. 2 factorization and Eq. 17 solve).
 *
 * Conventions
 *  - Every matrix is column-major FP64 unless stated. Leading dimensions are
 *    in elements.
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees or retains them beyond the call. Host pointers are read
 *    during the call only.
 *  - Work is enqueued on the context's HIP stream. Calls that return host
 *    values (status of a factorization, log-determinant, ranks during
 *    construction, refinement statistics) synchronize that stream.
 *  - Vectors passed to solve/matvec are in the caller's point order; the
 *    library gathers and scatters through the tree permutation.
 *  - No C++ exception crosses this boundary. Each call returns an hss_status;
 *    hss_last_error() gives a thread-local message for the last failure.
 *  - One context per host thread. Calls that overlap on one matrix race.
 */
#ifndef HSS_H_
#define HSS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hss_ctx_s* hss_ctx_t;
typedef struct hss_matrix_s* hss_matrix_t;
typedef struct hss_rankmlp_s* hss_rankmlp_t;  /* learned rank model (see below) */

typedef enum {
  HSS_OK = 0,
  HSS_ERR_INVALID_ARGUMENT = 1,
  HSS_ERR_NOT_SPD = 2,        /* a pivot block was not positive definite */
  HSS_ERR_OUT_OF_MEMORY = 3,
  HSS_ERR_DEVICE = 4,         /* a HIP runtime call failed */
  HSS_ERR_BAD_STATE = 5,      /* e.g. solve before factor */
  HSS_ERR_NOT_CONVERGED = 6,  /* iterative refinement did not reach its tolerance */
  HSS_ERR_UNSUPPORTED = 7
} hss_status;

/* Kernel families: the covariance kernels of the workloads and the Green's
 * functions of Table 3 (Laplace 2D, Yukawa; the paper's Matern with nu = 1/2
 * is HSS_K_EXPONENTIAL with length = mu). A_ij = f(|x_i - x_j|) + nugget*delta_ij. */
typedef enum {
  HSS_K_EXPONENTIAL = 0, /* sigma2 * exp(-d/length) */
  HSS_K_MATERN32 = 1,    /* sigma2 * (1 + sqrt3 d/length) exp(-sqrt3 d/length) */
  HSS_K_GAUSSIAN = 2,    /* sigma2 * exp(-d^2/length^2) */
  HSS_K_LAPLACE2D = 3,   /* -ln(eps + d) */
  HSS_K_YUKAWA = 4       /* exp(-alpha (eps + d)) / (eps + d) */
} hss_kernel_kind;

typedef struct {
  int32_t kind;     /* hss_kernel_kind */
  double length;    /* > 0 for the covariance kernels */
  double sigma2;    /* variance scale of the covariance kernels (usually 1) */
  double nugget;    /* >= 0, added on the diagonal only */
  double alpha;     /* Yukawa decay (Table 3: 1) */
  double eps;       /* Laplace/Yukawa regulariser (Table 3: 1e-9) */
} hss_kernel;

/* Construction modes; both sample each node's off-diagonal row block with the
 * caller's Gaussian test matrix and give the paper's format (orthonormal nested
 * bases U/E and couplings S, Sec. 2 Eq. 6).
 *  PLAIN: the paper's construction (Sec. 2, Eq. 2): each node's basis is the
 *         first k columns of the pivoted QR of the samples of its off-diagonal
 *         row block, projected onto the children's bases above the leaves, and
 *         each sibling coupling is the orthogonal projection of the exact block.
 *         The compressed matrix can be indefinite where the truncation error
 *         exceeds the smallest eigenvalues (the factorization then reports
 *         NOT_SPD).
 *  SCALED: the samples of a node are first scaled by the inverse Cholesky
 *         factor of its diagonal block, which keeps the HSS matrix SPD for any
 *         truncation (at a larger truncation error on smooth kernels). */
typedef enum { HSS_COMPRESS_PLAIN = 0, HSS_COMPRESS_SCALED = 1 } hss_compress_mode;

typedef struct {
  int32_t leaf_size;   /* 2..1024: maximum points per leaf */
  int32_t levels;      /* 0 = derive ceil(log2(N/leaf_size)); otherwise must equal it */
  int32_t rank;        /* 1..512 fixed rank per node; 0 = adaptive by tol */
  int32_t max_rank;    /* cap for adaptive ranks (0 = 128; at most 512) */
  double tol;          /* adaptive truncation: keep pivots with |R_jj| > tol*|R_00| */
  int32_t mode;        /* hss_compress_mode */
  /* Sample sizing (adaptive ranks, tol > 0). With neither of the two below,
   * all s columns of the test matrix are samples. Otherwise the last `probes`
   * columns form an independent probe and the first s_b columns the samples:
   * after the pivoted QR of each node, the judge computes
   * |(I - Q Q^T) Y_probe|_F / |Y_probe|_F for the node's scaled probe samples
   * and fails the node when it exceeds judge_factor * tol; any failure restarts
   * the construction with 2 s_b samples, up to s - probes (the last attempt is
   * kept whatever the judge says). */
  hss_rankmlp_t rank_model;  /* trained model: s_b = (largest predicted node rank) + 8 */
  int32_t sample_start;      /* without a model: s_b starts here (adaptive doubling) */
  int32_t probes;            /* probe columns (0 = 8) */
  double judge_factor;       /* 0 = 10 */
} hss_construct_opts;

/* Precision of the factorization (the mixed-precision form of the path; the paper
 * itself is FP64). All leave FP64 factors, applied by the same FP64 solve.
 *  FP64: every step in FP64.
 *  FP32: the leaf stage's four contractions of the diagonal product (Eq. 7:
 *        W = M Y, C = Y^T W, Z = W - V C / 2 and the rank-2r update of M) run
 *        on FP32 matrix cores, operands rounded to FP32, FP32 accumulation,
 *        the FP64 block M added to the product in FP64. The basis QR (the
 *        orthogonal transform itself), every pivot block and partial
 *        Cholesky, triangular solve and Schur complement (Eq. 10-12), and the
 *        stages above the leaves (whose blocks carry the growing norms of the
 *        merged Schur complements) stay FP64. Accuracy guard, in the same
 *        call: a leaf whose FP64 pivot fails after the FP32 products, or whose
 *        smallest pivot is below 2^-18 |D|_inf (largest absolute row sum;
 *        there the FP32 rounding of its products, about u32 |D|_inf, would be
 *        an O(1) relative error), is redone in FP64 before the stage above;
 *        a node above the leaves whose pivot
 *        fails (its block made indefinite by the perturbation below it) has
 *        its whole subtree and its ancestors redone in FP64. When at least half
 *        of the leaves are redone, later FP32 factorizations of the same matrix
 *        run FP64 from the start. hss_info.promoted_nodes counts the leaves
 *        factored in FP64. The result factors the HSS matrix with its other
 *        leaf blocks perturbed by the FP32 rounding: refine with
 *        hss_ulv_solve_refined.
 *  BF16: as FP32, with the four contractions on BF16 matrix cores (operands
 *        rounded to BF16, FP32 accumulation). Guard: smallest pivot below
 *        2^-2 |D|_inf, so only leaves whose redundant blocks keep pivots
 *        within a factor 4 of |D|_inf stay BF16 (strongly diagonally
 *        dominant leaves); the leaves of smooth kernels are redone in FP64.
 *  BF16X3: as BF16 with each operand split into two BF16 parts, x = hi + lo,
 *        and the products formed as hi*hi + hi*lo + lo*hi (FP32
 *        accumulation): about 2^-16 relative error per product. Guard:
 *        smallest pivot below 2^-10 |D|_inf.
 * The guard and the switch to FP64 after half of the leaves were redone apply
 * per precision; the three low precisions share one set of GEMM tile shapes
 * (hss_autotune, hss_set_gemm_variants). */
typedef enum {
  HSS_P_FP64 = 0,
  HSS_P_FP32 = 1,
  HSS_P_BF16 = 2,
  HSS_P_BF16X3 = 3
} hss_precision;

typedef struct {
  int32_t precision;   /* hss_precision */
} hss_factor_opts;

/* Host description of an HSS matrix, used by hss_import and hss_export.
 * Nodes are numbered in heap order: node 0 is the root, node k has children
 * 2k+1 and 2k+2; the leaves are nodes 2^L - 1 .. 2^(L+1) - 2 (L = levels).
 *  leaf_lo: 2^L + 1 entries; leaf i owns tree positions [leaf_lo[i], leaf_lo[i+1]).
 *  rank:    2^(L+1) - 1 entries, basis columns of each node (rank[0] ignored).
 *  D:       leaf diagonal blocks n_i x n_i, packed leaf after leaf.
 *  U:       leaf bases n_i x rank_i, packed leaf after leaf.
 *  E:       transfer matrices of nodes 1 .. 2^L - 2 (levels 1..L-1) in heap order,
 *           (rank[2k+1] + rank[2k+2]) x rank[k] each, packed.
 *  S:       couplings of the children of nodes 0 .. 2^L - 2 in heap order,
 *           rank[2k+1] x rank[2k+2] each, packed.
 *  perm:    N entries, tree position -> caller's point index (NULL = identity).
 * For L = 0 the matrix is the single block D (N x N). */
typedef struct {
  int64_t n;
  int32_t levels;
  const int64_t* leaf_lo;
  const int32_t* rank;
  const double* D;
  const double* U;
  const double* E;
  const double* S;
  const int64_t* perm;
} hss_desc;

/* Output view for hss_export: the caller provides buffers of at least the
 * sizes that hss_export_sizes reports. */
typedef struct {
  int64_t* leaf_lo;
  int32_t* rank;
  double* D;
  double* U;
  double* E;
  double* S;
  int64_t* perm;
} hss_desc_out;

typedef struct {
  int64_t n;
  int32_t levels;
  int32_t factored;          /* 1 after a successful hss_ulv_factor */
  int32_t precision;         /* precision of the last factorization */
  int32_t max_rank;          /* largest basis rank */
  int32_t failed_level;      /* on HSS_ERR_NOT_SPD: level of the failing node, else -1 */
  int32_t failed_node;       /* index of the failing node (heap index for a single tree), else -1 */
  int32_t failed_pivot;      /* local pivot index that failed, else -1 */
  int64_t bytes_representation;
  int64_t bytes_factor;
  double factor_ms;          /* device time of the last factorization (HIP events) */
  double solve_ms;           /* device time of the last solve */
  int32_t systems;           /* 1, or the number of systems of a batch */
  int32_t failed_system;     /* on HSS_ERR_NOT_SPD: system of the failing node, else -1 */
  int32_t promoted_nodes;    /* FP32 factorization: leaves factored in FP64 (accuracy guard) */
} hss_info;

/* ---- context ------------------------------------------------------------ */

/* Device memory for the library's own buffers (the representation, factors,
 * workspaces): alloc returns at least `bytes` of device memory on the
 * context's device (NULL on failure), free takes back a block alloc returned.
 * A block is freed through the allocator it came from, after the device has
 * finished all work (the library synchronizes the device first). Both NULL:
 * hipMalloc and hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} hss_allocator;

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream) and allocates the library's
 * device memory through `allocator` (NULL, or both functions NULL: hipMalloc;
 * copied, so the struct may be freed on return). Every later call with this
 * context -- and hss_matrix_destroy of its matrices -- uses that allocator.
 * Also resolves the static scratch array of hss_ulv_solve_noalloc on the
 * device. Errors: INVALID_ARGUMENT for NULL out, a bad device index or an
 * allocator with only one of its functions. */
hss_status hss_ctx_create(int32_t device, void* hip_stream, const hss_allocator* allocator, hss_ctx_t* out);
hss_status hss_ctx_destroy(hss_ctx_t ctx);
/* Replaces the stream work is enqueued on. */
hss_status hss_ctx_set_stream(hss_ctx_t ctx, void* hip_stream);

/* ---- construction (Sec. 2) ----------------------------------------------- */

/* Builds the HSS approximation of the kernel matrix on the points.
 *  d_points: N x dim, row-major (point-major), device memory, caller's order.
 *  d_omega:  N x s Gaussian test matrix, column-major with ld = N, rows in the
 *            caller's point order, device memory; s >= rank (fixed rank) or
 *            s >= the largest rank to be found (adaptive).
 * Steps: recursive coordinate bisection (longest box side, ties -> lowest
 * axis, order by (coordinate, index), left child = ceil(size/2)); leaf blocks
 * by kernel evaluation; randomized compression (opts->mode) level by level
 * with column-pivoted QR truncation (Eq. 2). Synchronizes once per level. Errors: INVALID_ARGUMENT for bad sizes or options,
 * NOT_SPD if a diagonal block is not positive definite. */
hss_status hss_construct(hss_ctx_t ctx, const double* d_points, int64_t n, int32_t dim,
                         const hss_kernel* kernel, const hss_construct_opts* opts,
                         const double* d_omega, int32_t s, hss_matrix_t* out);

/* What the sample sizing did in the last hss_construct of a matrix. */
typedef struct {
  int32_t samples;          /* sample columns of the kept attempt (s_b) */
  int32_t probes;           /* probe columns (0 when no judge ran) */
  int32_t attempts;         /* constructions run (1 + restarts) */
  int32_t judge_failures;   /* nodes failed by the judge over all attempts */
  int32_t predicted_max;    /* largest rank the model predicted (0 without a model) */
  int32_t max_rank;         /* largest rank kept */
  int64_t sample_bytes;     /* device bytes of the N x (s_b + probes) sample buffers of the kept attempt */
} hss_construct_stats;
hss_status hss_get_construct_stats(hss_matrix_t m, hss_construct_stats* out);

/* Uploads a host HSS matrix in the paper's format (Sec. 2): leaf dense blocks
 * D, leaf shared bases U, the transfer matrices E of the nested bases (Eq. 6:
 * the basis of a parent is blkdiag(children's bases) times E), and the
 * skeleton couplings S of sibling pairs; layout in hss_desc. Copies everything
 * (the host buffers may be freed on return) and synchronizes. Leaves the
 * matrix CONSTRUCTED. Errors: INVALID_ARGUMENT for NULL or inconsistent sizes
 * or a perm that is not a permutation (leaves of more than 1024 points
 * included); UNSUPPORTED for blocks above 1024 rows or ranks above 512. */
hss_status hss_import(hss_ctx_t ctx, const hss_desc* desc, hss_matrix_t* out);

/* Sizes (in elements) of the arrays hss_export writes: leaf_lo, rank, D, U, E, S, perm. */
hss_status hss_export_sizes(hss_matrix_t m, int64_t sizes[7]);
/* Copies the representation to host buffers. Synchronizes. */
hss_status hss_export(hss_ctx_t ctx, hss_matrix_t m, hss_desc_out* out);

/* ---- factorization and solve (Sec. 3.2) --------------------------------- */

/* HSS-ULV factorization (Alg. 2): per level from the leaves, the full-basis
 * QR [U^R U^S] of each node's basis, the diagonal product Q^T A Q (Eq. 7),
 * the partial Cholesky of the redundant rows (Eq. 10-12), the merge of sibling
 * Schur complements with their coupling into the parent block; then the
 * Cholesky of the root block. D/U/E/S are not modified. opts may be NULL (FP64).
 * Synchronizes to read the pivot status. Errors: NOT_SPD with the failing
 * (level, node, pivot) in hss_info. */
hss_status hss_ulv_factor(hss_ctx_t ctx, hss_matrix_t m, const hss_factor_opts* opts);

/* ULV solve (Eq. 17): x = A^{-1} b for nrhs columns. d_b, d_x: N x nrhs,
 * column-major with leading dimension ld >= N, caller's order, device memory;
 * d_x may equal d_b. Requires a successful factorization (BAD_STATE otherwise).
 * The solve is FP64 whatever the precision of the factorization (every
 * precision leaves FP64 factors). */
hss_status hss_ulv_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                         int64_t nrhs, int64_t ld);

/* The solve of hss_ulv_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same launches and results, bit for bit, with the per-node
 * vector workspace taken from a static device array of 2^22 doubles (32 MiB,
 * resolved by hss_ctx_create and held by each GPU until the process ends)
 * instead of the matrix's own workspace. Nothing is allocated, no graph is
 * recorded, and per-launch profiling is bypassed. The workspace needs
 * sum_n x nrhs doubles, sum_n being the sum of the block sizes of all nodes
 * (N plus, over the non-leaf nodes, the sum of their children's ranks; 458 560
 * at N = 262144, leaf 256, rank 96: up to nine right-hand sides); larger
 * requests fail with UNSUPPORTED and a message naming the limit. Every call on
 * one GPU shares the array: calls that overlap on one GPU (two streams, two
 * threads) race. Arguments, state and errors as hss_ulv_solve. */
hss_status hss_ulv_solve_noalloc(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x, int64_t nrhs,
                                 int64_t ld);

/* FP64 factorization and solve in one call (Alg. 2, then Eq. 17): the same
 * results as hss_ulv_factor (FP64) followed by hss_ulv_solve, for callers that
 * hold the right-hand sides at factorization time. A stage's forward sweep
 * needs only that stage's factors, so it runs on a second stream while the
 * stages above it are factored; the backward sweep follows the root. Leaves
 * the matrix FACTORED (or FAILED, with NOT_SPD as hss_ulv_factor; d_x is then
 * undefined). Arguments as hss_ulv_solve; d_x may equal d_b. hss_info's
 * factor_ms receives the time of the whole call. Synchronizes. */
hss_status hss_ulv_factor_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                                int64_t nrhs, int64_t ld);

/* Solve with iterative refinement: x_{k+1} = x_k + solve(b - A x_k), the
 * residual by the FP64 HSS matvec, until |b - A x|_2 <= tol |b|_2 for every
 * column, or max_iters corrections. If the residual stalls, switches to
 * preconditioned conjugate gradients with the factorization as preconditioner.
 * iters_out / relres_out (host, nullable) receive the correction count and the
 * largest final relative residual. Errors: NOT_CONVERGED (x holds the best iterate). */
hss_status hss_ulv_solve_refined(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                                 int64_t nrhs, int64_t ld, double tol, int32_t max_iters,
                                 int32_t* iters_out, double* relres_out);

/* FP64 HSS matrix-vector product y = A x with the nested-basis form of Sec. 2
 * (Eq. 6): up-sweep x~ = U^T x at the leaves and E^T [x~_c1; x~_c2] above,
 * sibling couplings y~_c1 = S x~_c2 and y~_c2 = S^T x~_c1, down-sweep
 * [y~_c1; y~_c2] += E y~, and y = D x + U y~ at the leaves. This is the product
 * A b of the construction error (Eq. 18) and the residual of the refinement.
 * d_x, d_y: N x nrhs device memory, column-major with ld >= N, caller's point
 * order; they must not alias. Allowed in any state after construction/import.
 * Errors: INVALID_ARGUMENT for NULL, aliasing or bad sizes. */
hss_status hss_matvec(hss_ctx_t ctx, hss_matrix_t m, const double* d_x, double* d_y,
                      int64_t nrhs, int64_t ld);

/* log det A = 2 * sum of log pivots of every L_RR and of the root factor
 * (the orthogonal transforms have |det| = 1). Requires FACTORED. Synchronizes. */
hss_status hss_logdet(hss_ctx_t ctx, hss_matrix_t m, double* h_out);

/* BLR^2-ULV (Sec. 3.1, Alg. 1), a variant factorization of the same matrix:
 * the leaf blocks with their shared bases are read as a weakly admissible
 * BLR^2 matrix (Sec. 2, the coupling between leaves i and j being their lowest
 * common ancestor's S carried into the leaf bases by the transfer matrices of
 * Eq. 6). Alg. 1: the diagonal product and partial Cholesky of every leaf
 * (Eq. 7, 10-12; the leaf stage of hss_ulv_factor), the permutation of all
 * skeleton rows to the end, and one dense Cholesky of that K x K skeleton
 * matrix (Eq. 13), K = sum of the leaf ranks. Storage K^2 doubles, work
 * K^3 / 3 flops: the cost that the nested basis of the HSS-ULV avoids.
 * Single trees whose leaves all sit on the deepest level; K <= 65536
 * (UNSUPPORTED otherwise). Shares the leaf factor buffers with hss_ulv_factor:
 * each factorization leaves the other's stale (hss_ulv_solve then returns
 * BAD_STATE until hss_ulv_factor runs again, and vice versa). FP64 only.
 * Synchronizes. Errors: NOT_SPD (a leaf pivot or a pivot of the skeleton
 * matrix; the message names which), OUT_OF_MEMORY. */
hss_status hss_blr2_factor(hss_ctx_t ctx, hss_matrix_t m);

/* BLR^2-ULV solve (Eq. 14): the leaf forward sweep, the two triangular solves
 * with the skeleton matrix's Cholesky factor, the leaf backward sweep.
 * Arguments as hss_ulv_solve (d_x may equal d_b); BAD_STATE without a valid
 * hss_blr2_factor. */
hss_status hss_blr2_solve(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                          int64_t nrhs, int64_t ld);

/* log det A from the BLR^2-ULV factors: 2 * sum of log pivots of every leaf
 * L_RR and of the skeleton matrix's Cholesky factor. BAD_STATE without a
 * valid hss_blr2_factor. */
hss_status hss_blr2_logdet(hss_ctx_t ctx, hss_matrix_t m, double* h_out);

/* The skeleton matrix order K of the BLR^2-ULV (valid before any
 * factorization) and, in *factor_ms (nullable), the GPU time of the last
 * successful hss_blr2_factor (0 if none). Errors: UNSUPPORTED for shapes the
 * BLR^2-ULV does not take. */
hss_status hss_blr2_stats(hss_matrix_t m, int64_t* skeleton_rows, float* factor_ms);

hss_status hss_get_info(hss_matrix_t m, hss_info* out);
/* The basis rank of every node (Sec. 2: columns of U at a leaf, of E above;
 * 0 at a root), into h_out (host, nullable for a size query; capacity
 * entries), in node order: heap order for a constructed or imported single
 * matrix (node 0 the root, node k with children 2k+1 and 2k+2). *needed
 * receives the node count. Errors: INVALID_ARGUMENT for NULL or a short
 * buffer. */
hss_status hss_get_ranks(hss_matrix_t m, int32_t* h_out, int64_t capacity, int64_t* needed);
/* N entries: tree position -> caller's point index. */
hss_status hss_get_permutation(hss_ctx_t ctx, hss_matrix_t m, int64_t* d_perm);

/* Reads one intermediate block of the factorization to host memory, for
 * checking the steps of Alg. 2 one by one. what = 0: the node's Schur
 * complement Sigma (rank x rank) in the coordinates of its basis; what = 1:
 * the node's merged diagonal block before the transform (n x n; for the root,
 * the block that the final Cholesky factors); what = 2..5: the stored factor
 * data of the node as laid out on the device (2: Householder vectors V, n x r;
 * 3: the WY triangle T, r x r; 4: the factor block, n x n, [R;S] order;
 * 5: the r coordinate signs). Requires FACTORED. */
hss_status hss_debug_node_block(hss_ctx_t ctx, hss_matrix_t m, int32_t node, int32_t what,
                                double* h_out, int64_t capacity);

/* Per-launch timing: when enabled, every kernel launch of the factorization
 * and solve is bracketed by two HIP events on the context stream (this adds a
 * small gap per launch). Enabling or disabling clears the records. */
hss_status hss_profile_enable(hss_ctx_t ctx, int32_t on);
/* Writes one line per (step, level): "<step> <level> <launches> <total ms>\n"
 * into buf (NUL-terminated, truncated to capacity); *needed receives the full
 * size. Synchronizes. */
hss_status hss_profile_read(hss_ctx_t ctx, char* buf, int64_t capacity, int64_t* needed);

/* ---- batches of independent systems ------------------------------------ */
/* A batch holds several HSS systems of any sizes and depths in one matrix
 * object. Their tree nodes are regrouped by height above the leaves, so every
 * step of the level-by-level factorization (Alg. 2) and of the solve sweeps
 * (Eq. 17) is one launch for all systems; a system whose tree is shallower
 * finishes at a lower height. Vectors of a batch are the systems' vectors
 * stacked in batch order: system k owns rows [offset_k, offset_k + N_k) of b
 * and x, in its own point order (offsets from hss_batch_query). The batch's
 * hss_logdet is the sum over systems; hss_batch_query gives each one.
 * hss_ulv_factor fails with NOT_SPD if any system fails (hss_info names the
 * first failing system; hss_batch_query flags all of them). A batch cannot be
 * exported (UNSUPPORTED). */

/* Copies `count` single matrices (constructed or imported; not batches) into a
 * new batch. The inputs stay valid and independent. */
hss_status hss_batch_create(hss_ctx_t ctx, int32_t count, const hss_matrix_t* mats, hss_matrix_t* out);

/* hss_construct of each system (arrays of `count` entries; kernels, opts and
 * omega per system), then hss_batch_create of the results. */
hss_status hss_construct_batched(hss_ctx_t ctx, int32_t count, const double* const* d_points, const int64_t* n,
                                 int32_t dim, const hss_kernel* kernels, const hss_construct_opts* opts,
                                 const double* const* d_omega, const int32_t* s, hss_matrix_t* out);

/* Host outputs, each nullable: h_offsets (count + 1 entries: first row of each
 * system, then the total N), h_failed (count: 1 where the last factorization
 * met a non-positive pivot), h_logdet (count: per-system log-determinant of
 * the last factorization). Synchronizes when h_failed or h_logdet is given;
 * those require a factorization to have run (BAD_STATE otherwise). */
hss_status hss_batch_query(hss_ctx_t ctx, hss_matrix_t m, int32_t count, int64_t* h_offsets, int32_t* h_failed,
                           double* h_logdet);

/* ---- launch recording and tuning ---------------------------------------- */
/* When on, an FP64 hss_ulv_factor records its whole launch sequence (every
 * stage, every step) into a HIP graph on first use and afterwards replays it
 * with a single graph launch (the mixed-precision factorizations read their
 * promotion counts back between stages and are never recorded); hss_ulv_solve (and the solves inside
 * hss_ulv_solve_refined) does the same per (precision, b, x, nrhs, ld). The
 * recording uses a private non-blocking stream; replays go to the context
 * stream. Ignored while profiling is enabled. Switching drops all graphs.
 * Synchronizes. */
hss_status hss_use_graphs(hss_ctx_t ctx, hss_matrix_t m, int32_t on);

/* Autotuner of the batched GEMM tile shapes (M x N x K per workgroup: 0:
 * 64x64x16, 1: 32x32x16, 2: 128x64x16, 3: 64x128x16, 4: 32x32x64, 5:
 * 64x64x32, 6: 64x96x16, 7: 96x96x16): runs the factorization in `precision`
 * once untimed, then `reps` rounds of one factorization per tile shape (the
 * shapes take turns), timing every batched GEMM launch with HIP events, and
 * keeps for each (stage, step) the shape with the best time over the rounds.
 * h_report (nullable, 9 floats) receives the GEMM milliseconds per
 * factorization (best over the rounds) for each uniform shape and for the
 * tuned choice. Leaves the matrix CONSTRUCTED: factor
 * afterwards. Drops recorded graphs. Synchronizes. */
hss_status hss_autotune(hss_ctx_t ctx, hss_matrix_t m, int32_t precision, int32_t reps, float* h_report);

/* The chosen tile shape of every (stage, step) GEMM batch, in order, into
 * h_out (nullable, up to capacity entries); *needed receives the count. */
hss_status hss_gemm_variants(hss_matrix_t m, int32_t precision, int32_t* h_out, int64_t capacity, int64_t* needed);

/* Sets the tile shape of every (stage, step) GEMM batch (the order of
 * hss_gemm_variants; count must match), e.g. to replay a saved tuning.
 * Drops recorded graphs. Synchronizes. */
hss_status hss_set_gemm_variants(hss_ctx_t ctx, hss_matrix_t m, int32_t precision, const int32_t* h_variants,
                                 int64_t count);

/* ---- learned rank model -------------------------------------------------- */
/* A multilayer perceptron 7 -> 128 -> 128 -> 128 -> 1 (ReLU between layers)
 * mapping the features of a tree node to y = log2(1 + rank) of the basis the
 * adaptive pivoted QR would keep (Eq. 2 with a tolerance; the paper itself uses
 * a fixed maximum rank). Features, per node, 7 floats: log2 of the point count
 * (clipped at 13), the bounding-box extents sorted in decreasing order divided
 * by the kernel length (3), the gap between the node's box and its sibling's
 * divided by the kernel length, log10 of the kernel length, -log10 of the
 * tolerance. Weights are FP32 on the device; training minimises the pinball
 * loss mean(max(tau (t - y), (tau - 1)(t - y))) with Adam. Feature arrays are
 * row-major n x 7 device memory; targets, outputs and ranks are device vectors
 * of n entries. Packed parameters (hss_rankmlp_param_count floats): W1 (128 x
 * 7), b1, W2 (128 x 128), b2, W3 (128 x 128), b3, W4 (1 x 128), b4, every W
 * column-major (out x in). */
typedef struct {
  int32_t batch;                  /* minibatch size (1..65536) */
  float lr, beta1, beta2, eps;    /* Adam */
  float tau;                      /* pinball quantile in (0, 1) */
} hss_train_opts;
hss_status hss_rankmlp_param_count(int64_t* out);
/* The model's features (7 floats per node, heap order: node k >= 1 at row
 * k - 1) of the cluster tree hss_construct builds on these points with this
 * leaf size; *needed receives the float count (h_out NULL: size query).
 * Synchronizes. */
hss_status hss_rank_features(hss_ctx_t ctx, const double* d_points, int64_t n, int32_t dim, int32_t leaf_size,
                             double length, double tol, float* h_out, int64_t capacity, int64_t* needed);
/* Creates a model with all weights zero (load them with hss_rankmlp_set_weights). */
hss_status hss_rankmlp_create(hss_ctx_t ctx, hss_rankmlp_t* out);
hss_status hss_rankmlp_destroy(hss_rankmlp_t mlp);
/* Copies packed host parameters in and resets the Adam state. Synchronizes. */
hss_status hss_rankmlp_set_weights(hss_ctx_t ctx, hss_rankmlp_t mlp, const float* h_params);
hss_status hss_rankmlp_get_weights(hss_ctx_t ctx, hss_rankmlp_t mlp, float* h_params);
/* d_out[j] = network output y for feature row j. */
hss_status hss_rankmlp_forward(hss_ctx_t ctx, hss_rankmlp_t mlp, const float* d_feats, int64_t n, float* d_out);
/* d_ranks[j] = ceil(2^y - 1 - 1e-3) clipped to [1, cap] (the slack keeps an
 * output equal to a target on its rank despite rounding). */
hss_status hss_rankmlp_predict(hss_ctx_t ctx, hss_rankmlp_t mlp, const float* d_feats, int64_t n, int32_t cap,
                               int32_t* d_ranks);
/* Gradient of the mean pinball loss over the n rows (n <= 65536) with respect
 * to the packed parameters (h_grads, nullable) and the loss (h_loss, nullable).
 * Synchronizes. */
hss_status hss_rankmlp_grad(hss_ctx_t ctx, hss_rankmlp_t mlp, const float* d_feats, const float* d_targets, int64_t n,
                            float tau, float* h_grads, float* h_loss);
/* Minibatch Adam: the consecutive `batch`-sized chunks of d_order (indices into
 * the n rows, each checked to lie in [0, n)) are the minibatches, a short tail
 * being a smaller one; one Adam step per minibatch, with the bias-corrected
 * moments of the published algorithm. h_losses (nullable) receives each
 * step's loss before its update (ceil(order_len / batch) floats). Synchronizes. */
hss_status hss_rankmlp_train(hss_ctx_t ctx, hss_rankmlp_t mlp, const float* d_feats, const float* d_targets,
                             int64_t n, const int64_t* d_order, int64_t order_len, const hss_train_opts* opts,
                             float* h_losses);

hss_status hss_matrix_destroy(hss_matrix_t m);

const char* hss_status_string(hss_status s);
const char* hss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HSS_H_ */
