// ULV solve that allocates nothing, for callers that cannot call hipMalloc
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// it): the solve's per-node vector workspace comes from a static device array
// instead of the matrix's own workspace, which the ordinary solve allocates on
// first use and grows with the number of right-hand sides.
#include <mutex>

#include "hss_internal.h"

namespace hss {

// Per-node vector workspace of the solve: sum over nodes of the node's block
// size, times the number of right-hand sides, in doubles. 2^22 doubles (32 MiB)
// per GPU, held until the process ends: N = 262144, leaf 256, rank 96 has a
// node-size sum of 458 560, so nine right-hand sides fit.
constexpr int64_t kScratchDoubles = int64_t(1) << 22;

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

// Called by hss_ctx_create with `device` current: the device address of this
// GPU's copy of the array (host code never passes the array's name itself).
void noalloc_init(int device) {
  HSS_CHECK(device >= 0 && device < kMaxDevices, HSS_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  HSS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  HSS_CHECK(p != nullptr, HSS_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[device] = (double*)p;
}

static double* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace hss

using namespace hss;

extern "C" hss_status hss_ulv_solve_noalloc(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                                            int64_t nrhs, int64_t ld) {
  try {
    HSS_CHECK(ctx && m && d_b && d_x, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
    HSS_CHECK(nrhs >= 1 && ld >= m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld >= n");
    HSS_CHECK(m->state == 1, HSS_ERR_BAD_STATE, "matrix is not factored");
    HSS_CHECK(m->ctx == ctx, HSS_ERR_INVALID_ARGUMENT, "matrix belongs to another context");
    HSS_CHECK(m->sum_n > 0 && nrhs <= kScratchDoubles / m->sum_n, HSS_ERR_UNSUPPORTED,
              "hss_ulv_solve_noalloc: the workspace needs " + std::to_string(m->sum_n) + " x " +
                  std::to_string(nrhs) + " doubles, above the static scratch of " +
                  std::to_string(kScratchDoubles) + " (at most " + std::to_string(kScratchDoubles / m->sum_n) +
                  " right-hand sides for this matrix)");
    double* ws = scratch_ptr(ctx->device);
    HSS_CHECK(ws != nullptr, HSS_ERR_BAD_STATE, "the scratch array of this device was not resolved");
    // per-launch profiling would create events: it is bypassed for this call
    const bool prof = ctx->prof;
    ctx->prof = false;
    try {
      solve_fp64_ws(m, d_b, d_x, nrhs, ld, ws);
    } catch (...) {
      ctx->prof = prof;
      throw;
    }
    ctx->prof = prof;
    return HSS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.st;
  } catch (...) {
    set_error("unexpected internal exception");
    return HSS_ERR_DEVICE;
  }
}
