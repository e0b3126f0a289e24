// Iterative refinement of the mixed-precision solve: the residual is computed
// with the FP64 HSS matvec, the correction with the (FP32) ULV solve. When the
// residual stops dropping by at least a factor 2 per correction, the iteration
// switches to preconditioned conjugate gradients on the FP64 HSS matrix with the
// same ULV solve as the (SPD) preconditioner.
#include <cmath>

#include "hss_internal.h"

namespace hss {

// out[c] = sum_i a[i, c] * b[i, c]  (per-column dot products, two-stage)
__global__ __launch_bounds__(256) void k_coldot_part(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, int64_t ld, double* __restrict__ part) {
  const int c = blockIdx.y;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += a[i + c * ld] * b[i + c * ld];
  __shared__ double s[256];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c * gridDim.x + blockIdx.x] = s[0];
}

__global__ void k_coldot_final(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  const int c = blockIdx.x;
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += part[c * nparts + i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = s[0];
}

// y[:, c] = alpha[c] * x[:, c] + beta[c] * y[:, c]  (coefficients on the device)
__global__ void k_axpby_cols(const double* __restrict__ x, double* __restrict__ y, int64_t n, int64_t ldx,
                             int64_t ldy, const double* __restrict__ alpha, const double* __restrict__ beta) {
  const int c = blockIdx.y;
  const double a = alpha[c], bb = beta[c];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i + c * ldy] = a * x[i + c * ldx] + bb * y[i + c * ldy];
}

struct RefineWS {
  double *r, *z, *p, *q, *part, *coef, *dots;
  int64_t ld;
};

static constexpr int kParts = 128;

static void coldot(const double* a, const double* b, int64_t n, int64_t ld, int64_t nrhs, RefineWS& w,
                   double* out_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot_part, dim3(kParts, nrhs), dim3(256), 0, s, a, b, n, ld, w.part);
  HSS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_coldot_final, dim3(nrhs), dim3(256), 0, s, (const double*)w.part, kParts, out_dev);
  HSS_HIP(hipGetLastError());
}

static void axpby(const double* x, double* y, int64_t n, int64_t ldx, int64_t ldy, int64_t nrhs,
                  const std::vector<double>& alpha, const std::vector<double>& beta, RefineWS& w, hipStream_t s) {
  std::vector<double> ab(2 * nrhs);
  for (int64_t c = 0; c < nrhs; ++c) {
    ab[c] = alpha[c];
    ab[nrhs + c] = beta[c];
  }
  HSS_HIP(hipMemcpyAsync(w.coef, ab.data(), sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_axpby_cols, dim3(256, nrhs), dim3(256), 0, s, x, y, n, ldx, ldy, (const double*)w.coef,
                     (const double*)(w.coef + nrhs));
  HSS_HIP(hipGetLastError());
}

static std::vector<double> read_dev(const double* d, int64_t k, hipStream_t s) {
  std::vector<double> h(k);
  HSS_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HSS_HIP(hipStreamSynchronize(s));
  return h;
}

static void lp_solve(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld) {
  solve_run(m, b, x, nrhs, ld);
}

// returns (iterations, worst relative residual, converged)
void refine(hss_matrix_t m, const double* b, double* x, int64_t nrhs, int64_t ld, double tol, int max_iters,
            int* iters_out, double* relres_out, bool* converged) {
  hipStream_t s = m->ctx->stream;
  const int64_t n = m->n;
  const int64_t need = 4 * n * nrhs + (int64_t)kParts * nrhs + 4 * nrhs + 8;
  if (m->tmp_len < need) {
    if (m->dtmp) dev_free(m->dtmp);
    m->dtmp = (double*)dev_alloc(sizeof(double) * need);
    m->tmp_len = need;
  }
  RefineWS w;
  w.ld = n;
  w.r = m->dtmp;
  w.z = w.r + n * nrhs;
  w.p = w.z + n * nrhs;
  w.q = w.p + n * nrhs;
  w.part = w.q + n * nrhs;
  w.coef = w.part + (int64_t)kParts * nrhs;
  w.dots = w.coef + 2 * nrhs;
  const std::vector<double> one(nrhs, 1.0), minus(nrhs, -1.0), zero(nrhs, 0.0);
  // ||b|| per column (b has leading dimension ld; copy into r first)
  HSS_HIP(hipMemcpy2DAsync(w.r, sizeof(double) * n, b, sizeof(double) * ld, sizeof(double) * n, nrhs,
                           hipMemcpyDeviceToDevice, s));
  coldot(w.r, w.r, n, n, nrhs, w, w.dots, s);
  std::vector<double> bn = read_dev(w.dots, nrhs, s);
  for (auto& v : bn) v = std::sqrt(v) > 0 ? std::sqrt(v) : 1.0;
  lp_solve(m, b, x, nrhs, ld);
  auto residual = [&](std::vector<double>& rel) {
    // r = b - A x
    matvec_fp64(m, x, w.q, nrhs, ld == n ? n : ld);
    HSS_HIP(hipMemcpy2DAsync(w.r, sizeof(double) * n, b, sizeof(double) * ld, sizeof(double) * n, nrhs,
                             hipMemcpyDeviceToDevice, s));
    axpby(w.q, w.r, n, ld == n ? n : ld, n, nrhs, minus, one, w, s);
    coldot(w.r, w.r, n, n, nrhs, w, w.dots, s);
    std::vector<double> rr = read_dev(w.dots, nrhs, s);
    double worst = 0.0;
    rel.resize(nrhs);
    for (int64_t c = 0; c < nrhs; ++c) {
      rel[c] = std::sqrt(rr[c]) / bn[c];
      worst = std::max(worst, rel[c]);
    }
    return worst;
  };
  HSS_CHECK(ld == n, HSS_ERR_UNSUPPORTED, "refinement needs ld == n");
  std::vector<double> rel;
  double worst = residual(rel), prev = 1e300;
  int it = 0;
  bool use_cg = false;
  while (worst > tol && it < max_iters) {
    if (worst > 0.5 * prev) {
      use_cg = true;
      break;
    }
    prev = worst;
    // x += solve(r)
    lp_solve(m, w.r, w.z, nrhs, n);
    axpby(w.z, x, n, n, ld, nrhs, one, one, w, s);
    ++it;
    worst = residual(rel);
  }
  if (use_cg && worst > tol) {
    // PCG from the current x: r = b - A x already in w.r
    lp_solve(m, w.r, w.z, nrhs, n);
    HSS_HIP(hipMemcpyAsync(w.p, w.z, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, s));
    coldot(w.r, w.z, n, n, nrhs, w, w.dots, s);
    std::vector<double> rz = read_dev(w.dots, nrhs, s);
    while (worst > tol && it < max_iters) {
      matvec_fp64(m, w.p, w.q, nrhs, n);
      coldot(w.p, w.q, n, n, nrhs, w, w.dots, s);
      std::vector<double> pq = read_dev(w.dots, nrhs, s);
      std::vector<double> alpha(nrhs), malpha(nrhs);
      for (int64_t c = 0; c < nrhs; ++c) {
        alpha[c] = (pq[c] != 0.0 && rel[c] > tol) ? rz[c] / pq[c] : 0.0;
        malpha[c] = -alpha[c];
      }
      axpby(w.p, x, n, n, ld, nrhs, alpha, one, w, s);
      axpby(w.q, w.r, n, n, n, nrhs, malpha, one, w, s);
      ++it;
      coldot(w.r, w.r, n, n, nrhs, w, w.dots, s);
      std::vector<double> rr = read_dev(w.dots, nrhs, s);
      worst = 0.0;
      for (int64_t c = 0; c < nrhs; ++c) {
        rel[c] = std::sqrt(rr[c]) / bn[c];
        worst = std::max(worst, rel[c]);
      }
      if (worst <= tol) break;
      lp_solve(m, w.r, w.z, nrhs, n);
      coldot(w.r, w.z, n, n, nrhs, w, w.dots, s);
      std::vector<double> rz2 = read_dev(w.dots, nrhs, s);
      std::vector<double> beta(nrhs);
      for (int64_t c = 0; c < nrhs; ++c) beta[c] = rz[c] != 0.0 ? rz2[c] / rz[c] : 0.0;
      rz = rz2;
      axpby(w.z, w.p, n, n, n, nrhs, one, beta, w, s);
    }
    // recompute the true residual (the recurrence drifts)
    worst = residual(rel);
  }
  *iters_out = it;
  *relres_out = worst;
  *converged = worst <= tol;
}

}  // namespace hss

using namespace hss;

extern "C" hss_status hss_ulv_solve_refined(hss_ctx_t ctx, hss_matrix_t m, const double* d_b, double* d_x,
                                            int64_t nrhs, int64_t ld, double tol, int32_t max_iters,
                                            int32_t* iters_out, double* relres_out) {
  try {
    hss::CtxScope cs_(ctx);
    HSS_CHECK(ctx && m && d_b && d_x, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
    HSS_CHECK(nrhs >= 1 && ld == m->n, HSS_ERR_INVALID_ARGUMENT, "need nrhs >= 1 and ld == n");
    HSS_CHECK(d_b != d_x, HSS_ERR_INVALID_ARGUMENT, "b and x must not alias");
    HSS_CHECK(tol > 0.0 && max_iters >= 0, HSS_ERR_INVALID_ARGUMENT, "need tol > 0 and max_iters >= 0");
    HSS_CHECK(m->state == 1, HSS_ERR_BAD_STATE, "matrix is not factored");
    int it = 0;
    double rr = 0.0;
    bool ok = false;
    refine(m, d_b, d_x, nrhs, ld, tol, max_iters, &it, &rr, &ok);
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rr;
    if (!ok) {
      set_error("refinement stopped at relative residual " + std::to_string(rr) + " after " + std::to_string(it) +
                " corrections");
      return HSS_ERR_NOT_CONVERGED;
    }
    return HSS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.st;
  } catch (...) {
    set_error("unexpected internal exception");
    return HSS_ERR_DEVICE;
  }
}
