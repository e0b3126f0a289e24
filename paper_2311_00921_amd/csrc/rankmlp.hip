// Learned rank model: a multilayer perceptron 7 -> 128 -> 128 -> 128 -> 1 with
// ReLU activations that maps the features of a tree node (point count, box
// extents, sibling gap, kernel length, tolerance) to log2(1 + rank) of the basis
// the adaptive pivoted QR (Eq. 2 with a tolerance) would keep. FP32 weights
// (the master copy) on the device; forward, backward (pinball loss) and Adam
// run in hand-written kernels, the layer products on the matrix cores through
// the batched GEMM.
//
// Activations are stored feature-major: H_l is (width x B) column-major, one
// column per sample. Packed parameter order: W1 (128 x 7), b1, W2 (128 x 128),
// b2, W3 (128 x 128), b3, W4 (1 x 128), b4; each W column-major (out x in).
#include <cmath>
#include <map>

#include "hss_internal.h"

namespace hss {

constexpr int kLayers = 4;
constexpr int kSizes[kLayers + 1] = {7, 128, 128, 128, 1};

static int64_t w_off(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += (int64_t)kSizes[i + 1] * kSizes[i] + kSizes[i + 1];
  return o;
}
static int64_t b_off(int l) { return w_off(l) + (int64_t)kSizes[l + 1] * kSizes[l]; }
static int64_t param_count() { return w_off(kLayers); }

}  // namespace hss

struct hss_rankmlp_s {
  hss_ctx_t ctx = nullptr;
  float* P = nullptr;   // parameters
  float* G = nullptr;   // gradients
  float* M1 = nullptr;  // Adam first moment
  float* M2 = nullptr;  // Adam second moment
  int64_t adam_t = 0;
  // workspaces for a batch of up to cap_b samples
  int64_t cap_b = 0;
  float* H[hss::kLayers + 1] = {nullptr};  // activations (H[0] = inputs, H[4] = output)
  float* D[hss::kLayers + 1] = {nullptr};  // gradients with respect to the pre-activations / activations
  float* tgt = nullptr;
  float* loss_part = nullptr;
  // GEMM descriptor sets per batch size
  struct Plan {
    hss::GemmBatch fwd[hss::kLayers], dw[hss::kLayers], dh[hss::kLayers];
  };
  std::map<int64_t, Plan> plans;
};

namespace hss {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// H0[:, j] = feats[order[first + j], :], t[j] = targets[order[first + j]] (order NULL: identity)
__global__ void k_mlp_gather(const float* __restrict__ feats, const float* __restrict__ targets,
                             const int64_t* __restrict__ order, int64_t first, int64_t B, float* __restrict__ H0,
                             float* __restrict__ t) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < B * 7; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / 7;
    const int f = (int)(e % 7);
    const int64_t src = order ? order[first + j] : first + j;
    H0[f + 7 * j] = feats[src * 7 + f];
    if (f == 0 && targets) t[j] = targets[src];
  }
}

// H = max(Z + b, 0) in place (relu) or Z + b (last layer)
__global__ void k_mlp_bias_act(float* __restrict__ Z, const float* __restrict__ b, int rows, int64_t B, int relu) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * B; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows);
    const float v = Z[e] + b[i];
    Z[e] = relu ? fmaxf(v, 0.0f) : v;
  }
}

// dL/dy of the mean pinball loss and per-block partial loss sums
__global__ void k_mlp_pinball(const float* __restrict__ y, const float* __restrict__ t, int64_t B, float tau,
                              float* __restrict__ g, float* __restrict__ part) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < B; j += (int64_t)gridDim.x * blockDim.x) {
    const float d = t[j] - y[j];
    acc += fmaxf(tau * d, (tau - 1.0f) * d);
    g[j] = (t[j] > y[j] ? -tau : 1.0f - tau) / (float)B;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// db[i] = sum_j G[i, j]  (one block per row)
__global__ void k_mlp_rowsum(const float* __restrict__ Gm, int rows, int64_t B, float* __restrict__ db) {
  __shared__ float red[256];
  const int i = blockIdx.x;
  float acc = 0.0f;
  for (int64_t j = threadIdx.x; j < B; j += blockDim.x) acc += Gm[i + (int64_t)rows * j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[i] = red[0];
}

// G = dH * (H > 0) in place on dH (the ReLU derivative, from the stored activation)
__global__ void k_mlp_relu_back(float* __restrict__ dH, const float* __restrict__ H, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    if (!(H[e] > 0.0f)) dH[e] = 0.0f;
}

// Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m/c1) / (sqrt(v/c2) + eps)
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

// rank = ceil(2^y - 1 - 1e-3) clipped to [1, cap]: the slack keeps an output that
// equals a target (log2(1 + rank)) on that rank despite rounding
__global__ void k_mlp_rank(const float* __restrict__ y, int64_t n, int cap, int32_t* __restrict__ r) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    float v = ceilf(exp2f(y[j]) - 1.0f - 1e-3f);
    v = fminf(fmaxf(v, 1.0f), (float)cap);
    r[j] = (int32_t)v;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

static void ensure_batch(hss_rankmlp_t r, int64_t B) {
  if (r->cap_b >= B) return;
  for (int l = 0; l <= kLayers; ++l) {
    dev_free(r->H[l]);
    dev_free(r->D[l]);
    r->H[l] = (float*)dev_alloc(sizeof(float) * kSizes[l] * B);
    r->D[l] = (float*)dev_alloc(sizeof(float) * kSizes[l] * B);
  }
  dev_free(r->tgt);
  dev_free(r->loss_part);
  r->tgt = (float*)dev_alloc(sizeof(float) * B);
  r->loss_part = (float*)dev_alloc(sizeof(float) * 4096);
  for (auto& kv : r->plans)
    for (int l = 0; l < kLayers; ++l) {
      gemm_free(kv.second.fwd[l]);
      gemm_free(kv.second.dw[l]);
      gemm_free(kv.second.dh[l]);
    }
  r->plans.clear();
  r->cap_b = B;
}

static hss_rankmlp_s::Plan& plan_for(hss_rankmlp_t r, int64_t B) {
  auto it = r->plans.find(B);
  if (it != r->plans.end()) return it->second;
  hipStream_t s = r->ctx->stream;
  hss_rankmlp_s::Plan& p = r->plans[B];
  const int b = (int)B;
  for (int l = 0; l < kLayers; ++l) {
    const int in = kSizes[l], out = kSizes[l + 1];
    float* W = r->P + w_off(l);
    float* dW = r->G + w_off(l);
    // Z_{l+1} = W_l H_l  (out x B)
    p.fwd[l].host = {{W, r->H[l], nullptr, r->H[l + 1], out, b, in, out, in, 0, out, 0, 0, nullptr}};
    // dW_l = G_{l+1} H_l^T  (out x in)
    p.dw[l].host = {{r->D[l + 1], r->H[l], nullptr, dW, out, in, b, out, in, 0, out, 0, 0, nullptr}};
    // dH_l = W_l^T G_{l+1}  (in x B)
    p.dh[l].host = {{W, r->D[l + 1], nullptr, r->D[l], in, b, out, out, out, 0, in, 0, 0, nullptr}};
    gemm_upload(p.fwd[l], s);
    gemm_upload(p.dw[l], s);
    gemm_upload(p.dh[l], s);
  }
  return p;
}

// forward of a batch already gathered into H[0]
static void mlp_forward(hss_rankmlp_t r, hss_rankmlp_s::Plan& p, int64_t B) {
  hipStream_t s = r->ctx->stream;
  for (int l = 0; l < kLayers; ++l) {
    gemm_launch_f32(p.fwd[l], false, false, 1.0f, 0.0f, s);
    const int out = kSizes[l + 1];
    hipLaunchKernelGGL(k_mlp_bias_act, dim3(grid_for(out * B)), dim3(256), 0, s, r->H[l + 1],
                       (const float*)(r->P + b_off(l)), out, B, l < kLayers - 1 ? 1 : 0);
    HSS_HIP(hipGetLastError());
  }
}

// loss partial sums and all gradients of the mean pinball loss of a gathered batch
static int mlp_backward(hss_rankmlp_t r, hss_rankmlp_s::Plan& p, int64_t B, float tau) {
  hipStream_t s = r->ctx->stream;
  const int nb = (int)std::min<int64_t>((B + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mlp_pinball, dim3(nb), dim3(256), 0, s, (const float*)r->H[kLayers], (const float*)r->tgt, B,
                     tau, r->D[kLayers], r->loss_part);
  HSS_HIP(hipGetLastError());
  for (int l = kLayers - 1; l >= 0; --l) {
    const int out = kSizes[l + 1];
    gemm_launch_f32(p.dw[l], false, true, 1.0f, 0.0f, s);
    hipLaunchKernelGGL(k_mlp_rowsum, dim3(out), dim3(256), 0, s, (const float*)r->D[l + 1], out, B,
                       r->G + b_off(l));
    HSS_HIP(hipGetLastError());
    if (l > 0) {
      gemm_launch_f32(p.dh[l], true, false, 1.0f, 0.0f, s);
      hipLaunchKernelGGL(k_mlp_relu_back, dim3(grid_for(kSizes[l] * B)), dim3(256), 0, s, r->D[l],
                         (const float*)r->H[l], (int64_t)kSizes[l] * B);
      HSS_HIP(hipGetLastError());
    }
  }
  return nb;
}

static float read_loss(hss_rankmlp_t r, int nb) {
  std::vector<float> h(nb);
  HSS_HIP(hipMemcpyAsync(h.data(), r->loss_part, sizeof(float) * nb, hipMemcpyDeviceToHost, r->ctx->stream));
  HSS_HIP(hipStreamSynchronize(r->ctx->stream));
  double acc = 0.0;
  for (float v : h) acc += v;
  return (float)acc;
}

static void gather(hss_rankmlp_t r, const float* feats, const float* targets, const int64_t* order, int64_t first,
                   int64_t B) {
  hipLaunchKernelGGL(k_mlp_gather, dim3(grid_for(B * 7)), dim3(256), 0, r->ctx->stream, feats, targets, order, first,
                     B, r->H[0], r->tgt);
  HSS_HIP(hipGetLastError());
}

// Predicted ranks of n feature rows (device in, device out); used by the construction.
void rankmlp_predict(hss_rankmlp_t r, const float* d_feats, int64_t n, int cap, int32_t* d_ranks) {
  const int64_t chunk = 65536;
  ensure_batch(r, std::min<int64_t>(n, chunk));
  for (int64_t f0 = 0; f0 < n; f0 += chunk) {
    const int64_t B = std::min<int64_t>(chunk, n - f0);
    auto& p = plan_for(r, B);
    gather(r, d_feats, nullptr, nullptr, f0, B);
    mlp_forward(r, p, B);
    hipLaunchKernelGGL(k_mlp_rank, dim3(grid_for(B)), dim3(256), 0, r->ctx->stream, (const float*)r->H[kLayers], B,
                       cap, d_ranks + f0);
    HSS_HIP(hipGetLastError());
  }
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

hss_status hss_rankmlp_param_count(int64_t* out) {
  HSS_API_BEGIN
  HSS_CHECK(out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = param_count();
  HSS_API_END
}

hss_status hss_rankmlp_create(hss_ctx_t ctx, hss_rankmlp_t* out) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_HIP(hipSetDevice(ctx->device));
  hss_rankmlp_t r = new hss_rankmlp_s();
  r->ctx = ctx;
  const int64_t np = param_count();
  try {
    r->P = (float*)dev_alloc(sizeof(float) * np);
    r->G = (float*)dev_alloc(sizeof(float) * np);
    r->M1 = (float*)dev_alloc(sizeof(float) * np);
    r->M2 = (float*)dev_alloc(sizeof(float) * np);
    std::vector<float> z(np, 0.0f);
    HSS_HIP(hipMemcpyAsync(r->P, z.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
    HSS_HIP(hipMemcpyAsync(r->M1, z.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
    HSS_HIP(hipMemcpyAsync(r->M2, z.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
    HSS_HIP(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    hss_rankmlp_destroy(r);
    throw;
  }
  *out = r;
  HSS_API_END
}

hss_status hss_rankmlp_destroy(hss_rankmlp_t r) {
  HSS_API_BEGIN
  if (!r) return HSS_OK;
  if (r->ctx) (void)hipStreamSynchronize(r->ctx->stream);
  for (auto& kv : r->plans)
    for (int l = 0; l < kLayers; ++l) {
      gemm_free(kv.second.fwd[l]);
      gemm_free(kv.second.dw[l]);
      gemm_free(kv.second.dh[l]);
    }
  for (int l = 0; l <= kLayers; ++l) {
    dev_free(r->H[l]);
    dev_free(r->D[l]);
  }
  dev_free(r->tgt);
  dev_free(r->loss_part);
  dev_free(r->P);
  dev_free(r->G);
  dev_free(r->M1);
  dev_free(r->M2);
  delete r;
  HSS_API_END
}

hss_status hss_rankmlp_set_weights(hss_ctx_t ctx, hss_rankmlp_t r, const float* h_params) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && h_params, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  const int64_t np = param_count();
  std::vector<float> z(np, 0.0f);
  HSS_HIP(hipMemcpyAsync(r->P, h_params, sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
  HSS_HIP(hipMemcpyAsync(r->M1, z.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
  HSS_HIP(hipMemcpyAsync(r->M2, z.data(), sizeof(float) * np, hipMemcpyHostToDevice, ctx->stream));
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  r->adam_t = 0;
  HSS_API_END
}

hss_status hss_rankmlp_get_weights(hss_ctx_t ctx, hss_rankmlp_t r, float* h_params) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && h_params, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_HIP(hipMemcpyAsync(h_params, r->P, sizeof(float) * param_count(), hipMemcpyDeviceToHost, ctx->stream));
  HSS_HIP(hipStreamSynchronize(ctx->stream));
  HSS_API_END
}

hss_status hss_rankmlp_forward(hss_ctx_t ctx, hss_rankmlp_t r, const float* d_feats, int64_t n, float* d_out) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && d_feats && d_out, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(n >= 1, HSS_ERR_INVALID_ARGUMENT, "n must be >= 1");
  const int64_t chunk = 65536;
  ensure_batch(r, std::min<int64_t>(n, chunk));
  for (int64_t f0 = 0; f0 < n; f0 += chunk) {
    const int64_t B = std::min<int64_t>(chunk, n - f0);
    auto& p = plan_for(r, B);
    gather(r, d_feats, nullptr, nullptr, f0, B);
    mlp_forward(r, p, B);
    HSS_HIP(hipMemcpyAsync(d_out + f0, r->H[kLayers], sizeof(float) * B, hipMemcpyDeviceToDevice, ctx->stream));
  }
  HSS_API_END
}

hss_status hss_rankmlp_predict(hss_ctx_t ctx, hss_rankmlp_t r, const float* d_feats, int64_t n, int32_t cap,
                               int32_t* d_ranks) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && d_feats && d_ranks, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(n >= 1 && cap >= 1, HSS_ERR_INVALID_ARGUMENT, "need n >= 1 and cap >= 1");
  rankmlp_predict(r, d_feats, n, cap, d_ranks);
  HSS_API_END
}

hss_status hss_rankmlp_grad(hss_ctx_t ctx, hss_rankmlp_t r, const float* d_feats, const float* d_targets, int64_t n,
                            float tau, float* h_grads, float* h_loss) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && d_feats && d_targets, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(n >= 1 && n <= 65536, HSS_ERR_INVALID_ARGUMENT, "n must be in [1, 65536]");
  HSS_CHECK(tau > 0.0f && tau < 1.0f, HSS_ERR_INVALID_ARGUMENT, "tau must be in (0, 1)");
  ensure_batch(r, n);
  auto& p = plan_for(r, n);
  gather(r, d_feats, d_targets, nullptr, 0, n);
  mlp_forward(r, p, n);
  const int nb = mlp_backward(r, p, n, tau);
  const float loss = read_loss(r, nb) / (float)n;
  if (h_loss) *h_loss = loss;
  if (h_grads) {
    HSS_HIP(hipMemcpyAsync(h_grads, r->G, sizeof(float) * param_count(), hipMemcpyDeviceToHost, ctx->stream));
    HSS_HIP(hipStreamSynchronize(ctx->stream));
  }
  HSS_API_END
}

hss_status hss_rankmlp_train(hss_ctx_t ctx, hss_rankmlp_t r, const float* d_feats, const float* d_targets, int64_t n,
                             const int64_t* d_order, int64_t order_len, const hss_train_opts* o, float* h_losses) {
  HSS_API_BEGIN
  hss::CtxScope cs_(ctx);
  HSS_CHECK(ctx && r && d_feats && d_targets && d_order && o, HSS_ERR_INVALID_ARGUMENT, "NULL argument");
  HSS_CHECK(n >= 1 && order_len >= 1, HSS_ERR_INVALID_ARGUMENT, "need n >= 1 and order_len >= 1");
  HSS_CHECK(o->batch >= 1 && o->batch <= 65536, HSS_ERR_INVALID_ARGUMENT, "batch must be in [1, 65536]");
  HSS_CHECK(o->tau > 0.0f && o->tau < 1.0f, HSS_ERR_INVALID_ARGUMENT, "tau must be in (0, 1)");
  HSS_CHECK(o->lr > 0.0f && o->beta1 >= 0.0f && o->beta1 < 1.0f && o->beta2 >= 0.0f && o->beta2 < 1.0f &&
                o->eps > 0.0f,
            HSS_ERR_INVALID_ARGUMENT, "bad Adam parameters");
  hipStream_t s = ctx->stream;
  {
    // the gather kernel indexes the features with these values: check them here
    std::vector<int64_t> ord(order_len);
    HSS_HIP(hipMemcpyAsync(ord.data(), d_order, sizeof(int64_t) * order_len, hipMemcpyDeviceToHost, s));
    HSS_HIP(hipStreamSynchronize(s));
    for (int64_t v : ord) HSS_CHECK(v >= 0 && v < n, HSS_ERR_INVALID_ARGUMENT, "order entry out of range");
  }
  ensure_batch(r, std::min<int64_t>(o->batch, order_len));
  const int64_t np = param_count();
  int64_t step = 0;
  std::vector<float> parts;
  for (int64_t s0 = 0; s0 < order_len; s0 += o->batch, ++step) {
    const int64_t B = std::min<int64_t>(o->batch, order_len - s0);
    auto& p = plan_for(r, B);
    gather(r, d_feats, d_targets, d_order, s0, B);
    mlp_forward(r, p, B);
    const int nb = mlp_backward(r, p, B, o->tau);
    if (h_losses) h_losses[step] = read_loss(r, nb) / (float)B;
    r->adam_t += 1;
    const float c1 = 1.0f - std::pow(o->beta1, (float)r->adam_t);
    const float c2 = 1.0f - std::pow(o->beta2, (float)r->adam_t);
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(np)), dim3(256), 0, s, r->P, (const float*)r->G, r->M1, r->M2, np,
                       o->lr, o->beta1, o->beta2, o->eps, c1, c2);
    HSS_HIP(hipGetLastError());
  }
  HSS_HIP(hipStreamSynchronize(s));
  HSS_API_END
}

}  // extern "C"
