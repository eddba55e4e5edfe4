// unet.cpp -- the learned surrogate of libdd: a 4-level U-Net (32, 64, 128,
// 256 channels at 64^2, 32^2, 16^2, 8^2) mapping a scan's first-arrival-time
// map plus kappa = D dwell / pitch^2 and sigma / pitch to the logarithm of the
// dimensionless damage map at the end of the scan, trained and run with the
// BF16 MFMA kernels of unet_kernels.hip.  Predictions are judged by the exact
// kernels (one exact row per map) and replaced by the exact map when the
// judge rejects them or the scan lies outside the training range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../../include/dd.h"
#include "dd_runtime.h"
#include "unet_kernels.h"

using namespace dd;

namespace {

constexpr int S = 64;  // input side

struct Conv {
  int H, ci, co;
  int64_t w_off, b_off;  // weights [9 ci][co], bias [co] in the flat parameter vector
  DevBuf col, Z, A;      // im2col (BF16), pre-activation, activation (FP32)
};

#define UN_HIP(call, what)                               \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, what);     \
  } while (0)

}  // namespace

struct dd_unet {
  std::vector<Conv> L;
  int64_t head_w = 0, n_params = 0;
  DevBuf w, wb, g, m, v;  // master FP32, BF16 copy, gradient, Adam moments
  int64_t step = 0;
  int capB = 0, B = 0;     // allocated batch capacity, batch of the last forward
  DevBuf p1, p2, p3, c3, c2, c1, y;
  DevBuf dA0, dA1, dZ, dZb, dcol, ds1, ds2, ds3, part, mse_part;
  size_t part_elems = 0;
};

namespace {

// 14 convolutions; indices follow the forward order.
void build_layers(dd_unet& u) {
  struct Spec {
    int H, ci, co;
  };
  const Spec specs[] = {
      {64, 3, 32},   {64, 32, 32},   {32, 32, 64},   {32, 64, 64},  {16, 64, 128},
      {16, 128, 128}, {8, 128, 256},  {8, 256, 256},  {16, 384, 128}, {16, 128, 128},
      {32, 192, 64},  {32, 64, 64},   {64, 96, 32},   {64, 32, 32}};
  int64_t off = 0;
  for (const Spec& s : specs) {
    Conv c;
    c.H = s.H;
    c.ci = s.ci;
    c.co = s.co;
    c.w_off = off;
    off += 9LL * s.ci * s.co;
    c.b_off = off;
    off += s.co;
    u.L.push_back(std::move(c));
  }
  u.head_w = off;  // 32 weights then 1 bias
  off += 33;
  u.n_params = off;
}

int64_t M_of(const dd_unet& u, const Conv& c) { return (int64_t)u.B * c.H * c.H; }

int wgrad_splits(const Conv& c, int64_t M) {
  const int tiles = ((9 * c.ci + 63) / 64) * ((c.co + 63) / 64);
  int64_t s = std::max<int64_t>(1, std::min<int64_t>(M / 256, 2048 / std::max(tiles, 1)));
  return (int)std::min<int64_t>(s, 512);
}

dd_status ensure_capacity(dd_unet& u, int B) {
  if (B <= u.capB) return DD_OK;
  const int64_t M64 = (int64_t)B * 4096, M32 = (int64_t)B * 1024, M16 = (int64_t)B * 256,
                M8 = (int64_t)B * 64;
  size_t max_mco = 0, max_mci = 0, max_col = 0, max_part = 0;
  for (Conv& c : u.L) {
    const int64_t M = (int64_t)B * c.H * c.H;
    UN_HIP(c.col.ensure(sizeof(__bf16) * M * 9 * c.ci), "device allocation");
    UN_HIP(c.Z.ensure(sizeof(float) * M * c.co), "device allocation");
    UN_HIP(c.A.ensure(sizeof(float) * M * c.co), "device allocation");
    max_mco = std::max(max_mco, (size_t)(M * c.co));
    max_mci = std::max(max_mci, (size_t)(M * c.ci));
    max_col = std::max(max_col, (size_t)(M * 9 * c.ci));
    const int sp = nn::gemm_splits(9 * c.ci, (int)M, wgrad_splits(c, M));
    max_part = std::max(max_part, (size_t)sp * 9 * c.ci * c.co);
  }
  UN_HIP(u.p1.ensure(sizeof(float) * M32 * 32), "device allocation");
  UN_HIP(u.p2.ensure(sizeof(float) * M16 * 64), "device allocation");
  UN_HIP(u.p3.ensure(sizeof(float) * M8 * 128), "device allocation");
  UN_HIP(u.c3.ensure(sizeof(float) * M16 * 384), "device allocation");
  UN_HIP(u.c2.ensure(sizeof(float) * M32 * 192), "device allocation");
  UN_HIP(u.c1.ensure(sizeof(float) * M64 * 96), "device allocation");
  UN_HIP(u.y.ensure(sizeof(float) * M64), "device allocation");
  const size_t dmax = std::max(max_mco, max_mci);
  UN_HIP(u.dA0.ensure(sizeof(float) * dmax), "device allocation");
  UN_HIP(u.dA1.ensure(sizeof(float) * dmax), "device allocation");
  UN_HIP(u.dZ.ensure(sizeof(float) * max_mco), "device allocation");
  UN_HIP(u.dZb.ensure(sizeof(__bf16) * max_mco), "device allocation");
  UN_HIP(u.dcol.ensure(sizeof(float) * max_col), "device allocation");
  UN_HIP(u.ds1.ensure(sizeof(float) * M64 * 32), "device allocation");
  UN_HIP(u.ds2.ensure(sizeof(float) * M32 * 64), "device allocation");
  UN_HIP(u.ds3.ensure(sizeof(float) * M16 * 128), "device allocation");
  UN_HIP(u.part.ensure(sizeof(float) * max_part), "device allocation");
  UN_HIP(u.mse_part.ensure(sizeof(double) * 1024), "device allocation");
  u.part_elems = max_part;
  u.capB = B;
  return DD_OK;
}

dd_status conv_fwd(dd_unet& u, Conv& c, const float* in, hipStream_t st) {
  const int64_t M = M_of(u, c);
  UN_HIP(nn::im2col(in, u.B, c.H, c.H, c.ci, c.col.as<__bf16>(), st), "im2col");
  UN_HIP(nn::gemm_bias_silu(c.col.as<__bf16>(), 9 * c.ci, u.wb.as<__bf16>() + c.w_off, c.co,
                            c.A.as<float>(), c.Z.as<float>(), c.co, u.w.as<float>() + c.b_off,
                            (int)M, c.co, 9 * c.ci, st),
         "conv GEMM");
  return DD_OK;
}

// dA -> gradients of the layer's weights and bias; dX (input gradient) if
// requested.
dd_status conv_bwd(dd_unet& u, Conv& c, const float* dA, float* dX, hipStream_t st) {
  const int64_t M = M_of(u, c);
  UN_HIP(nn::silu_bwd(dA, c.Z.as<float>(), M * c.co, u.dZ.as<float>(), u.dZb.as<__bf16>(), st),
         "SiLU backward");
  UN_HIP(nn::colsum_add(u.dZ.as<float>(), (int)M, c.co, u.g.as<float>() + c.b_off, st),
         "bias gradient");
  const int want = wgrad_splits(c, M);
  const int sp = nn::gemm_splits(9 * c.ci, (int)M, want);
  UN_HIP(nn::gemm(c.col.as<__bf16>(), 9 * c.ci, true, u.dZb.as<__bf16>(), c.co, false,
                  u.part.as<float>(), c.co, 9 * c.ci, c.co, (int)M, want, st),
         "weight-gradient GEMM");
  UN_HIP(nn::sum_splits(u.part.as<float>(), sp, 9LL * c.ci * c.co, u.g.as<float>() + c.w_off, st),
         "weight-gradient reduction");
  if (dX) {
    UN_HIP(nn::gemm(u.dZb.as<__bf16>(), c.co, false, u.wb.as<__bf16>() + c.w_off, c.co, true,
                    u.dcol.as<float>(), 9 * c.ci, (int)M, 9 * c.ci, c.co, 1, st),
           "data-gradient GEMM");
    UN_HIP(nn::col2im(u.dcol.as<float>(), u.B, c.H, c.H, c.ci, dX, st), "col2im");
  }
  return DD_OK;
}

dd_status forward(dd_unet& u, const float* x, hipStream_t st) {
  auto& L = u.L;
  const int B = u.B;
  dd_status rc;
#define STEP(expr)        \
  if ((rc = (expr)) != DD_OK) return rc
  STEP(conv_fwd(u, L[0], x, st));
  STEP(conv_fwd(u, L[1], L[0].A.as<float>(), st));
  UN_HIP(nn::pool_fwd(L[1].A.as<float>(), B, 64, 64, 32, u.p1.as<float>(), st), "pool");
  STEP(conv_fwd(u, L[2], u.p1.as<float>(), st));
  STEP(conv_fwd(u, L[3], L[2].A.as<float>(), st));
  UN_HIP(nn::pool_fwd(L[3].A.as<float>(), B, 32, 32, 64, u.p2.as<float>(), st), "pool");
  STEP(conv_fwd(u, L[4], u.p2.as<float>(), st));
  STEP(conv_fwd(u, L[5], L[4].A.as<float>(), st));
  UN_HIP(nn::pool_fwd(L[5].A.as<float>(), B, 16, 16, 128, u.p3.as<float>(), st), "pool");
  STEP(conv_fwd(u, L[6], u.p3.as<float>(), st));
  STEP(conv_fwd(u, L[7], L[6].A.as<float>(), st));
  UN_HIP(nn::up_concat(L[7].A.as<float>(), B, 8, 8, 256, L[5].A.as<float>(), 128, u.c3.as<float>(),
                       st),
         "upsample");
  STEP(conv_fwd(u, L[8], u.c3.as<float>(), st));
  STEP(conv_fwd(u, L[9], L[8].A.as<float>(), st));
  UN_HIP(nn::up_concat(L[9].A.as<float>(), B, 16, 16, 128, L[3].A.as<float>(), 64, u.c2.as<float>(),
                       st),
         "upsample");
  STEP(conv_fwd(u, L[10], u.c2.as<float>(), st));
  STEP(conv_fwd(u, L[11], L[10].A.as<float>(), st));
  UN_HIP(nn::up_concat(L[11].A.as<float>(), B, 32, 32, 64, L[1].A.as<float>(), 32, u.c1.as<float>(),
                       st),
         "upsample");
  STEP(conv_fwd(u, L[12], u.c1.as<float>(), st));
  STEP(conv_fwd(u, L[13], L[12].A.as<float>(), st));
  UN_HIP(nn::head_fwd(L[13].A.as<float>(), (int64_t)B * 4096, 32, u.w.as<float>() + u.head_w,
                      u.w.as<float>() + u.head_w + 32, u.y.as<float>(), st),
         "head");
  return DD_OK;
}

dd_status backward(dd_unet& u, const float* dy, hipStream_t st) {
  auto& L = u.L;
  const int B = u.B;
  const int64_t M64 = (int64_t)B * 4096, M32 = (int64_t)B * 1024, M16 = (int64_t)B * 256;
  float* a0 = u.dA0.as<float>();
  float* a1 = u.dA1.as<float>();
  dd_status rc;
  UN_HIP(nn::fill(u.ds1.as<float>(), M64 * 32, 0.f, st), "fill");
  UN_HIP(nn::fill(u.ds2.as<float>(), M32 * 64, 0.f, st), "fill");
  UN_HIP(nn::fill(u.ds3.as<float>(), M16 * 128, 0.f, st), "fill");
  UN_HIP(nn::head_bwd(dy, L[13].A.as<float>(), M64, 32, u.w.as<float>() + u.head_w, a0,
                      u.g.as<float>() + u.head_w, st),
         "head backward");
  STEP(conv_bwd(u, L[13], a0, a1, st));
  STEP(conv_bwd(u, L[12], a1, a0, st));  // a0 = d c1 [64^2][96]
  UN_HIP(nn::up_concat_bwd(a0, B, 32, 32, 64, 32, a1, u.ds1.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[11], a1, a0, st));
  STEP(conv_bwd(u, L[10], a0, a1, st));  // a1 = d c2 [32^2][192]
  UN_HIP(nn::up_concat_bwd(a1, B, 16, 16, 128, 64, a0, u.ds2.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[9], a0, a1, st));
  STEP(conv_bwd(u, L[8], a1, a0, st));  // a0 = d c3 [16^2][384]
  UN_HIP(nn::up_concat_bwd(a0, B, 8, 8, 256, 128, a1, u.ds3.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[7], a1, a0, st));
  STEP(conv_bwd(u, L[6], a0, a1, st));  // a1 = d p3 [8^2][128]
  UN_HIP(nn::pool_bwd_add(a1, B, 16, 16, 128, u.ds3.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[5], u.ds3.as<float>(), a0, st));
  STEP(conv_bwd(u, L[4], a0, a1, st));  // a1 = d p2 [16^2][64]
  UN_HIP(nn::pool_bwd_add(a1, B, 32, 32, 64, u.ds2.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[3], u.ds2.as<float>(), a0, st));
  STEP(conv_bwd(u, L[2], a0, a1, st));  // a1 = d p1 [32^2][32]
  UN_HIP(nn::pool_bwd_add(a1, B, 64, 64, 32, u.ds1.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[1], u.ds1.as<float>(), a0, st));
  STEP(conv_bwd(u, L[0], a0, nullptr, st));
#undef STEP
  return DD_OK;
}

// Surrogate inputs of one scan: channel 0 the first-visit time of each probe
// over the scan duration, channel 1 (log10 kappa + 1) / 3 with kappa = D dwell /
// pitch^2 (dwell per probe position), channel 2 (sigma/pitch - 0.6) / 0.4.
void scan_features(const dd_scan* s, float* x) {
  const int n = s->desc.nx * s->desc.ny;
  std::vector<int64_t> first(n, -1);
  for (int64_t v = 0; v < s->V; ++v)
    if (first[s->ids[v]] < 0) first[s->ids[v]] = v;
  const double kap = s->desc.D_m2s * s->desc.dwell_s / (s->desc.pitch_m * s->desc.pitch_m);
  const float c1 = (float)((std::log10(kap) + 1.0) / 3.0);
  const float c2 = (float)((s->desc.sigma_m / s->desc.pitch_m - 0.6) / 0.4);
  for (int p = 0; p < n; ++p) {
    x[3 * p + 0] = first[p] < 0 ? 1.0f : (float)((double)first[p] / (double)s->V);
    x[3 * p + 1] = c1;
    x[3 * p + 2] = c2;
  }
}

bool in_training_range(const dd_scan* s) {
  const double kap = s->desc.D_m2s * s->desc.dwell_s / (s->desc.pitch_m * s->desc.pitch_m);
  const double sh = s->desc.sigma_m / s->desc.pitch_m;
  return s->desc.nx == S && s->desc.ny == S && kap >= 0.99e-4 && kap <= 101.0 && sh >= 0.199 &&
         sh <= 1.001;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
dd_status dd_unet_create(uint64_t seed, dd_unet** out) {
  if (!out) return fail(DD_EINVAL, "out is NULL");
  *out = nullptr;
  dd_status rc = ensure_device();
  if (rc != DD_OK) return rc;
  dd_unet* u = new (std::nothrow) dd_unet();
  if (!u) return fail(DD_ENOMEM, "out of host memory");
  build_layers(*u);
  // He-normal weights, zero biases; the head starts at zero weight and a
  // bias near the mean log target.
  std::vector<float> w(u->n_params, 0.f);
  std::mt19937_64 gen(seed);
  for (const Conv& c : u->L) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.0f / (9.0f * c.ci)));
    for (int64_t k = 0; k < 9LL * c.ci * c.co; ++k) w[c.w_off + k] = nd(gen);
  }
  {
    std::normal_distribution<float> nd(0.f, std::sqrt(1.0f / 32.0f));
    for (int k = 0; k < 32; ++k) w[u->head_w + k] = nd(gen);
    w[u->head_w + 32] = 0.f;
  }
  hipError_t e = u->w.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->wb.ensure(sizeof(__bf16) * u->n_params);
  if (e == hipSuccess) e = u->g.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->m.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->v.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = hipMemcpy(u->w.p, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = nn::to_bf16(u->w.as<float>(), u->n_params, u->wb.as<__bf16>(), nullptr);
  if (e == hipSuccess) e = nn::fill(u->g.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = nn::fill(u->m.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = nn::fill(u->v.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete u;
    return hip_fail(e, "surrogate allocation");
  }
  *out = u;
  return DD_OK;
}

void dd_unet_destroy(dd_unet* u) {
  if (!u) return;
  for (DevBuf* b : {&u->w, &u->wb, &u->g, &u->m, &u->v, &u->p1, &u->p2, &u->p3, &u->c3, &u->c2,
                    &u->c1, &u->y, &u->dA0, &u->dA1, &u->dZ, &u->dZb, &u->dcol, &u->ds1, &u->ds2,
                    &u->ds3, &u->part, &u->mse_part})
    b->release();
  for (Conv& c : u->L) {
    c.col.release();
    c.Z.release();
    c.A.release();
  }
  delete u;
}

int64_t dd_unet_num_params(const dd_unet* u) { return u ? u->n_params : -1; }

dd_status dd_unet_params(dd_unet* u, float* host_get, const float* host_set) {
  if (!u || (!host_get && !host_set)) return fail(DD_EINVAL, "NULL argument");
  if (host_get)
    UN_HIP(hipMemcpy(host_get, u->w.p, sizeof(float) * u->n_params, hipMemcpyDeviceToHost),
           "parameter copy");
  if (host_set) {
    UN_HIP(hipMemcpy(u->w.p, host_set, sizeof(float) * u->n_params, hipMemcpyHostToDevice),
           "parameter copy");
    UN_HIP(nn::to_bf16(u->w.as<float>(), u->n_params, u->wb.as<__bf16>(), nullptr), "bf16 copy");
    UN_HIP(hipDeviceSynchronize(), "synchronize");
  }
  return DD_OK;
}

dd_status dd_unet_grads(const dd_unet* u, float* host_out) {
  if (!u || !host_out) return fail(DD_EINVAL, "NULL argument");
  UN_HIP(hipMemcpy(host_out, u->g.p, sizeof(float) * u->n_params, hipMemcpyDeviceToHost),
         "gradient copy");
  return DD_OK;
}

dd_status dd_unet_forward(dd_unet* u, int32_t batch, const float* x, float* y, void* stream) {
  if (!u || !x || !y || batch < 1) return fail(DD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  dd_status rc = ensure_capacity(*u, batch);
  if (rc != DD_OK) return rc;
  u->B = batch;
  rc = forward(*u, x, st);
  if (rc != DD_OK) return rc;
  UN_HIP(hipMemcpyAsync(y, u->y.p, sizeof(float) * batch * 4096, hipMemcpyDeviceToDevice, st),
         "output copy");
  return DD_OK;
}

dd_status dd_unet_backward(dd_unet* u, const float* dy, void* stream) {
  if (!u || !dy || u->B < 1) return fail(DD_EINVAL, "backward needs a forward first");
  return backward(*u, dy, (hipStream_t)stream);
}

dd_status dd_unet_mse(dd_unet* u, int64_t n, const float* y, const float* t, float* dy,
                      double* loss_host, void* stream) {
  if (!u || n < 1 || !y || !t || !dy) return fail(DD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  dd_status rc = ensure_capacity(*u, std::max(u->capB, 1));
  if (rc != DD_OK) return rc;
  const int nb = 256;
  UN_HIP(nn::mse(y, t, n, dy, u->mse_part.as<double>(), nb, st), "loss");
  if (loss_host) {
    double part[256];
    UN_HIP(hipMemcpyAsync(part, u->mse_part.p, sizeof part, hipMemcpyDeviceToHost, st), "copy");
    UN_HIP(hipStreamSynchronize(st), "synchronize");
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    *loss_host = s / (double)n;
  }
  return DD_OK;
}

dd_status dd_unet_adam(dd_unet* u, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!u || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(DD_EINVAL, "bad Adam parameters");
  u->step += 1;
  const float bc1 = 1.0f - std::pow(beta1, (float)u->step);
  const float bc2 = 1.0f - std::pow(beta2, (float)u->step);
  UN_HIP(nn::adam(u->w.as<float>(), u->m.as<float>(), u->v.as<float>(), u->g.as<float>(),
                  u->n_params, lr, beta1, beta2, eps, bc1, bc2, u->wb.as<__bf16>(),
                  (hipStream_t)stream),
         "Adam step");
  return DD_OK;
}

dd_status dd_surrogate_inputs(dd_scan* const* scans, int32_t n, float* x, void* stream) {
  if (!scans || n < 1 || !x) return fail(DD_EINVAL, "bad arguments");
  for (int32_t k = 0; k < n; ++k)
    if (!scans[k] || scans[k]->desc.nx != S || scans[k]->desc.ny != S)
      return fail(DD_EINVAL, "surrogate inputs need 64x64 probe grids (scan %d)", k);
  std::vector<float> h((size_t)n * S * S * 3);
  for (int32_t k = 0; k < n; ++k) scan_features(scans[k], h.data() + (size_t)k * S * S * 3);
  hipStream_t st = (hipStream_t)stream;
  UN_HIP(hipMemcpyAsync(x, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st), "copy");
  UN_HIP(hipStreamSynchronize(st), "synchronize");
  return DD_OK;
}

dd_status dd_surrogate_targets(dd_scan* const* scans, int32_t n, const double* psi, float* t,
                               void* stream) {
  if (!scans || n < 1 || !psi || !t) return fail(DD_EINVAL, "bad arguments");
  std::vector<double> pref(n);
  for (int32_t k = 0; k < n; ++k) {
    if (!scans[k]) return fail(DD_EINVAL, "scan %d is NULL", k);
    pref[k] = scans[k]->pref > 0 ? scans[k]->pref : 1.0;
  }
  hipStream_t st = (hipStream_t)stream;
  DevBuf d;
  UN_HIP(d.ensure(sizeof(double) * n), "device allocation");
  UN_HIP(hipMemcpyAsync(d.p, pref.data(), sizeof(double) * n, hipMemcpyHostToDevice, st), "copy");
  UN_HIP(nn::log_target(psi, (int64_t)n * S * S, S * S, d.as<double>(), t, st), "targets");
  UN_HIP(hipStreamSynchronize(st), "synchronize");
  d.release();
  return DD_OK;
}

dd_status dd_unet_predict(dd_unet* u, dd_scan* const* scans, int32_t n, double spot_tol,
                          dd_precision p, double* psi, int32_t* used_fallback, void* stream) {
  if (!u || !scans || n < 1 || !psi || !used_fallback || !(spot_tol >= 0))
    return fail(DD_EINVAL, "bad arguments");
  for (int32_t k = 0; k < n; ++k)
    if (!scans[k]) return fail(DD_EINVAL, "scan %d is NULL", k);
  hipStream_t st = (hipStream_t)stream;
  const bool mixed = p == DD_MIXED;
  // 1. network prediction for the scans inside the training range
  std::vector<int32_t> ok_idx, fb_idx;
  for (int32_t k = 0; k < n; ++k) (in_training_range(scans[k]) ? ok_idx : fb_idx).push_back(k);
  const int chunk = 64;
  DevBuf x, yb, prefd, spot;
  dd_status rc;
  if (!ok_idx.empty()) {
    UN_HIP(x.ensure(sizeof(float) * chunk * S * S * 3), "device allocation");
    UN_HIP(yb.ensure(sizeof(float) * chunk * S * S), "device allocation");
    UN_HIP(prefd.ensure(sizeof(double) * chunk), "device allocation");
    for (size_t b0 = 0; b0 < ok_idx.size(); b0 += chunk) {
      const int nb = (int)std::min<size_t>(chunk, ok_idx.size() - b0);
      std::vector<dd_scan*> sub(nb);
      std::vector<double> pref(nb);
      for (int q = 0; q < nb; ++q) {
        sub[q] = scans[ok_idx[b0 + q]];
        pref[q] = sub[q]->pref;
      }
      rc = dd_surrogate_inputs(sub.data(), nb, x.as<float>(), st);
      if (rc != DD_OK) return rc;
      rc = dd_unet_forward(u, nb, x.as<float>(), yb.as<float>(), st);
      if (rc != DD_OK) return rc;
      UN_HIP(hipMemcpyAsync(prefd.p, pref.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st),
             "copy");
      // predictions land in their scans' output slots (maps are contiguous
      // only within the chunk, so write each map separately)
      for (int q = 0; q < nb; ++q)
        UN_HIP(nn::exp_out(yb.as<float>() + (size_t)q * S * S, S * S, S * S, prefd.as<double>() + q,
                           psi + (size_t)ok_idx[b0 + q] * S * S, st),
               "prediction output");
      UN_HIP(hipStreamSynchronize(st), "synchronize");
    }
  }
  // 2. judge: the exact middle row (row 31) of every predicted map
  std::vector<double> row_exact;
  if (!ok_idx.empty()) {
    const int row = 31;
    std::vector<dd_scan*> sub(ok_idx.size());
    for (size_t q = 0; q < ok_idx.size(); ++q) sub[q] = scans[ok_idx[q]];
    UN_HIP(spot.ensure(sizeof(double) * ok_idx.size() * S), "device allocation");
    std::vector<double*> outs(ok_idx.size());
    for (size_t q = 0; q < ok_idx.size(); ++q) outs[q] = spot.as<double>() + q * S;
    rc = run_batch(sub.data(), (int32_t)sub.size(), DD_Q_FINAL_AT_PROBES, mixed, outs.data(), 1, st,
                   row, 1);
    if (rc != DD_OK) return rc;
    row_exact.resize(ok_idx.size() * S);
    std::vector<double> row_pred(ok_idx.size() * S);
    UN_HIP(hipMemcpyAsync(row_exact.data(), spot.p, sizeof(double) * row_exact.size(),
                          hipMemcpyDeviceToHost, st),
           "copy");
    for (size_t q = 0; q < ok_idx.size(); ++q)
      UN_HIP(hipMemcpyAsync(row_pred.data() + q * S, psi + (size_t)ok_idx[q] * S * S + row * S,
                            sizeof(double) * S, hipMemcpyDeviceToHost, st),
             "copy");
    UN_HIP(hipStreamSynchronize(st), "synchronize");
    std::vector<int32_t> keep;
    for (size_t q = 0; q < ok_idx.size(); ++q) {
      double num = 0, den = 0;
      for (int c = 0; c < S; ++c) {
        const double d = row_pred[q * S + c] - row_exact[q * S + c];
        num += d * d;
        den += row_exact[q * S + c] * row_exact[q * S + c];
      }
      const double rel = den > 0 ? std::sqrt(num / den) : (num > 0 ? 1.0 : 0.0);
      if (rel <= spot_tol && std::isfinite(rel))
        keep.push_back(ok_idx[q]);
      else
        fb_idx.push_back(ok_idx[q]);
    }
    ok_idx.swap(keep);
  }
  // 3. fallback: the exact final map
  for (int32_t k = 0; k < n; ++k) used_fallback[k] = 0;
  if (!fb_idx.empty()) {
    std::sort(fb_idx.begin(), fb_idx.end());
    std::vector<dd_scan*> sub(fb_idx.size());
    std::vector<double*> outs(fb_idx.size());
    for (size_t q = 0; q < fb_idx.size(); ++q) {
      sub[q] = scans[fb_idx[q]];
      outs[q] = psi + (size_t)fb_idx[q] * S * S;
      used_fallback[fb_idx[q]] = 1;
    }
    rc = run_batch(sub.data(), (int32_t)sub.size(), DD_Q_FINAL_AT_PROBES, mixed, outs.data(), 1, st,
                   0, -1);
    if (rc != DD_OK) return rc;
  }
  return DD_OK;
}
