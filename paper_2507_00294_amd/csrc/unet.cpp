// unet.cpp -- the learned surrogate of libdd.
//
// A 4-level U-Net (32, 64, 128, 256 channels at 64^2, 32^2, 16^2, 8^2) maps a
// 64x64 scan's per-probe inputs -- the first-arrival-time map, kappa = D dwell
// / pitch^2, sigma / pitch, the time since the probe's last visit and the
// probe's own-visit term -- to the dimensionless damage map at the end of the
// scan (Eq. 6 at every probe position, without the Q0 / (4 pi D) prefactor).
// The own-visit term O (the a = 0 limit of the bracket of Eq. 6 summed over
// the probe's own visits, a closed form) is also an additive prior: the
// prediction is O + exp(y) with y the network output, so the network learns
// (the logarithm of) what the other probes contribute.  Training minimises
// the per-map relative L2 error, the accuracy measure of the surrogate.
//
// Kernels: 3x3 convolutions on BF16 MFMA over LDS halo tiles (unet_conv.hip)
// for the forward pass and the data gradient -- the decoder's upsampling and
// skip concatenation are read directly by its first convolution, and the
// output head is reduced in the last convolution's epilogue -- im2col +
// split-K MFMA GEMM for the weight gradient, FP32 elementwise kernels and Adam
// (unet_kernels.hip).
// Predictions are judged by the exact kernels (an exact 8 x 8 probe sub-grid
// per map) and replaced by the exact map when the judge rejects them or the
// scan lies outside the training range.
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

constexpr int S = 64;        // input side
constexpr int NPX = S * S;   // pixels per map
constexpr int CIN = DD_SURROGATE_CHANNELS;
constexpr int KPAD0 = 64;    // row length of the first layer's im2col (9 CIN padded)
constexpr int kPredictChunk = 2048;  // maps per inference forward pass (per-map rate measured
                                     // 427k/s at 512, 492k/s at 1024, 511k/s at 2000 maps)
// Probes the exact judge evaluates per predicted map: the 8 x 8 sub-grid of
// stride 9 (rows and columns 0, 9, ..., 63), corners and borders included.
const dd::MapSel kJudge{0, 0, 9, 8, 8};

struct Conv {
  int H, lg, ci, co, kpad;
  int64_t w_off, b_off, wf_off, wd_off;
  DevBuf Z, A;  // pre-activation (FP32, training only), activation (BF16 NHWC)
};

#define UN_HIP(call, what)                           \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

}  // namespace

struct dd_unet {
  std::vector<Conv> L;
  nn::ConvTable tab{};
  int64_t head_w = 0, n_params = 0, n_wf = 0, n_wd = 0;
  DevBuf w, wf, wd, g, m, v;  // FP32 master, BF16 forward / dgrad layouts, gradient, Adam moments
  int64_t step = 0;
  int capB = 0, capB_train = 0, B = 0;
  bool last_train = false;
  DevBuf p1, p2, p3, y, col0;
  DevBuf col, dA0, dA1, dZ, dZb, ds1, ds2, ds3, part, loss_map, norm_part, scale_norm;
  size_t part_elems = 0;
  // second stream (default priority, non-blocking) on which predict runs the
  // exact judge while the network runs on the caller's stream
  hipStream_t judge_stream = nullptr;
  hipEvent_t judge_done = nullptr;
  // predict's buffers (input chunk, own-visit term, per-scan pointers and
  // prefactors, judge rows, spot errors), kept between calls
  DevBuf px, pown, pfeat, pout, ppref, pspot, prel;
};

namespace {

// 14 convolutions in forward order.
void build_layers(dd_unet& u) {
  struct Spec {
    int H, ci, co;
  };
  const Spec specs[] = {
      {64, CIN, 32},  {64, 32, 32},  {32, 32, 64},  {32, 64, 64},   {16, 64, 128},
      {16, 128, 128}, {8, 128, 256}, {8, 256, 256}, {16, 384, 128}, {16, 128, 128},
      {32, 192, 64},  {32, 64, 64},  {64, 96, 32},  {64, 32, 32}};
  int64_t off = 0, offf = 0, offd = 0;
  u.tab.n = 0;
  for (const Spec& s : specs) {
    Conv c;
    c.H = s.H;
    c.lg = 0;
    while ((1 << c.lg) < s.H) ++c.lg;
    c.ci = s.ci;
    c.co = s.co;
    c.kpad = s.ci % 32 == 0 ? 9 * s.ci : KPAD0;
    c.w_off = off;
    off += 9LL * s.ci * s.co;
    c.b_off = off;
    off += s.co;
    c.wf_off = offf;
    offf += (int64_t)s.co * c.kpad;
    const bool dgrad = s.ci % 32 == 0;
    c.wd_off = dgrad ? offd : 0;
    if (dgrad) offd += 9LL * s.ci * s.co;
    u.tab.l[u.tab.n++] = nn::ConvDesc{c.ci, c.co, c.kpad, dgrad ? 1 : 0, c.w_off, c.wf_off, c.wd_off};
    u.L.push_back(std::move(c));
  }
  u.head_w = off;  // 32 weights then 1 bias
  off += 33;
  u.n_params = off;
  u.n_wf = offf;
  u.n_wd = offd;
}

int64_t M_of(const dd_unet& u, const Conv& c) { return (int64_t)u.B * c.H * c.H; }

int wgrad_splits(const Conv& c, int64_t M) {
  const int tiles = ((9 * c.ci + 63) / 64) * ((c.co + 63) / 64);
  int64_t s = std::max<int64_t>(1, std::min<int64_t>(M / 256, 2048 / std::max(tiles, 1)));
  return (int)std::min<int64_t>(s, 512);
}

// Buffers of a forward pass over B maps; with `train`, also what the backward
// pass needs.
dd_status ensure_capacity(dd_unet& u, int B, bool train) {
  const int64_t M64 = (int64_t)B * NPX, M32 = M64 / 4, M16 = M64 / 16, M8 = M64 / 64;
  const size_t nL = u.L.size();
  if (B > u.capB) {
    // the last layer's activation is only kept for training
    for (size_t l = 0; l + 1 < nL; ++l) {
      Conv& c = u.L[l];
      UN_HIP(c.A.ensure(sizeof(__bf16) * (int64_t)B * c.H * c.H * c.co), "device allocation");
    }
    UN_HIP(u.p1.ensure(sizeof(__bf16) * M32 * 32), "device allocation");
    UN_HIP(u.p2.ensure(sizeof(__bf16) * M16 * 64), "device allocation");
    UN_HIP(u.p3.ensure(sizeof(__bf16) * M8 * 128), "device allocation");
    UN_HIP(u.y.ensure(sizeof(float) * M64), "device allocation");
    u.capB = B;
  }
  if (train && B > u.capB_train) {
    size_t max_mco = 0, max_mci = 0, max_col = 0, max_part = 0;
    UN_HIP(u.L[nL - 1].A.ensure(sizeof(__bf16) * M64 * u.L[nL - 1].co), "device allocation");
    UN_HIP(u.col0.ensure(sizeof(__bf16) * M64 * KPAD0), "device allocation");
    for (Conv& c : u.L) {
      const int64_t M = (int64_t)B * c.H * c.H;
      UN_HIP(c.Z.ensure(sizeof(float) * M * c.co), "device allocation");
      max_mco = std::max(max_mco, (size_t)(M * c.co));
      max_mci = std::max(max_mci, (size_t)(M * c.ci));
      if (c.ci % 32 == 0) max_col = std::max(max_col, (size_t)(M * 9 * c.ci));
      const int sp = nn::gemm_splits(9 * c.ci, (int)M, wgrad_splits(c, M));
      max_part = std::max(max_part, (size_t)sp * 9 * c.ci * c.co);
    }
    const size_t dmax = std::max(max_mco, max_mci);
    UN_HIP(u.col.ensure(sizeof(__bf16) * max_col), "device allocation");
    UN_HIP(u.dA0.ensure(sizeof(float) * dmax), "device allocation");
    UN_HIP(u.dA1.ensure(sizeof(float) * dmax), "device allocation");
    UN_HIP(u.dZ.ensure(sizeof(float) * max_mco), "device allocation");
    UN_HIP(u.dZb.ensure(sizeof(__bf16) * max_mco), "device allocation");
    UN_HIP(u.ds1.ensure(sizeof(float) * M64 * 32), "device allocation");
    UN_HIP(u.ds2.ensure(sizeof(float) * M32 * 64), "device allocation");
    UN_HIP(u.ds3.ensure(sizeof(float) * M16 * 128), "device allocation");
    UN_HIP(u.part.ensure(sizeof(float) * max_part), "device allocation");
    u.part_elems = max_part;
    u.capB_train = B;
  }
  return DD_OK;
}

// Input of a convolution: the network input x0 (first layer, FP32), a plain
// activation x, or (coarse != NULL) the decoder's concatenation
// [nearest-2x upsampling of coarse (c1 channels), x (the skip map)].
struct In {
  const __bf16* x = nullptr;
  const __bf16* coarse = nullptr;
  int c1 = 0;
  const float* x0 = nullptr;
};

// pool: where the 2x2 average of the activation goes (layers 1, 3, 5), or NULL
dd_status conv_fwd(dd_unet& u, size_t l, In in, bool train, hipStream_t st,
                   __bf16* pool = nullptr) {
  Conv& c = u.L[l];
  const __bf16* wt = u.wf.as<__bf16>() + c.wf_off;
  const float* bias = u.w.as<float>() + c.b_off;
  float* z = train ? c.Z.as<float>() : nullptr;
  if (c.ci % 32 != 0) {
    UN_HIP(nn::conv3_first_silu(in.x0, u.B, c.lg, c.ci, wt, bias, c.A.as<__bf16>(), z, st), "conv");
  } else if (in.coarse) {
    UN_HIP(nn::conv3_upcat_silu(in.coarse, in.c1, in.x, c.ci - in.c1, u.B, c.lg, wt, bias,
                                c.A.as<__bf16>(), z, c.co, st),
           "conv");
  } else if (l + 1 == u.L.size()) {
    UN_HIP(nn::conv3_silu_head(in.x, u.B, c.lg, c.ci, wt, bias, u.w.as<float>() + u.head_w,
                               train ? c.A.as<__bf16>() : nullptr, z, u.y.as<float>(), st),
           "conv");
  } else {
    UN_HIP(nn::conv3_silu(in.x, u.B, c.lg, c.ci, wt, bias, c.A.as<__bf16>(), z, c.co, pool, st),
           "conv");
  }
  return DD_OK;
}

// Backward of one convolution: from dA (gradient of its activation) and its
// input, the gradients of its weights and bias, and dX (the gradient of its
// input, of the concatenation for a decoder input) when requested.
dd_status conv_bwd(dd_unet& u, Conv& c, In in, const float* dA, float* dX, hipStream_t st) {
  const int64_t M = M_of(u, c);
  UN_HIP(nn::silu_bwd(dA, c.Z.as<float>(), M * c.co, u.dZ.as<float>(), u.dZb.as<__bf16>(), st),
         "SiLU backward");
  UN_HIP(nn::colsum_add(u.dZ.as<float>(), (int)M, c.co, u.g.as<float>() + c.b_off, st),
         "bias gradient");
  const __bf16* col = u.col.as<__bf16>();
  int ld = 9 * c.ci;
  if (c.ci % 32 != 0) {
    UN_HIP(nn::im2col(in.x0, u.B, c.H, c.H, c.ci, KPAD0, u.col0.as<__bf16>(), st), "im2col");
    col = u.col0.as<__bf16>();
    ld = KPAD0;
  } else if (in.coarse) {
    UN_HIP(nn::im2col_upcat(in.coarse, in.c1, in.x, c.ci - in.c1, u.B, c.H, u.col.as<__bf16>(), st),
           "im2col");
  } else {
    UN_HIP(nn::im2col(in.x, u.B, c.H, c.H, c.ci, ld, u.col.as<__bf16>(), st), "im2col");
  }
  const int want = wgrad_splits(c, M);
  const int sp = nn::gemm_splits(9 * c.ci, (int)M, want);
  UN_HIP(nn::gemm(col, ld, true, u.dZb.as<__bf16>(), c.co, false, u.part.as<float>(), c.co,
                  9 * c.ci, c.co, (int)M, want, st),
         "weight-gradient GEMM");
  UN_HIP(nn::sum_splits(u.part.as<float>(), sp, 9LL * c.ci * c.co, u.g.as<float>() + c.w_off, st),
         "weight-gradient reduction");
  if (dX)
    UN_HIP(nn::conv3_plain(u.dZ.as<float>(), u.B, c.lg, c.co, u.wd.as<__bf16>() + c.wd_off, dX,
                           c.ci, st),
           "data-gradient convolution");
  return DD_OK;
}

// The input of every layer, in forward order.
std::vector<In> layer_inputs(dd_unet& u, const float* x) {
  auto A = [&](int l) { return (const __bf16*)u.L[l].A.as<__bf16>(); };
  In first;
  first.x0 = x;
  return {first,
          In{A(0)},
          In{u.p1.as<__bf16>()},
          In{A(2)},
          In{u.p2.as<__bf16>()},
          In{A(4)},
          In{u.p3.as<__bf16>()},
          In{A(6)},
          In{A(5), A(7), 256},  // [up(8^2 x 256), skip 16^2 x 128]
          In{A(8)},
          In{A(3), A(9), 128},  // [up(16^2 x 128), skip 32^2 x 64]
          In{A(10)},
          In{A(1), A(11), 64},  // [up(32^2 x 64), skip 64^2 x 32]
          In{A(12)}};
}

#define STEP(expr) \
  if ((rc = (expr)) != DD_OK) return rc

dd_status forward(dd_unet& u, const float* x, bool train, hipStream_t st) {
  auto& L = u.L;
  dd_status rc;
  u.last_train = train;
  const std::vector<In> in = layer_inputs(u, x);
  STEP(conv_fwd(u, 0, in[0], train, st));
  // the 2x2 poolings run in the epilogues of layers 1, 3 and 5
  STEP(conv_fwd(u, 1, in[1], train, st, u.p1.as<__bf16>()));
  STEP(conv_fwd(u, 2, in[2], train, st));
  STEP(conv_fwd(u, 3, in[3], train, st, u.p2.as<__bf16>()));
  STEP(conv_fwd(u, 4, in[4], train, st));
  STEP(conv_fwd(u, 5, in[5], train, st, u.p3.as<__bf16>()));
  for (size_t l = 6; l < L.size(); ++l) STEP(conv_fwd(u, l, in[l], train, st));
  return DD_OK;
}

dd_status backward(dd_unet& u, const float* x, const float* dy, hipStream_t st) {
  auto& L = u.L;
  const int B = u.B;
  const int64_t M64 = (int64_t)B * NPX, M32 = M64 / 4, M16 = M64 / 16;
  float* a0 = u.dA0.as<float>();
  float* a1 = u.dA1.as<float>();
  dd_status rc;
  const std::vector<In> in = layer_inputs(u, x);
  UN_HIP(nn::fill(u.ds1.as<float>(), M64 * 32, 0.f, st), "fill");
  UN_HIP(nn::fill(u.ds2.as<float>(), M32 * 64, 0.f, st), "fill");
  UN_HIP(nn::fill(u.ds3.as<float>(), M16 * 128, 0.f, st), "fill");
  UN_HIP(nn::head_bwd(dy, L[13].A.as<__bf16>(), M64, 32, u.w.as<float>() + u.head_w, a0,
                      u.g.as<float>() + u.head_w, st),
         "head backward");
  STEP(conv_bwd(u, L[13], in[13], a0, a1, st));
  STEP(conv_bwd(u, L[12], in[12], a1, a0, st));  // a0 = d[up, skip] at 64^2 x 96
  UN_HIP(nn::up_concat_bwd(a0, B, 32, 32, 64, 32, a1, u.ds1.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[11], in[11], a1, a0, st));
  STEP(conv_bwd(u, L[10], in[10], a0, a1, st));  // a1 = d[up, skip] at 32^2 x 192
  UN_HIP(nn::up_concat_bwd(a1, B, 16, 16, 128, 64, a0, u.ds2.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[9], in[9], a0, a1, st));
  STEP(conv_bwd(u, L[8], in[8], a1, a0, st));  // a0 = d[up, skip] at 16^2 x 384
  UN_HIP(nn::up_concat_bwd(a0, B, 8, 8, 256, 128, a1, u.ds3.as<float>(), st), "upsample backward");
  STEP(conv_bwd(u, L[7], in[7], a1, a0, st));
  STEP(conv_bwd(u, L[6], in[6], a0, a1, st));  // a1 = d p3 [8^2][128]
  UN_HIP(nn::pool_bwd_add(a1, B, 16, 16, 128, u.ds3.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[5], in[5], u.ds3.as<float>(), a0, st));
  STEP(conv_bwd(u, L[4], in[4], a0, a1, st));  // a1 = d p2 [16^2][64]
  UN_HIP(nn::pool_bwd_add(a1, B, 32, 32, 64, u.ds2.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[3], in[3], u.ds2.as<float>(), a0, st));
  STEP(conv_bwd(u, L[2], in[2], a0, a1, st));  // a1 = d p1 [32^2][32]
  UN_HIP(nn::pool_bwd_add(a1, B, 64, 64, 32, u.ds1.as<float>(), st), "pool backward");
  STEP(conv_bwd(u, L[1], in[1], u.ds1.as<float>(), a0, st));
  STEP(conv_bwd(u, L[0], in[0], a0, nullptr, st));
  return DD_OK;
}
#undef STEP

// Per-probe surrogate table of a 64x64 scan (CIN + 1 floats per probe):
//   0: first visit start / scan duration;
//   1: (log10 kappa + 1) / 3 with kappa = D dwell / pitch^2;
//   2: (sigma / pitch - 0.6) / 0.4;
//   3: ln(lambda_last) / ln(V), lambda_last = V - (index of the last visit):
//      the time from the start of the probe's last visit to the end of the
//      scan, in dwells;
//   4: (ln O + 4) / 4;
//   5: O = sum over the probe's visits of ln(b1 / b0) with
//      b0 = 2 sigma_hat^2 + 4 kappa (lambda - 1), b1 = b0 + 4 kappa, lambda =
//      V - v for visit index v: the a = 0 bracket of Eq. 6 at the end of the
//      scan, i.e. the dimensionless damage that a probe's own visits leave at
//      its centre.
// Returns false when a probe is never visited (the scan is then outside what
// the surrogate accepts).
bool scan_table(const dd_scan* s, float* tab) {
  const int n = s->desc.nx * s->desc.ny;
  const int64_t V = s->V;
  std::vector<int64_t> first(n, -1), last(n, -1);
  std::vector<double> own(n, 0.0);
  const double kap = s->kappa, s2 = s->s2;
  for (int64_t v = 0; v < V; ++v) {
    const int p = s->ids[v];
    if (first[p] < 0) first[p] = v;
    last[p] = v;
    const double lam = (double)(V - v);
    const double b0 = s2 + 4.0 * kap * (lam - 1.0);
    own[p] += std::log1p(4.0 * kap / b0);
  }
  const float c1 = (float)((std::log10(kap) + 1.0) / 3.0);
  const float c2 = (float)((s->desc.sigma_m / s->desc.pitch_m - 0.6) / 0.4);
  const double lnV = std::log((double)V);
  for (int p = 0; p < n; ++p) {
    if (first[p] < 0 || !(own[p] > 0)) return false;
    float* t = tab + (size_t)p * (CIN + 1);
    t[0] = (float)((double)first[p] / (double)V);
    t[1] = c1;
    t[2] = c2;
    t[3] = (float)(std::log((double)(V - last[p])) / lnV);
    t[4] = (float)((std::log(own[p]) + 4.0) / 4.0);
    t[5] = (float)own[p];
  }
  return true;
}

bool in_training_range(const dd_scan* s) {
  const double kap = s->kappa;
  const double sh = s->desc.sigma_m / s->desc.pitch_m;
  return s->desc.nx == S && s->desc.ny == S && kap >= 0.99 * 2.5e-5 && kap <= 101.0 && sh >= 0.199 &&
         sh <= 1.001 && s->V >= NPX;
}

// Builds (once) the scan's device table; ok = false if the scan is not
// accepted.
dd_status ensure_table(dd_scan* s, hipStream_t st, bool& ok) {
  ok = false;
  if (s->sur_state == 0) {
    std::vector<float> h;
    if (s->desc.nx == S && s->desc.ny == S && s->V >= NPX) {
      h.resize((size_t)NPX * (CIN + 1));
      if (!scan_table(s, h.data())) h.clear();
    }
    if (h.empty()) {
      s->sur_state = -1;  // the scan itself is outside what the surrogate accepts
    } else {
      // a device error leaves the state unset, so a later call retries
      UN_HIP(s->sur.ensure(sizeof(float) * h.size()), "device allocation");
      UN_HIP(hipMemcpyAsync(s->sur.p, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice,
                            st),
             "copy");
      UN_HIP(hipStreamSynchronize(st), "synchronize");
      s->sur_state = 1;
    }
  }
  ok = s->sur_state == 1;
  return DD_OK;
}

// Device array of the pointers in v.
template <typename T>
dd_status upload_ptrs(const std::vector<T*>& v, DevBuf& d, hipStream_t st) {
  UN_HIP(d.ensure(sizeof(T*) * std::max<size_t>(v.size(), 1)), "device allocation");
  UN_HIP(hipMemcpyAsync(d.p, v.data(), sizeof(T*) * v.size(), hipMemcpyHostToDevice, st), "copy");
  return DD_OK;
}

dd_status refresh_layouts(dd_unet* u, hipStream_t st) {
  UN_HIP(nn::prep_weights(u->w.as<float>(), u->tab, u->wf.as<__bf16>(), u->wd.as<__bf16>(), st),
         "weight layouts");
  return DD_OK;
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
  // He-normal weights, zero biases, a zero head (the first prediction is
  // own + exp(head bias)).
  std::vector<float> w(u->n_params, 0.f);
  std::mt19937_64 gen(seed);
  for (const Conv& c : u->L) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.0f / (9.0f * c.ci)));
    for (int64_t k = 0; k < 9LL * c.ci * c.co; ++k) w[c.w_off + k] = nd(gen);
  }
  hipError_t e = u->w.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->wf.ensure(sizeof(__bf16) * u->n_wf);
  if (e == hipSuccess) e = u->wd.ensure(sizeof(__bf16) * u->n_wd);
  if (e == hipSuccess) e = u->g.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->m.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->v.ensure(sizeof(float) * u->n_params);
  if (e == hipSuccess) e = u->loss_map.ensure(sizeof(double) * 4096);
  if (e == hipSuccess) e = u->norm_part.ensure(sizeof(double) * nn::kNormBlocks);
  if (e == hipSuccess) e = u->scale_norm.ensure(sizeof(float) * 2);
  if (e == hipSuccess)
    e = hipMemcpy(u->w.p, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = nn::prep_weights(u->w.as<float>(), u->tab, u->wf.as<__bf16>(), u->wd.as<__bf16>(), nullptr);
  if (e == hipSuccess) e = nn::fill(u->g.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = nn::fill(u->m.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = nn::fill(u->v.as<float>(), u->n_params, 0.f, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dd_unet_destroy(u);
    return hip_fail(e, "surrogate allocation");
  }
  *out = u;
  return DD_OK;
}

void dd_unet_destroy(dd_unet* u) {
  if (!u) return;
  for (DevBuf* b : {&u->w, &u->wf, &u->wd, &u->g, &u->m, &u->v, &u->col0, &u->p1, &u->p2, &u->p3,
                    &u->y, &u->col, &u->dA0, &u->dA1, &u->dZ, &u->dZb,
                    &u->ds1, &u->ds2, &u->ds3, &u->part, &u->loss_map, &u->norm_part,
                    &u->scale_norm, &u->px, &u->pown, &u->pfeat, &u->pout, &u->ppref, &u->pspot,
                    &u->prel})
    b->release();
  for (Conv& c : u->L) {
    c.Z.release();
    c.A.release();
  }
  if (u->judge_done) (void)hipEventDestroy(u->judge_done);
  if (u->judge_stream) (void)hipStreamDestroy(u->judge_stream);
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
    dd_status rc = refresh_layouts(u, nullptr);
    if (rc != DD_OK) return rc;
    UN_HIP(hipDeviceSynchronize(), "synchronize");
  }
  return DD_OK;
}

dd_status dd_unet_adam_state(dd_unet* u, float* m_get, float* v_get, int64_t* step_get,
                             const float* m_set, const float* v_set, const int64_t* step_set) {
  if (!u || (!m_get && !v_get && !step_get && !m_set && !v_set && !step_set))
    return fail(DD_EINVAL, "NULL argument");
  if (step_set && *step_set < 0) return fail(DD_EINVAL, "negative Adam step");
  const size_t bytes = sizeof(float) * u->n_params;
  if (m_get) UN_HIP(hipMemcpy(m_get, u->m.p, bytes, hipMemcpyDeviceToHost), "moment copy");
  if (v_get) UN_HIP(hipMemcpy(v_get, u->v.p, bytes, hipMemcpyDeviceToHost), "moment copy");
  if (step_get) *step_get = u->step;
  if (m_set) UN_HIP(hipMemcpy(u->m.p, m_set, bytes, hipMemcpyHostToDevice), "moment copy");
  if (v_set) UN_HIP(hipMemcpy(u->v.p, v_set, bytes, hipMemcpyHostToDevice), "moment copy");
  if (step_set) u->step = *step_set;
  return DD_OK;
}

dd_status dd_unet_grads(const dd_unet* u, float* host_out) {
  if (!u || !host_out) return fail(DD_EINVAL, "NULL argument");
  UN_HIP(hipMemcpy(host_out, u->g.p, sizeof(float) * u->n_params, hipMemcpyDeviceToHost),
         "gradient copy");
  return DD_OK;
}

dd_status dd_unet_forward(dd_unet* u, int32_t batch, const float* x, float* y, int32_t train,
                          void* stream) {
  if (!u || !x || !y || batch < 1) return fail(DD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  dd_status rc = ensure_capacity(*u, batch, train != 0);
  if (rc != DD_OK) return rc;
  u->B = batch;
  rc = forward(*u, x, train != 0, st);
  if (rc != DD_OK) return rc;
  UN_HIP(hipMemcpyAsync(y, u->y.p, sizeof(float) * batch * NPX, hipMemcpyDeviceToDevice, st),
         "output copy");
  return DD_OK;
}

dd_status dd_unet_backward(dd_unet* u, const float* x, const float* dy, void* stream) {
  if (!u || !x || !dy || u->B < 1 || !u->last_train)
    return fail(DD_EINVAL, "backward needs a training forward pass first");
  return backward(*u, x, dy, (hipStream_t)stream);
}

dd_status dd_unet_loss(dd_unet* u, int32_t maps, const float* y, const float* own, const float* t,
                       float anchor, float* dy, double* loss_host, void* stream) {
  if (!u || maps < 1 || maps > 4096 || !y || !own || !t || !dy || !(anchor >= 0))
    return fail(DD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  UN_HIP(nn::rel_l2(y, own, t, maps, NPX, anchor, dy, u->loss_map.as<double>(), st), "loss");
  if (loss_host) {
    std::vector<double> part(maps);
    UN_HIP(hipMemcpyAsync(part.data(), u->loss_map.p, sizeof(double) * maps, hipMemcpyDeviceToHost,
                          st),
           "copy");
    UN_HIP(hipStreamSynchronize(st), "synchronize");
    double s = 0.0;
    for (double p : part) s += p;
    *loss_host = s / maps;
  }
  return DD_OK;
}

dd_status dd_unet_adam(dd_unet* u, float lr, float beta1, float beta2, float eps, float clip,
                       float* grad_norm_host, void* stream) {
  if (!u || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) ||
      !(clip >= 0))
    return fail(DD_EINVAL, "bad Adam parameters");
  hipStream_t st = (hipStream_t)stream;
  u->step += 1;
  const float bc1 = 1.0f - std::pow(beta1, (float)u->step);
  const float bc2 = 1.0f - std::pow(beta2, (float)u->step);
  UN_HIP(nn::clip_scale(u->g.as<float>(), u->n_params, clip, u->norm_part.as<double>(),
                        u->scale_norm.as<float>(), st),
         "gradient norm");
  UN_HIP(nn::adam(u->w.as<float>(), u->m.as<float>(), u->v.as<float>(), u->g.as<float>(),
                  u->scale_norm.as<float>(), u->n_params, lr, beta1, beta2, eps, bc1, bc2, st),
         "Adam step");
  dd_status rc = refresh_layouts(u, st);
  if (rc != DD_OK) return rc;
  if (grad_norm_host) {
    float sn[2];
    UN_HIP(hipMemcpyAsync(sn, u->scale_norm.p, sizeof sn, hipMemcpyDeviceToHost, st), "copy");
    UN_HIP(hipStreamSynchronize(st), "synchronize");
    *grad_norm_host = sn[1];
  }
  return DD_OK;
}

dd_status dd_surrogate_batch(const float* x_all, const float* own_all, const float* t_all,
                             int64_t n_all, const int32_t* idx, const int32_t* transform,
                             int32_t nb, float* xb, float* ob, float* tb, void* stream) {
  if (!x_all || !own_all || !t_all || n_all < 1 || !idx || !transform || nb < 1 || !xb || !ob ||
      !tb)
    return fail(DD_EINVAL, "bad arguments");
  UN_HIP(nn::gather_batch(x_all, own_all, t_all, n_all, CIN, S, idx, transform, nb, xb, ob, tb,
                          (hipStream_t)stream),
         "batch gather");
  return DD_OK;
}

dd_status dd_surrogate_inputs(dd_scan* const* scans, int32_t n, float* x, float* own,
                              void* stream) {
  if (!scans || n < 1 || !x || !own) return fail(DD_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  std::vector<const float*> ptrs(n);
  for (int32_t k = 0; k < n; ++k) {
    if (!scans[k]) return fail(DD_EINVAL, "scan %d is NULL", k);
    bool ok = false;
    dd_status rc = ensure_table(scans[k], st, ok);
    if (rc != DD_OK) return rc;
    if (!ok)
      return fail(DD_EINVAL,
                  "scan %d: the surrogate needs a 64x64 probe grid with every probe visited", k);
    ptrs[k] = scans[k]->sur.as<float>();
  }
  DevBuf d;
  dd_status rc = upload_ptrs(ptrs, d, st);
  if (rc != DD_OK) return rc;
  UN_HIP(nn::gather_features(d.as<const float*>(), n, CIN, NPX, x, own, st), "input gather");
  UN_HIP(hipStreamSynchronize(st), "synchronize");
  return DD_OK;
}

dd_status dd_surrogate_targets(dd_scan* const* scans, int32_t n, const double* psi, float* t,
                               void* stream) {
  if (!scans || n < 1 || !psi || !t) return fail(DD_EINVAL, "bad arguments");
  std::vector<double> pref(n);
  for (int32_t k = 0; k < n; ++k) {
    if (!scans[k]) return fail(DD_EINVAL, "scan %d is NULL", k);
    pref[k] = scans[k]->pref;
  }
  hipStream_t st = (hipStream_t)stream;
  DevBuf d;
  UN_HIP(d.ensure(sizeof(double) * n), "device allocation");
  UN_HIP(hipMemcpyAsync(d.p, pref.data(), sizeof(double) * n, hipMemcpyHostToDevice, st), "copy");
  UN_HIP(nn::target(psi, (int64_t)n * NPX, NPX, d.as<double>(), t, st), "targets");
  UN_HIP(hipStreamSynchronize(st), "synchronize");
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
  dd_status rc;
  // 1. network prediction for the accepted scans inside the training range
  std::vector<int32_t> ok_idx, fb_idx;
  for (int32_t k = 0; k < n; ++k) {
    bool ok = false;
    if (in_training_range(scans[k])) {
      rc = ensure_table(scans[k], st, ok);
      if (rc != DD_OK) return rc;
    }
    (ok ? ok_idx : fb_idx).push_back(k);
  }
  const size_t nok = ok_idx.size();
  DevBuf &x = u->px, &own = u->pown, &d_feat = u->pfeat, &d_out = u->pout, &d_pref = u->ppref,
         &spot = u->pspot, &rel = u->prel;
  if (nok) {
    std::vector<const float*> feat(nok);
    std::vector<double*> outs(nok);
    std::vector<double> pref(nok);
    for (size_t q = 0; q < nok; ++q) {
      feat[q] = scans[ok_idx[q]]->sur.as<float>();
      outs[q] = psi + (size_t)ok_idx[q] * NPX;
      pref[q] = scans[ok_idx[q]]->pref;
    }
    if ((rc = upload_ptrs(feat, d_feat, st)) != DD_OK) return rc;
    if ((rc = upload_ptrs(outs, d_out, st)) != DD_OK) return rc;
    UN_HIP(d_pref.ensure(sizeof(double) * nok), "device allocation");
    UN_HIP(hipMemcpyAsync(d_pref.p, pref.data(), sizeof(double) * nok, hipMemcpyHostToDevice, st),
           "copy");
    const int chunk = (int)std::min<size_t>(kPredictChunk, nok);
    UN_HIP(x.ensure(sizeof(float) * chunk * NPX * CIN), "device allocation");
    UN_HIP(own.ensure(sizeof(float) * chunk * NPX), "device allocation");
    if ((rc = ensure_capacity(*u, chunk, false)) != DD_OK) return rc;
    UN_HIP(spot.ensure(sizeof(double) * nok * kJudge.w * kJudge.h), "device allocation");
    UN_HIP(rel.ensure(sizeof(double) * nok), "device allocation");
    if (!u->judge_stream)
      UN_HIP(hipStreamCreateWithFlags(&u->judge_stream, hipStreamNonBlocking), "stream creation");
    if (!u->judge_done)
      UN_HIP(hipEventCreateWithFlags(&u->judge_done, hipEventDisableTiming), "event creation");
    // the network, enqueued on the caller's stream
    for (size_t b0 = 0; b0 < nok; b0 += chunk) {
      const int nb = (int)std::min<size_t>(chunk, nok - b0);
      UN_HIP(nn::gather_features(d_feat.as<const float*>() + b0, nb, CIN, NPX, x.as<float>(),
                                 own.as<float>(), st),
             "input gather");
      u->B = nb;
      if ((rc = forward(*u, x.as<float>(), false, st)) != DD_OK) return rc;
      UN_HIP(nn::output(u->y.as<float>(), own.as<float>(), nb, NPX, d_pref.as<double>() + b0,
                        d_out.as<double*>() + b0, st),
             "prediction output");
    }
    // 2. judge: the exact values of every predicted map on the 8 x 8 probe
    // sub-grid of stride 9 (rows and columns 0, 9, ..., 63: corners, borders
    // and interior, 1/64 of the map's pairs), planned on the host and run on
    // the judge stream while the network runs
    std::vector<dd_scan*> sub(nok);
    for (size_t q = 0; q < nok; ++q) sub[q] = scans[ok_idx[q]];
    std::vector<double*> rows(nok);
    for (size_t q = 0; q < nok; ++q) rows[q] = spot.as<double>() + q * kJudge.w * kJudge.h;
    rc = run_batch(sub.data(), (int32_t)nok, DD_Q_FINAL_AT_PROBES, mixed, rows.data(), 1,
                   u->judge_stream, kJudge);
    if (rc != DD_OK) return rc;
    UN_HIP(hipEventRecord(u->judge_done, u->judge_stream), "event record");
    UN_HIP(hipStreamWaitEvent(st, u->judge_done, 0), "stream wait");
    UN_HIP(nn::spot(d_out.as<const double*>(), spot.as<double>(), (int)nok, S, kJudge.x0,
                    kJudge.y0, kJudge.step, kJudge.w, kJudge.h, rel.as<double>(), st),
           "spot check");
    std::vector<double> relh(nok);
    UN_HIP(hipMemcpyAsync(relh.data(), rel.p, sizeof(double) * nok, hipMemcpyDeviceToHost, st),
           "copy");
    UN_HIP(hipStreamSynchronize(st), "synchronize");
    for (size_t q = 0; q < nok; ++q)
      if (!(relh[q] <= spot_tol)) fb_idx.push_back(ok_idx[q]);
  }
  // 3. fallback: the exact final map
  for (int32_t k = 0; k < n; ++k) used_fallback[k] = 0;
  if (!fb_idx.empty()) {
    std::sort(fb_idx.begin(), fb_idx.end());
    std::vector<dd_scan*> sub(fb_idx.size());
    std::vector<double*> outs(fb_idx.size());
    for (size_t q = 0; q < fb_idx.size(); ++q) {
      sub[q] = scans[fb_idx[q]];
      outs[q] = psi + (size_t)fb_idx[q] * NPX;
      used_fallback[fb_idx[q]] = 1;
    }
    rc = run_batch(sub.data(), (int32_t)sub.size(), DD_Q_FINAL_AT_PROBES, mixed, outs.data(), 1, st,
                   MapSel{});
    if (rc != DD_OK) return rc;
  }
  UN_HIP(hipStreamSynchronize(st), "synchronize");
  return DD_OK;
}
