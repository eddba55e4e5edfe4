// unet_kernels.h -- launchers of the surrogate's HIP kernels (unet_conv.hip,
// unet_kernels.hip).  All activations are NHWC FP32; GEMM operands BF16.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dd {
namespace nn {

// One convolution layer for the weight-layout kernel.
struct ConvDesc {
  int ci, co, kpad, has_dgrad;  // kpad: row length of the forward layout (>= 9 ci)
  int64_t w_off, wf_off, wd_off;  // FP32 master, BF16 forward [co][kpad], BF16 dgrad [ci][9 co]
};
constexpr int kMaxConv = 16;
struct ConvTable {
  int n;
  ConvDesc l[kMaxConv];
};
constexpr int kNormBlocks = 256;  // partial sums of the gradient norm

// 3x3 convolutions (unet_conv.hip) of x [B][side][side][ci], side = 2^lg in
// 8..64, weights wt [co][9 ci] (k = tap ci + c):
//   conv3_silu:        z = conv + bias, act = SiLU(z) (z stored when non-NULL;
//                      with pool non-NULL, side >= 16, also the 2x2 average of
//                      act, [B][side/2][side/2][co]: the four BF16 values in row order, x 0.25,
//                      rounded to BF16);
//   conv3_upcat_silu:  the same on the channel concatenation [nearest-2x
//                      upsampling of coarse [B][side/2][side/2][c1], skip
//                      [B][side][side][c2]];
//   conv3_silu_head:   co = 32, then y = SiLU(z) . head[0..31] + head[32]
//                      (act and z stored when non-NULL);
//   conv3_plain:       out = conv (the data gradient, with the dgrad layout);
//   conv3_first_silu:  ci < 32 with 9 ci <= 64, co = 32, weights [32][64].
// ci, c1 and co must be multiples of 32 except in conv3_first_silu.
hipError_t conv3_silu(const __bf16* x, int B, int lg, int ci, const __bf16* wt, const float* bias,
                      __bf16* act, float* z, int co, __bf16* pool, hipStream_t st);
hipError_t conv3_upcat_silu(const __bf16* coarse, int c1, const __bf16* skip, int c2, int B,
                            int lg, const __bf16* wt, const float* bias, __bf16* act, float* z,
                            int co, hipStream_t st);
hipError_t conv3_silu_head(const __bf16* x, int B, int lg, int ci, const __bf16* wt,
                           const float* bias, const float* head, __bf16* act, float* z, float* y,
                           hipStream_t st);
hipError_t conv3_plain(const float* x, int B, int lg, int ci, const __bf16* wt, float* out, int co,
                       hipStream_t st);
hipError_t conv3_first_silu(const float* x, int B, int lg, int ci, const __bf16* wt,
                            const float* bias, __bf16* act, float* z, hipStream_t st);

// C = A B on BF16 MFMA (FP32 accumulation); ta/tb select transposed storage;
// with ksplit > 1 the partial matrices (gemm_splits() of them) are written at
// C + s*M*ldc and must be added by sum_splits.
hipError_t gemm(const __bf16* A, int lda, bool ta, const __bf16* B, int ldb, bool tb, float* C,
                int ldc, int M, int N, int K, int ksplit, hipStream_t st);
int gemm_splits(int M, int K, int ksplit);
hipError_t sum_splits(const float* part, int splits, int64_t n, float* out, hipStream_t st);
hipError_t im2col(const float* x, int B, int H, int W, int C, int ld, __bf16* col, hipStream_t st);
hipError_t im2col(const __bf16* x, int B, int H, int W, int C, int ld, __bf16* col,
                  hipStream_t st);
// im2col of the virtual concatenation [upsampled coarse (c1), skip (c2)].
hipError_t im2col_upcat(const __bf16* coarse, int c1, const __bf16* skip, int c2, int B, int H,
                        __bf16* col, hipStream_t st);
hipError_t silu_bwd(const float* dA, const float* Z, int64_t n, float* dZ, __bf16* dZb,
                    hipStream_t st);
hipError_t colsum_add(const float* dZ, int M, int N, float* db, hipStream_t st);
hipError_t pool_bwd_add(const float* dy, int B, int H, int W, int C, float* dx, hipStream_t st);
hipError_t up_concat_bwd(const float* dout, int B, int h, int w, int C1, int C2, float* dx,
                         float* dskip, hipStream_t st);
hipError_t head_bwd(const float* dy, const __bf16* a, int64_t M, int C, const float* w, float* da,
                    float* dw, hipStream_t st);
// Squared relative L2 error per map (loss_map[b]) of prediction own + exp(y)
// against t; dy of the mean over maps of that error plus the anchor term
// (anchor / npx) sum (r/t)^2 (y - ln r)^2, r = max(t - own, 1e-6 t).
hipError_t rel_l2(const float* y, const float* own, const float* t, int maps, int npx, float anchor,
                  float* dy, double* loss_map, hipStream_t st);
// scale_norm[0] = clipping factor of g (global norm), scale_norm[1] = |g|;
// partial holds kNormBlocks doubles.
hipError_t clip_scale(const float* g, int64_t n, float clip, double* partial, float* scale_norm,
                      hipStream_t st);
hipError_t adam(float* w, float* m, float* v, const float* g, const float* scale, int64_t n,
                float lr, float b1, float b2, float eps, float bc1, float bc2, hipStream_t st);
hipError_t prep_weights(const float* w, const ConvTable& tab, __bf16* wf, __bf16* wd,
                        hipStream_t st);
hipError_t gather_batch(const float* x_all, const float* own_all, const float* t_all,
                        int64_t n_all, int cin, int side, const int32_t* idx, const int32_t* tf,
                        int nb, float* xb, float* ob, float* tb, hipStream_t st);
hipError_t gather_features(const float* const* feat, int nb, int cin, int npx, float* x,
                           float* own, hipStream_t st);
hipError_t output(const float* y, const float* own, int nb, int npx, const double* pref,
                  double* const* out, hipStream_t st);
hipError_t target(const double* psi, int64_t n, int64_t per_map, const double* pref, float* t,
                  hipStream_t st);
// Relative L2 error per map of the predicted values on the probe sub-grid
// (x0 + step u, y0 + step v), u < w, v < h, of side x side maps against the
// exact values exact[map][v w + u].
hipError_t spot(const double* const* pred, const double* exact, int maps, int side, int x0,
                int y0, int step, int w, int h, double* rel, hipStream_t st);
hipError_t fill(float* x, int64_t n, float v, hipStream_t st);

}  // namespace nn
}  // namespace dd
