// unet_kernels.hip -- kernels of the learned surrogate: a U-Net trained and
// run with BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation) on gfx950.
//
// A 3x3 convolution is an im2col (activations FP32 -> BF16 columns) followed by
// a GEMM Z = Xcol W (M = pixels, N = output channels, K = 9 input channels).
// Backward: dW = Xcol^T dZ (split over M, partials added in a fixed order),
// dXcol = dZ W^T, then col2im (a gather, no atomics).  Elementwise kernels
// cover bias + SiLU, 2x2 average pooling, nearest 2x upsampling, the channel
// concatenation of skip connections, the 1x1 output head (FP32), the loss and
// Adam with FP32 master weights.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "unet_kernels.h"

namespace dd {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// GEMM C[M][N] = A[M][K] B[K][N] on BF16 MFMA with FP32 accumulation.
// A element (i, k) is at A[i*lda + k] (TA = false) or A[k*lda + i] (TA = true);
// B element (k, j) is at B[k*ldb + j] (TB = false) or B[j*ldb + k] (TB = true).
// Block tile 64 x 64, K step 32, 256 threads = 4 waves in 2 x 2, each wave a
// 32 x 32 tile = 2 x 2 MFMA 16x16x32 tiles.  LDS holds A as [m][k] and B as
// [n][k] (k contiguous), so that each lane reads its 8 consecutive k values
// of a fragment with one 16-byte read.  blockIdx.z splits K into `ksplit`
// ranges of `kchunk` (a multiple of 32); split s writes its partial C to
// C + s*M*ldc.  Epilogue: EPI_STORE stores C; EPI_BIAS_SILU adds bias[j],
// stores Z = C + bias to Cz and SiLU(Z) to C.
constexpr int BM = 64, BN = 64, BK = 32, LDS_K = BK + 8;  // +8 bf16 padding per row
enum { EPI_STORE = 0, EPI_BIAS_SILU = 1 };

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm(const __bf16* __restrict__ A, int lda,
                                              const __bf16* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc,
                                              float* __restrict__ Cz,
                                              const float* __restrict__ bias, int M, int N, int K,
                                              int kchunk) {
  __shared__ __bf16 As[BM][LDS_K];
  __shared__ __bf16 Bs[BN][LDS_K];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // stage A (64 x 32) and B (32 x 64): 2048 elements each, 8 per thread
    {
      const int r = tid >> 2, c8 = (tid & 3) * 8;  // row r of the tile, k offset c8
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = m0 + r, k = k0 + c8 + e;
        __bf16 v = (__bf16)0.0f;
        if (i < M && k < kend) v = TA ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k];
        As[r][c8 + e] = v;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = n0 + r, k = k0 + c8 + e;
        __bf16 v = (__bf16)0.0f;
        if (j < N && k < kend) v = TB ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j];
        Bs[r][c8 + e] = v;
      }
    }
    __syncthreads();
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int row = wm * 32 + a * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) af[a][e] = As[row][8 * (lane >> 4) + e];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wn * 32 + b * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) bfr[b][e] = Bs[col][8 * (lane >> 4) + e];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  float* Cs = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * 32 + a * 16 + 4 * (lane >> 4) + v;
        const int j = n0 + wn * 32 + b * 16 + (lane & 15);
        if (i < M && j < N) {
          float z = acc[a][b][v];
          if (EPI == EPI_BIAS_SILU) {
            z += bias[j];
            Cz[(int64_t)i * ldc + j] = z;
            Cs[(int64_t)i * ldc + j] = silu(z);
          } else {
            Cs[(int64_t)i * ldc + j] = z;
          }
        }
      }
}

// Sum of `splits` partial matrices in order: out[e] = sum_s part[s*n + e].
__global__ void __launch_bounds__(256) k_sum_splits(const float* __restrict__ part, int splits,
                                                    int64_t n, float* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[(int64_t)k * n + e];
    out[e] = s;
  }
}

// ---------------------------------------------------------------------------
// im2col for a 3x3 convolution with zero padding 1 (NHWC, FP32 -> BF16):
// col[m][(ky*3+kx)*C + c] = x[n][y+ky-1][x+kx-1][c], m = (n*H + y)*W + x.
__global__ void __launch_bounds__(256) k_im2col(const float* __restrict__ x, int B, int H, int W,
                                                int C, __bf16* __restrict__ col) {
  const int64_t K = 9 * (int64_t)C, total = (int64_t)B * H * W * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / K;
    const int k = (int)(e % K);
    const int tap = k / C, c = k % C;
    const int ky = tap / 3, kx = tap % 3;
    const int xx = (int)(m % W), yy = (int)((m / W) % H), n = (int)(m / ((int64_t)W * H));
    const int sy = yy + ky - 1, sx = xx + kx - 1;
    float v = 0.f;
    if (sy >= 0 && sy < H && sx >= 0 && sx < W) v = x[(((int64_t)n * H + sy) * W + sx) * C + c];
    col[e] = (__bf16)v;
  }
}

// col2im (the adjoint of k_im2col): dx[n][y][x][c] = sum over taps of
// dcol[m'][(ky*3+kx)*C + c] with m' the pixel (y-ky+1, x-kx+1); a gather in
// fixed tap order.
__global__ void __launch_bounds__(256) k_col2im(const float* __restrict__ dcol, int B, int H,
                                                int W, int C, float* __restrict__ dx) {
  const int64_t total = (int64_t)B * H * W * C, K = 9 * (int64_t)C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int xx = (int)(p % W), yy = (int)((p / W) % H), n = (int)(p / ((int64_t)W * H));
    float s = 0.f;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int ty = yy - ky + 1, tx = xx - kx + 1;
        if (ty >= 0 && ty < H && tx >= 0 && tx < W)
          s += dcol[(((int64_t)n * H + ty) * W + tx) * K + (ky * 3 + kx) * C + c];
      }
    dx[e] = s;
  }
}

// dZ = dA * SiLU'(Z); also its BF16 copy for the MFMA GEMMs.
__global__ void __launch_bounds__(256) k_silu_bwd(const float* __restrict__ dA,
                                                  const float* __restrict__ Z, int64_t n,
                                                  float* __restrict__ dZ, __bf16* __restrict__ dZb) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float g = dA[e] * silu_grad(Z[e]);
    dZ[e] = g;
    dZb[e] = (__bf16)g;
  }
}

// Column sums db[j] = sum_i dZ[i][j] for a [M][N] matrix; one block per
// column group, rows in a fixed order (deterministic).
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ dZ, int M, int N,
                                                float* __restrict__ db) {
  __shared__ float red[256];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < M; i += 256) s += dZ[(int64_t)i * N + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = red[0];
}

// 2x2 average pooling (NHWC) and its adjoint (which accumulates).
__global__ void __launch_bounds__(256) k_pool_fwd(const float* __restrict__ x, int B, int H, int W,
                                                  int C, float* __restrict__ y) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t total = (int64_t)B * Ho * Wo * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int xo = (int)(p % Wo), yo = (int)((p / Wo) % Ho), n = (int)(p / ((int64_t)Wo * Ho));
    const int64_t base = (((int64_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
    y[e] = 0.25f * (x[base] + x[base + C] + x[base + (int64_t)W * C] + x[base + (int64_t)W * C + C]);
  }
}

__global__ void __launch_bounds__(256) k_pool_bwd(const float* __restrict__ dy, int B, int H, int W,
                                                  int C, float* __restrict__ dx) {
  const int64_t total = (int64_t)B * H * W * C;
  const int Ho = H / 2, Wo = W / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int xx = (int)(p % W), yy = (int)((p / W) % H), n = (int)(p / ((int64_t)W * H));
    dx[e] += 0.25f * dy[(((int64_t)n * Ho + yy / 2) * Wo + xx / 2) * C + c];
  }
}

// Nearest 2x upsampling of x [B][h][w][C1] written into channels [0, C1) of
// a [B][2h][2w][Ct] buffer, and the copy of skip [B][2h][2w][C2] into
// channels [C1, C1+C2): the decoder's concatenation input.
__global__ void __launch_bounds__(256) k_up_concat(const float* __restrict__ x, int B, int h, int w,
                                                   int C1, const float* __restrict__ skip, int C2,
                                                   float* __restrict__ out) {
  const int H = 2 * h, W = 2 * w, Ct = C1 + C2;
  const int64_t total = (int64_t)B * H * W * Ct;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % Ct);
    const int64_t p = e / Ct;
    const int xx = (int)(p % W), yy = (int)((p / W) % H), n = (int)(p / ((int64_t)W * H));
    out[e] = c < C1 ? x[(((int64_t)n * h + yy / 2) * w + xx / 2) * C1 + c]
                    : skip[p * C2 + (c - C1)];
  }
}

// Adjoint of k_up_concat: dx [B][h][w][C1] = sum of the 4 children (overwrite);
// dskip += the skip channels.
__global__ void __launch_bounds__(256) k_up_concat_bwd(const float* __restrict__ dout, int B, int h,
                                                       int w, int C1, int C2,
                                                       float* __restrict__ dx,
                                                       float* __restrict__ dskip) {
  const int H = 2 * h, W = 2 * w, Ct = C1 + C2;
  const int64_t n1 = (int64_t)B * h * w * C1, n2 = (int64_t)B * H * W * C2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n1 + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n1) {
      const int c = (int)(e % C1);
      const int64_t p = e / C1;
      const int xx = (int)(p % w), yy = (int)((p / w) % h), n = (int)(p / ((int64_t)w * h));
      const int64_t b = (((int64_t)n * H + 2 * yy) * W + 2 * xx) * Ct + c;
      dx[e] = dout[b] + dout[b + Ct] + dout[b + (int64_t)W * Ct] + dout[b + (int64_t)W * Ct + Ct];
    } else {
      const int64_t f = e - n1;
      const int c = (int)(f % C2);
      const int64_t p = f / C2;
      dskip[f] += dout[p * Ct + C1 + c];
    }
  }
}

// 1x1 output head in FP32: y[m] = sum_c a[m][c] w[c] + b.
__global__ void __launch_bounds__(256) k_head_fwd(const float* __restrict__ a, int64_t M, int C,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ b,
                                                  float* __restrict__ y) {
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M;
       m += (int64_t)gridDim.x * blockDim.x) {
    float s = b[0];
    for (int c = 0; c < C; ++c) s = fmaf(a[m * C + c], w[c], s);
    y[m] = s;
  }
}

// Head backward: da[m][c] = dy[m] w[c].
__global__ void __launch_bounds__(256) k_head_bwd_data(const float* __restrict__ dy, int64_t M,
                                                       int C, const float* __restrict__ w,
                                                       float* __restrict__ da) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M * C;
       e += (int64_t)gridDim.x * blockDim.x)
    da[e] = dy[e / C] * w[e % C];
}

// Head weight gradient: dw[c] = sum_m dy[m] a[m][c] (c < C), db = sum_m dy[m]
// (slot C); one block per output, fixed order.
__global__ void __launch_bounds__(256) k_head_bwd_w(const float* __restrict__ dy,
                                                    const float* __restrict__ a, int64_t M, int C,
                                                    float* __restrict__ dw) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t m = threadIdx.x; m < M; m += 256) s += dy[m] * (c < C ? a[m * C + c] : 1.0f);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dw[c] = red[0];
}

// Mean squared error over masked elements: per-block partial sums (fixed
// order) and the gradient dy = 2 (y - t) / count.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             int64_t n, float inv_n, float* __restrict__ dy,
                                             double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[e] - t[e];
    dy[e] = 2.0f * d * inv_n;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam with FP32 master weights (bias-corrected), then the BF16 copy used by
// the GEMMs.  bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2, __bf16* __restrict__ wb) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[e] = wi;
    wb[e] = (__bf16)wi;
  }
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* __restrict__ x, int64_t n,
                                                 __bf16* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (__bf16)x[e];
}

__global__ void __launch_bounds__(256) k_fill(float* __restrict__ x, int64_t n, float v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
}

// Surrogate output transform: psi = exp(y) * pref_k for map k (maps of
// `per_map` pixels), in double; and the training target log(psi / pref_k).
__global__ void __launch_bounds__(256) k_exp_out(const float* __restrict__ y, int64_t n,
                                                 int64_t per_map, const double* __restrict__ pref,
                                                 double* __restrict__ psi) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    psi[e] = exp((double)y[e]) * pref[e / per_map];
}

__global__ void __launch_bounds__(256) k_log_target(const double* __restrict__ psi, int64_t n,
                                                    int64_t per_map, const double* __restrict__ pref,
                                                    float* __restrict__ t) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    t[e] = (float)log(fmax(psi[e] / pref[e / per_map], 1e-300));
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

hipError_t gemm(const __bf16* A, int lda, bool ta, const __bf16* B, int ldb, bool tb, float* C,
                int ldc, int M, int N, int K, int ksplit, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  ksplit = ksplit < 1 ? 1 : ksplit;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = (kchunk + BK - 1) / BK * BK;
  ksplit = (K + kchunk - 1) / kchunk;
  if (ksplit < 1) ksplit = 1;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, ksplit);
#define DD_GEMM(TA_, TB_)                                                                      \
  hipLaunchKernelGGL((k_gemm<TA_, TB_, EPI_STORE>), grid, dim3(256), 0, st, A, lda, B, ldb, C, \
                     ldc, (float*)nullptr, (const float*)nullptr, M, N, K, kchunk)
  if (!ta && !tb) DD_GEMM(false, false);
  else if (!ta && tb) DD_GEMM(false, true);
  else if (ta && !tb) DD_GEMM(true, false);
  else DD_GEMM(true, true);
#undef DD_GEMM
  return hipGetLastError();
}

int gemm_splits(int M, int K, int ksplit) {
  ksplit = ksplit < 1 ? 1 : ksplit;
  int kchunk = (K + ksplit - 1) / ksplit;
  kchunk = (kchunk + BK - 1) / BK * BK;
  (void)M;
  return (K + kchunk - 1) / kchunk;
}

hipError_t gemm_bias_silu(const __bf16* A, int lda, const __bf16* B, int ldb, float* act, float* z,
                          int ldc, const float* bias, int M, int N, int K, hipStream_t st) {
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, 1);
  hipLaunchKernelGGL((k_gemm<false, false, EPI_BIAS_SILU>), grid, dim3(256), 0, st, A, lda, B, ldb,
                     act, ldc, z, bias, M, N, K, ((K + BK - 1) / BK) * BK);
  return hipGetLastError();
}

hipError_t sum_splits(const float* part, int splits, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(n)), dim3(256), 0, st, part, splits, n, out);
  return hipGetLastError();
}

hipError_t im2col(const float* x, int B, int H, int W, int C, __bf16* col, hipStream_t st) {
  hipLaunchKernelGGL(k_im2col, dim3(blocks_for((int64_t)B * H * W * 9 * C)), dim3(256), 0, st, x,
                     B, H, W, C, col);
  return hipGetLastError();
}

hipError_t col2im(const float* dcol, int B, int H, int W, int C, float* dx, hipStream_t st) {
  hipLaunchKernelGGL(k_col2im, dim3(blocks_for((int64_t)B * H * W * C)), dim3(256), 0, st, dcol, B,
                     H, W, C, dx);
  return hipGetLastError();
}

hipError_t silu_bwd(const float* dA, const float* Z, int64_t n, float* dZ, __bf16* dZb,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_silu_bwd, dim3(blocks_for(n)), dim3(256), 0, st, dA, Z, n, dZ, dZb);
  return hipGetLastError();
}

hipError_t colsum_add(const float* dZ, int M, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, st, dZ, M, N, db);
  return hipGetLastError();
}

hipError_t pool_fwd(const float* x, int B, int H, int W, int C, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_fwd, dim3(blocks_for((int64_t)B * H * W * C / 4)), dim3(256), 0, st, x,
                     B, H, W, C, y);
  return hipGetLastError();
}

hipError_t pool_bwd_add(const float* dy, int B, int H, int W, int C, float* dx, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for((int64_t)B * H * W * C)), dim3(256), 0, st, dy, B,
                     H, W, C, dx);
  return hipGetLastError();
}

hipError_t up_concat(const float* x, int B, int h, int w, int C1, const float* skip, int C2,
                     float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_up_concat, dim3(blocks_for((int64_t)B * 4 * h * w * (C1 + C2))), dim3(256),
                     0, st, x, B, h, w, C1, skip, C2, out);
  return hipGetLastError();
}

hipError_t up_concat_bwd(const float* dout, int B, int h, int w, int C1, int C2, float* dx,
                         float* dskip, hipStream_t st) {
  const int64_t n = (int64_t)B * h * w * C1 + (int64_t)B * 4 * h * w * C2;
  hipLaunchKernelGGL(k_up_concat_bwd, dim3(blocks_for(n)), dim3(256), 0, st, dout, B, h, w, C1, C2,
                     dx, dskip);
  return hipGetLastError();
}

hipError_t head_fwd(const float* a, int64_t M, int C, const float* w, const float* b, float* y,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_head_fwd, dim3(blocks_for(M)), dim3(256), 0, st, a, M, C, w, b, y);
  return hipGetLastError();
}

hipError_t head_bwd(const float* dy, const float* a, int64_t M, int C, const float* w, float* da,
                    float* dw, hipStream_t st) {
  hipLaunchKernelGGL(k_head_bwd_data, dim3(blocks_for(M * C)), dim3(256), 0, st, dy, M, C, w, da);
  hipLaunchKernelGGL(k_head_bwd_w, dim3(C + 1), dim3(256), 0, st, dy, a, M, C, dw);
  return hipGetLastError();
}

hipError_t mse(const float* y, const float* t, int64_t n, float* dy, double* partial, int nblocks,
               hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, st, y, t, n, 1.0f / (float)n, dy, partial);
  return hipGetLastError();
}

hipError_t adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                float eps, float bc1, float bc2, __bf16* wb, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps,
                     bc1, bc2, wb);
  return hipGetLastError();
}

hipError_t to_bf16(const float* x, int64_t n, __bf16* y, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t fill(float* x, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

hipError_t exp_out(const float* y, int64_t n, int64_t per_map, const double* pref, double* psi,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_exp_out, dim3(blocks_for(n)), dim3(256), 0, st, y, n, per_map, pref, psi);
  return hipGetLastError();
}

hipError_t log_target(const double* psi, int64_t n, int64_t per_map, const double* pref, float* t,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_log_target, dim3(blocks_for(n)), dim3(256), 0, st, psi, n, per_map, pref, t);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace dd
