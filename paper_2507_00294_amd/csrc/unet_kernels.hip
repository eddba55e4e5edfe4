// unet_kernels.hip -- kernels of the learned surrogate other than the
// implicit-GEMM convolution (unet_conv.hip): the weight-gradient GEMM on BF16
// MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation) over im2col columns, the
// first layer's im2col, SiLU backward, bias gradients, the adjoint of the 2x2 pooling,
// nearest 2x upsampling with the skip concatenation, the FP32 1x1 head, the
// relative-L2 loss, gradient-norm clipping, Adam with FP32 master weights and
// the rearrangement of the weights into the convolution's BF16 layouts, the
// dihedral mini-batch gather of training, and the surrogate's input gather,
// output transform and spot-check.
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
// im2col for a 3x3 convolution with zero padding 1 (NHWC, FP32 -> BF16), rows
// of ld >= 9 C columns (columns past 9 C are zero):
// col[m][(ky*3+kx)*C + c] = x[n][y+ky-1][x+kx-1][c], m = (n*H + y)*W + x.
template <typename T>
__global__ void __launch_bounds__(256) k_im2col(const T* __restrict__ x, int B, int H, int W,
                                                int C, int ld, __bf16* __restrict__ col) {
  const int64_t K = 9 * (int64_t)C, total = (int64_t)B * H * W * ld;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / ld;
    const int k = (int)(e % ld);
    float v = 0.f;
    if (k < K) {
      const int tap = k / C, c = k % C;
      const int ky = tap / 3, kx = tap % 3;
      const int xx = (int)(m % W), yy = (int)((m / W) % H), n = (int)(m / ((int64_t)W * H));
      const int sy = yy + ky - 1, sx = xx + kx - 1;
      if (sy >= 0 && sy < H && sx >= 0 && sx < W)
        v = (float)x[(((int64_t)n * H + sy) * W + sx) * C + c];
    }
    col[e] = (__bf16)v;
  }
}

// im2col of the decoder input: channel c < c1 of pixel (n, y, x) is channel c
// of the coarse map at (n, y/2, x/2), channel c1 + c' is channel c' of skip;
// rows of 9 (c1 + c2) columns.
__global__ void __launch_bounds__(256) k_im2col_upcat(const __bf16* __restrict__ coarse, int c1,
                                                      const __bf16* __restrict__ skip, int c2,
                                                      int B, int H, __bf16* __restrict__ col) {
  const int C = c1 + c2, h = H / 2;
  const int64_t K = 9 * (int64_t)C, total = (int64_t)B * H * H * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / K;
    const int k = (int)(e % K);
    const int tap = k / C, c = k % C;
    const int ky = tap / 3, kx = tap % 3;
    const int xx = (int)(m % H), yy = (int)((m / H) % H), n = (int)(m / ((int64_t)H * H));
    const int sy = yy + ky - 1, sx = xx + kx - 1;
    __bf16 v = (__bf16)0.f;
    if (sy >= 0 && sy < H && sx >= 0 && sx < H)
      v = c < c1 ? coarse[(((int64_t)n * h + sy / 2) * h + sx / 2) * c1 + c]
                 : skip[(((int64_t)n * H + sy) * H + sx) * c2 + (c - c1)];
    col[e] = v;
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

// Adjoint of the 2x2 average pooling (which runs in the convolution
// epilogue) on FP32 gradients (accumulates).
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

// Adjoint of the decoder input [nearest-2x upsampling of x [B][h][w][C1],
// skip [B][2h][2w][C2]] (channel concatenation): dx = sum of the 4 children
// (overwrite); dskip += the skip channels.
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
                                                    const __bf16* __restrict__ a, int64_t M, int C,
                                                    float* __restrict__ dw) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t m = threadIdx.x; m < M; m += 256) s += dy[m] * (c < C ? (float)a[m * C + c] : 1.0f);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dw[c] = red[0];
}

// Loss of a batch of maps (one block per map of n pixels).  The prediction
// is own + exp(y) (exp argument capped at 80); map b's loss is its squared
// relative L2 error |pred - t|^2 / |t|^2, written to loss_map[b].  The
// objective whose gradient dy is returned (for the mean over maps) adds the
// anchor (anchor / n) sum_i (r_i / t_i)^2 (y_i - ln r_i)^2 with r_i = max(t_i
// - own_i, 1e-6 t_i): the same per-pixel weight as the relative error, but a
// gradient that does not vanish when exp(y) is far below r.  Sums are in
// double, in a fixed order.
__global__ void __launch_bounds__(256) k_rel_l2(const float* __restrict__ y,
                                                const float* __restrict__ own,
                                                const float* __restrict__ t, int n, float inv_maps,
                                                float anchor, float* __restrict__ dy,
                                                double* __restrict__ loss_map) {
  __shared__ double red[256];
  const int64_t base = (int64_t)blockIdx.x * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double ti = t[base + i];
    s += ti * ti;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double den = red[0] > 0.0 ? red[0] : 1.0;
  __syncthreads();
  const float scale = (float)(2.0 / den) * inv_maps;
  const float ascale = 2.0f * anchor / (float)n * inv_maps;
  double num = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float yi = y[base + i], ti = t[base + i], oi = own[base + i];
    const float e = __expf(fminf(yi, 80.0f));
    const float d = oi + e - ti;
    num += (double)d * d;
    float g = scale * d * e;
    if (ti > 0.f) {
      const float r = fmaxf(ti - oi, 1e-6f * ti), wr = r / ti;
      g += ascale * wr * wr * (yi - __logf(r));
    }
    dy[base + i] = g;
  }
  red[threadIdx.x] = num;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_map[blockIdx.x] = red[0] / den;
}

// Sum of squares of g: one partial per block (the grid has kNormBlocks blocks).
__global__ void __launch_bounds__(256) k_sumsq(const float* __restrict__ g, int64_t n,
                                               double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    s += (double)g[e] * g[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// scale_norm[0] = min(1, clip / |g|) (1 when clip <= 0, 0 when |g| is not
// finite, which skips the update); scale_norm[1] = |g|.
__global__ void __launch_bounds__(256) k_clip_scale(const double* __restrict__ partial, float clip,
                                                    float* __restrict__ scale_norm) {
  __shared__ double red[256];
  red[threadIdx.x] = partial[threadIdx.x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = sqrt(red[0]);
    double sc = 1.0;
    if (clip > 0.f && norm > clip) sc = clip / norm;
    if (!(norm <= 1e300)) sc = 0.0;
    scale_norm[0] = (float)sc;
    scale_norm[1] = (float)norm;
  }
}

// Adam with FP32 master weights (bias-corrected) on the scaled gradient
// g * scale[0].  bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              const float* __restrict__ scale, int64_t n, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2) {
  const float sc = scale[0];
  if (sc == 0.f) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e] * sc;
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// BF16 weight layouts of the convolutions from the FP32 master vector (layer
// blockIdx.y), whose weights W[k][j] (k = tap ci + c) start at w_off:
//   forward  wf[j][k], k < kpad (zero for k >= 9 ci);
//   dgrad    wd[c][t co + j] = W[(8 - t) ci + c][j] (mirrored taps).
__global__ void __launch_bounds__(256) k_prep_weights(const float* __restrict__ w, ConvTable tab,
                                                      __bf16* __restrict__ wf,
                                                      __bf16* __restrict__ wd) {
  const ConvDesc L = tab.l[blockIdx.y];
  const int64_t nf = (int64_t)L.co * L.kpad, nd = L.has_dgrad ? 9LL * L.ci * L.co : 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nf + nd;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nf) {
      const int j = (int)(e / L.kpad), k = (int)(e % L.kpad);
      wf[L.wf_off + e] = k < 9 * L.ci ? (__bf16)w[L.w_off + (int64_t)k * L.co + j] : (__bf16)0.f;
    } else {
      const int64_t f = e - nf;
      const int K2 = 9 * L.co;
      const int c = (int)(f / K2), r = (int)(f % K2);
      const int t = r / L.co, j = r % L.co;
      wd[L.wd_off + f] = (__bf16)w[L.w_off + ((int64_t)(8 - t) * L.ci + c) * L.co + j];
    }
  }
}

// Dihedral transform of a side x side map: destination pixel (i, j) reads
// source pixel T_f(i, j), f in 0..7: transpose if f & 1, then mirror rows if
// f & 2 and columns if f & 4.
__device__ __forceinline__ int dihedral_src(int i, int j, int f, int side) {
  if (f & 1) {
    const int t = i;
    i = j;
    j = t;
  }
  if (f & 2) i = side - 1 - i;
  if (f & 4) j = side - 1 - j;
  return i * side + j;
}

// Training mini-batch: map idx[b] of (x_all [cin channels], own_all, t_all;
// n_all maps) under the dihedral transform tf[b], into slot b of (xb, ob,
// tb); an index outside [0, n_all) gives a zero slot.
__global__ void __launch_bounds__(256) k_gather_batch(
    const float* __restrict__ x_all, const float* __restrict__ own_all,
    const float* __restrict__ t_all, int64_t n_all, int cin, int side,
    const int32_t* __restrict__ idx, const int32_t* __restrict__ tf, int nb,
    float* __restrict__ xb, float* __restrict__ ob, float* __restrict__ tb) {
  const int npx = side * side;
  const int64_t total = (int64_t)nb * npx;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / npx), p = (int)(e % npx);
    const int64_t m = idx[b];
    if (m < 0 || m >= n_all) {
      for (int c = 0; c < cin; ++c) xb[e * cin + c] = 0.f;
      ob[e] = 0.f;
      tb[e] = 0.f;
      continue;
    }
    const int64_t src = m * npx + dihedral_src(p / side, p % side, tf[b] & 7, side);
    for (int c = 0; c < cin; ++c) xb[e * cin + c] = x_all[src * cin + c];
    ob[e] = own_all[src];
    tb[e] = t_all[src];
  }
}

// Inference inputs of map b from its scan's cached table feat[b] (cin inputs,
// then the own-visit term, per pixel).
__global__ void __launch_bounds__(256) k_gather_features(const float* const* __restrict__ feat,
                                                         int nb, int cin, int npx,
                                                         float* __restrict__ x,
                                                         float* __restrict__ own) {
  const int64_t total = (int64_t)nb * npx;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / npx), p = (int)(e % npx);
    const float* f = feat[b] + (int64_t)p * (cin + 1);
    for (int c = 0; c < cin; ++c) x[e * cin + c] = f[c];
    own[e] = f[cin];
  }
}

// Prediction output: map b, psi = pref[b] (own + exp(y)) in double, written to
// out[b] (npx values).
__global__ void __launch_bounds__(256) k_output(const float* __restrict__ y,
                                                const float* __restrict__ own, int nb, int npx,
                                                const double* __restrict__ pref,
                                                double* const* __restrict__ out) {
  const int64_t total = (int64_t)nb * npx;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / npx), p = (int)(e % npx);
    out[b][p] = pref[b] * ((double)own[e] + exp((double)fminf(y[e], 80.0f)));
  }
}

// Training target: the dimensionless map psi / pref (float).
__global__ void __launch_bounds__(256) k_target(const double* __restrict__ psi, int64_t n,
                                                int64_t per_map, const double* __restrict__ pref,
                                                float* __restrict__ t) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    t[e] = (float)(psi[e] / pref[e / per_map]);
}

// Spot check of map b: relative L2 distance between row `row` of pred[b]
// (side x side) and the exact row exact[b side ..]; one wave per map,
// fixed-order sums.
__global__ void __launch_bounds__(64) k_spot(const double* const* __restrict__ pred,
                                             const double* __restrict__ exact, int side, int x0,
                                             int y0, int step, int w, int h,
                                             double* __restrict__ rel) {
  __shared__ double a[64], b[64];
  const int m = blockIdx.x;
  double num = 0.0, den = 0.0;
  for (int c = threadIdx.x; c < w * h; c += 64) {
    const int u = c % w, v = c / w;
    const double e = exact[(int64_t)m * w * h + c];
    const double d = pred[m][(int64_t)(y0 + step * v) * side + x0 + step * u] - e;
    num += d * d;
    den += e * e;
  }
  a[threadIdx.x] = num;
  b[threadIdx.x] = den;
  __syncthreads();
  for (int s = 32; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      a[threadIdx.x] += a[threadIdx.x + s];
      b[threadIdx.x] += b[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rel[m] = b[0] > 0 ? sqrt(a[0] / b[0]) : (a[0] > 0 ? 1.0 : 0.0);
}

__global__ void __launch_bounds__(256) k_fill(float* __restrict__ x, int64_t n, float v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
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

hipError_t sum_splits(const float* part, int splits, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(n)), dim3(256), 0, st, part, splits, n, out);
  return hipGetLastError();
}

hipError_t im2col(const float* x, int B, int H, int W, int C, int ld, __bf16* col, hipStream_t st) {
  if (ld < 9 * C) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_im2col<float>, dim3(blocks_for((int64_t)B * H * W * ld)), dim3(256), 0, st,
                     x, B, H, W, C, ld, col);
  return hipGetLastError();
}

hipError_t im2col(const __bf16* x, int B, int H, int W, int C, int ld, __bf16* col,
                  hipStream_t st) {
  if (ld < 9 * C) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_im2col<__bf16>, dim3(blocks_for((int64_t)B * H * W * ld)), dim3(256), 0, st,
                     x, B, H, W, C, ld, col);
  return hipGetLastError();
}

hipError_t im2col_upcat(const __bf16* coarse, int c1, const __bf16* skip, int c2, int B, int H,
                        __bf16* col, hipStream_t st) {
  hipLaunchKernelGGL(k_im2col_upcat, dim3(blocks_for((int64_t)B * H * H * 9 * (c1 + c2))), dim3(256),
                     0, st, coarse, c1, skip, c2, B, H, col);
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

hipError_t pool_bwd_add(const float* dy, int B, int H, int W, int C, float* dx, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for((int64_t)B * H * W * C)), dim3(256), 0, st, dy, B,
                     H, W, C, dx);
  return hipGetLastError();
}

hipError_t up_concat_bwd(const float* dout, int B, int h, int w, int C1, int C2, float* dx,
                         float* dskip, hipStream_t st) {
  const int64_t n = (int64_t)B * h * w * C1 + (int64_t)B * 4 * h * w * C2;
  hipLaunchKernelGGL(k_up_concat_bwd, dim3(blocks_for(n)), dim3(256), 0, st, dout, B, h, w, C1, C2,
                     dx, dskip);
  return hipGetLastError();
}

hipError_t head_bwd(const float* dy, const __bf16* a, int64_t M, int C, const float* w, float* da,
                    float* dw, hipStream_t st) {
  hipLaunchKernelGGL(k_head_bwd_data, dim3(blocks_for(M * C)), dim3(256), 0, st, dy, M, C, w, da);
  hipLaunchKernelGGL(k_head_bwd_w, dim3(C + 1), dim3(256), 0, st, dy, a, M, C, dw);
  return hipGetLastError();
}

hipError_t rel_l2(const float* y, const float* own, const float* t, int maps, int npx, float anchor,
                  float* dy, double* loss_map, hipStream_t st) {
  hipLaunchKernelGGL(k_rel_l2, dim3(maps), dim3(256), 0, st, y, own, t, npx, 1.0f / (float)maps,
                     anchor, dy, loss_map);
  return hipGetLastError();
}

hipError_t clip_scale(const float* g, int64_t n, float clip, double* partial, float* scale_norm,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(kNormBlocks), dim3(256), 0, st, g, n, partial);
  hipLaunchKernelGGL(k_clip_scale, dim3(1), dim3(kNormBlocks), 0, st, partial, clip, scale_norm);
  return hipGetLastError();
}

hipError_t adam(float* w, float* m, float* v, const float* g, const float* scale, int64_t n,
                float lr, float b1, float b2, float eps, float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, w, m, v, g, scale, n, lr, b1, b2,
                     eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t prep_weights(const float* w, const ConvTable& tab, __bf16* wf, __bf16* wd,
                        hipStream_t st) {
  int64_t most = 0;
  for (int l = 0; l < tab.n; ++l) {
    const ConvDesc& L = tab.l[l];
    const int64_t n = (int64_t)L.co * L.kpad + (L.has_dgrad ? 9LL * L.ci * L.co : 0);
    most = n > most ? n : most;
  }
  hipLaunchKernelGGL(k_prep_weights, dim3(blocks_for(most), tab.n), dim3(256), 0, st, w, tab, wf,
                     wd);
  return hipGetLastError();
}

hipError_t gather_batch(const float* x_all, const float* own_all, const float* t_all,
                        int64_t n_all, int cin, int side, const int32_t* idx, const int32_t* tf,
                        int nb, float* xb, float* ob, float* tb, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_batch, dim3(blocks_for((int64_t)nb * side * side)), dim3(256), 0, st,
                     x_all, own_all, t_all, n_all, cin, side, idx, tf, nb, xb, ob, tb);
  return hipGetLastError();
}

hipError_t gather_features(const float* const* feat, int nb, int cin, int npx, float* x,
                           float* own, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_features, dim3(blocks_for((int64_t)nb * npx)), dim3(256), 0, st,
                     feat, nb, cin, npx, x, own);
  return hipGetLastError();
}

hipError_t output(const float* y, const float* own, int nb, int npx, const double* pref,
                  double* const* out, hipStream_t st) {
  hipLaunchKernelGGL(k_output, dim3(blocks_for((int64_t)nb * npx)), dim3(256), 0, st, y, own, nb,
                     npx, pref, out);
  return hipGetLastError();
}

hipError_t target(const double* psi, int64_t n, int64_t per_map, const double* pref, float* t,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_target, dim3(blocks_for(n)), dim3(256), 0, st, psi, n, per_map, pref, t);
  return hipGetLastError();
}

hipError_t spot(const double* const* pred, const double* exact, int maps, int side, int x0,
                int y0, int step, int w, int h, double* rel, hipStream_t st) {
  hipLaunchKernelGGL(k_spot, dim3(maps), dim3(64), 0, st, pred, exact, side, x0, y0, step, w, h,
                     rel);
  return hipGetLastError();
}

hipError_t fill(float* x, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace dd
