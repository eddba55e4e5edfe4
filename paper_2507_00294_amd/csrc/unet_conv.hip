// unet_conv.hip -- implicit-GEMM 3x3 convolution on BF16 MFMA for gfx950.
//
// out[m][n] = sum_k A[m][k] Wt[n][k] (+ bias, SiLU), with m a pixel of an
// NHWC activation (B images of side x side), n an output channel and
// k = tap * ci + c, tap = 3 ky + kx, the input pixel (y + ky - 1, x + kx - 1)
// (zero outside the image).  A is never materialised: each K step of 32 is
// one tap and 32 consecutive input channels, read straight from the FP32
// activation (one 16-byte load per 4 channels), rounded to BF16 and staged in
// LDS.  With TAPS = 1 the input is a plain BF16 row-major matrix [M][ci] (the
// first layer, whose 5-channel im2col is padded to 64 columns).
//
// Block: 256 threads = 4 waves, block tile 256 pixels x BN channels; wave w
// owns rows 64 w .. 64 w + 63 = 4 x (BN / 16) tiles of
// v_mfma_f32_16x16x32_bf16.  Fragment layout of that instruction (lane l):
// A row l % 16, k = 8 (l / 16) .. +7; B column l % 16, same k; D element v at
// row 4 (l / 16) + v, column l % 16.  LDS rows are padded to 40 BF16 (80 B) so
// that the 16-byte fragment reads of 16 consecutive rows hit distinct banks.
// The next K step's global loads are issued before the current step's MFMAs.
//
// The same kernel computes the data gradient of a convolution: dX = conv3(dZ)
// with the taps mirrored and the weights rearranged to [ci][tap' co + j].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "unet_kernels.h"

namespace dd {
namespace nn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CBM = 256, CLDK = 40;
// Widest channel tile: 128 needs 270 registers per lane (1 wave per SIMD), 64
// leaves room for 3.
constexpr int kMaxBN = 64;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

template <typename TIn>
struct AQuad;
template <>
struct AQuad<float> {
  typedef f32x4 T;
  static __device__ __forceinline__ T zero() { return f32x4{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ bf16x4 cvt(T v) {
    return bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
  }
};
template <>
struct AQuad<__bf16> {
  typedef bf16x4 T;
  static __device__ __forceinline__ T zero() {
    return bf16x4{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
  }
  static __device__ __forceinline__ bf16x4 cvt(T v) { return v; }
};

// EPI 0: out = acc.  EPI 1: z = acc + bias; out = SiLU(z); z stored if zout.
template <typename TIn, int TAPS, int BN, int EPI>
__global__ void __launch_bounds__(256) k_conv(const TIn* __restrict__ x, int M, int lg, int ci,
                                              const __bf16* __restrict__ wt,
                                              const float* __restrict__ bias,
                                              float* __restrict__ out, float* __restrict__ zout,
                                              int N) {
  typedef typename AQuad<TIn>::T Q;
  __shared__ __attribute__((aligned(16))) __bf16 As[CBM][CLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][CLDK];
  constexpr int NB = BN / 16;
  constexpr int BLOADS = BN * 4;  // 16-byte pieces of the B tile
  constexpr int BPT = (BLOADS + 255) / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * CBM, n0 = blockIdx.y * BN;
  const int side = 1 << lg, K = TAPS * ci, cchunks = ci >> 5, nsteps = TAPS * cchunks;
  const int q = tid & 7, r0 = tid >> 3;

  Q areg[8];
  bf16x8 breg[BPT];
  auto load = [&](int s) {
    const int tap = s / cchunks, cc = s - tap * cchunks;
    const int dy = TAPS == 9 ? tap / 3 - 1 : 0, dx = TAPS == 9 ? tap % 3 - 1 : 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int m = m0 + r0 + 32 * p;
      bool ok = m < M;
      if (TAPS == 9) {
        const int yy = ((m >> lg) & (side - 1)) + dy, xx = (m & (side - 1)) + dx;
        ok = ok && yy >= 0 && yy < side && xx >= 0 && xx < side;
      }
      areg[p] = AQuad<TIn>::zero();
      if (ok)
        areg[p] = *reinterpret_cast<const Q*>(x + (int64_t)(m + dy * side + dx) * ci + cc * 32 +
                                              4 * q);
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int idx = tid + 256 * e;
      if (idx < BLOADS) {
        const int j = idx >> 2, part = idx & 3;
        breg[e] = *reinterpret_cast<const bf16x8*>(wt + (int64_t)(n0 + j) * K + s * 32 + part * 8);
      }
    }
  };

  f32x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  load(0);
  for (int s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int p = 0; p < 8; ++p)
      *reinterpret_cast<bf16x4*>(&As[r0 + 32 * p][4 * q]) = AQuad<TIn>::cvt(areg[p]);
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int idx = tid + 256 * e;
      if (idx < BLOADS) *reinterpret_cast<bf16x8*>(&Bs[idx >> 2][(idx & 3) * 8]) = breg[e];
    }
    __syncthreads();
    if (s + 1 < nsteps) load(s + 1);
    bf16x8 af[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      af[a] = *reinterpret_cast<const bf16x8*>(&As[wave * 64 + a * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&Bs[b * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr, acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int col = n0 + b * 16 + (lane & 15);
      const float bs = EPI == 1 ? bias[col] : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wave * 64 + a * 16 + 4 * (lane >> 4) + v;
        if (row < M) {
          const int64_t o = (int64_t)row * N + col;
          if (EPI == 1) {
            const float z = acc[a][b][v] + bs;
            if (zout) zout[o] = z;
            out[o] = silu(z);
          } else {
            out[o] = acc[a][b][v];
          }
        }
      }
    }
}

template <typename TIn, int TAPS, int EPI>
hipError_t launch(const TIn* x, int M, int lg, int ci, const __bf16* wt, const float* bias,
                  float* out, float* z, int N, hipStream_t st) {
  const int bn = (kMaxBN >= 128 && N % 128 == 0) ? 128 : (N % 64 == 0) ? 64 : 32;
  dim3 grid((M + CBM - 1) / CBM, N / bn);
  if (bn == 128)
    hipLaunchKernelGGL((k_conv<TIn, TAPS, 128, EPI>), grid, dim3(256), 0, st, x, M, lg, ci, wt,
                       bias, out, z, N);
  else if (bn == 64)
    hipLaunchKernelGGL((k_conv<TIn, TAPS, 64, EPI>), grid, dim3(256), 0, st, x, M, lg, ci, wt,
                       bias, out, z, N);
  else
    hipLaunchKernelGGL((k_conv<TIn, TAPS, 32, EPI>), grid, dim3(256), 0, st, x, M, lg, ci, wt,
                       bias, out, z, N);
  return hipGetLastError();
}

bool shape_ok(int M, int ci, int N) { return M > 0 && ci > 0 && ci % 32 == 0 && N > 0 && N % 32 == 0; }

}  // namespace

hipError_t conv3_silu(const float* x, int B, int lg, int ci, const __bf16* wt, const float* bias,
                      float* act, float* z, int co, hipStream_t st) {
  const int M = B << (2 * lg);
  if (!shape_ok(M, ci, co)) return hipErrorInvalidValue;
  return launch<float, 9, 1>(x, M, lg, ci, wt, bias, act, z, co, st);
}

hipError_t conv3_plain(const float* x, int B, int lg, int ci, const __bf16* wt, float* out, int co,
                       hipStream_t st) {
  const int M = B << (2 * lg);
  if (!shape_ok(M, ci, co)) return hipErrorInvalidValue;
  return launch<float, 9, 0>(x, M, lg, ci, wt, nullptr, out, nullptr, co, st);
}

hipError_t rows_silu(const __bf16* a, int M, int k, const __bf16* wt, const float* bias, float* act,
                     float* z, int co, hipStream_t st) {
  if (!shape_ok(M, k, co)) return hipErrorInvalidValue;
  return launch<__bf16, 1, 1>(a, M, 0, k, wt, bias, act, z, co, st);
}

}  // namespace nn
}  // namespace dd
