// unet_conv.hip -- 3x3 convolutions of the surrogate on BF16 MFMA for gfx950.
//
// out[m][n] = sum_k A[m][k] Wt[n][k] (+ bias, SiLU), with m a pixel of an
// NHWC activation (B images of side x side, side = 2^lg), n an output channel
// and k = tap ci + c, tap = 3 ky + kx, reading input pixel (y + ky - 1,
// x + kx - 1) (zero outside the image).  A is never materialised.
//
// k_conv_halo (ci a multiple of 32): a block computes 256 consecutive output
// pixels -- 256 / side whole rows of one image, or 4 whole 8x8 images -- for
// BN output channels.  For each chunk of 32 input channels it stages the
// tile's input pixels plus a one-pixel halo (at most 400 pixels) in LDS as
// BF16, once, and all nine taps then read their A fragments from that tile
// (the nine-fold reuse of every input value stays on chip).  With BN = 64 the
// chunk's weights (9 taps x BN columns x 32, from [N][9 ci]) are staged in LDS
// once per block beside it, so the four waves share them; with BN = 32 each
// wave reads its weight fragments from L2 one tap ahead, which keeps the LDS
// footprint (and so the occupancy) of the 64^2 layers low.  Input modes: a plain activation, or the decoder's virtual
// concatenation [nearest-2x-upsampled coarse map, skip map] read directly
// from its two sources.  Epilogues: plain (the data gradient), bias + SiLU,
// and bias + SiLU followed by the 32 -> 1 output head reduced across lanes.
// Activations are stored in BF16 (the MFMA operand precision; every consumer
// rounds its input to BF16 anyway); pre-activations and gradients are FP32.
//
// k_conv_first (the 5-channel input layer): K = 45 padded to 64; the input
// halo tile is staged in LDS (FP32), each thread assembles its pixel's row of
// A from it (two K steps).
//
// Fragment layout of v_mfma_f32_16x16x32_bf16 (lane l): A row l % 16,
// k = 8 (l / 16) .. +7; B column l % 16, same k; D element v at row
// 4 (l / 16) + v, column l % 16.  The weights are the A operand and the
// activations the B operand, so D rows are output channels and columns
// pixels.  LDS rows hold 32 BF16 channels padded to 40
// (80 B), so 16 lanes reading 16 consecutive pixels hit distinct banks.
//
// The data gradient of a convolution is the same operation on dZ with the
// taps mirrored and the weights rearranged to [ci][tap' co + j].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "unet_kernels.h"

namespace dd {
namespace nn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CBM = 256;    // output pixels per block
constexpr int CLDK = 40;    // LDS row of the halo tile: 32 channels + 8 padding (BF16)
constexpr int CLDB = 40;    // LDS row of the staged weights
constexpr int HPMAX = 400;  // halo-tile pixels: 6 x 66, 10 x 34, 18 x 18 or 4 x 10 x 10

enum { IN_PLAIN = 0, IN_UPCAT = 1 };
enum { EPI_PLAIN = 0, EPI_SILU = 1, EPI_HEAD = 2 };

__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 v) {
  return bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
}

// Activations (inputs of IN_PLAIN / IN_UPCAT with TIn = __bf16, outputs of
// EPI_SILU / EPI_HEAD) are BF16; the data gradient reads and writes FP32.
struct ConvArgs {
  const void* x;     // IN_PLAIN: input [M][ci]; IN_UPCAT: skip map [M][ci - c1]
  const void* xc;    // IN_UPCAT: coarse map [M / 4][c1]
  int c1;            // IN_UPCAT: channels taken from the coarse map
  int M, lg, ci;     // output pixels, log2 side, input channels
  const __bf16* wt;  // [N][9 ci]
  const float* bias;
  void* out;         // [M][N]: BF16 activation (EPI_SILU, EPI_HEAD; may be NULL
                     // with EPI_HEAD) or FP32 (EPI_PLAIN)
  float* z;          // pre-activation [M][N] or NULL
  const float* hw;   // EPI_HEAD: 32 weights, then the bias
  float* y;          // EPI_HEAD: [M]
  int N;
  __bf16* pool;      // EPI_SILU: 2x2 average of the activation [M / 4][N], or NULL
};

// Epilogue of the block's accumulators.  The MFMAs take the weights as their
// first operand, so acc[a][b][v] is output channel n0 + b 16 + 4 (lane / 16)
// + v of pixel m0 + wave 64 + a 16 + lane % 16: every lane holds four
// consecutive channels of one pixel and stores them with one 8-byte (BF16)
// or 16-byte (FP32) store.
__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Tile pixel of fragment row group a of a wave: 64 consecutive pixels per
// wave, or, with COLS (64-pixel-wide images), a 16-pixel column strip of each
// of the tile's 4 rows (row a), so that the rows of a 2x2 pooling window sit
// in the same lane.
template <bool COLS>
__device__ __forceinline__ int tile_pixel(int wave, int a, int lane) {
  return COLS ? a * 64 + wave * 16 + (lane & 15) : wave * 64 + a * 16 + (lane & 15);
}

template <int NB, int EPI, bool COLS = false, int LG = 0>
__device__ __forceinline__ void epilogue(const ConvArgs& p, f32x4 (&acc)[4][NB], int m0, int n0,
                                         int wave, int lane) {
  const int c4 = 4 * (lane >> 4);
  if (EPI == EPI_HEAD) {
    // N = 32 = BN: this lane holds channels c4..c4+3 and 16+c4..16+c4+3 of its
    // pixel; SiLU, weight, then the sum over the pixel's four lanes.
    f32x4 w[2], bb[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      w[b] = *reinterpret_cast<const f32x4*>(p.hw + 16 * b + c4);
      bb[b] = *reinterpret_cast<const f32x4*>(p.bias + 16 * b + c4);
    }
    const float hb = p.hw[32];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int row = m0 + tile_pixel<COLS>(wave, a, lane);
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        f32x4 z, act;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          z[v] = acc[a][b][v] + bb[b][v];
          act[v] = silu(z[v]);
          s = __builtin_fmaf(act[v], w[b][v], s);
        }
        if (row < p.M) {
          const int64_t o = (int64_t)row * 32 + 16 * b + c4;
          if (p.out) *reinterpret_cast<bf16x4*>(static_cast<__bf16*>(p.out) + o) = to_bf16x4(act);
          if (p.z) *reinterpret_cast<f32x4*>(p.z + o) = z;
        }
      }
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      if (c4 == 0 && row < p.M) p.y[row] = s + hb;
    }
    return;
  }
  f32x4 bs[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
    bs[b] = EPI == EPI_SILU ? *reinterpret_cast<const f32x4*>(p.bias + n0 + 16 * b + c4)
                            : f32x4{0.f, 0.f, 0.f, 0.f};
  if (EPI == EPI_SILU && LG >= 4 && p.pool) {
    // Activation and its 2x2 average.  Vertical window partners are
    // fragment groups a and a ^ VA of the same lane, horizontal ones lanes
    // l and l ^ 1; the sum runs in the order of the separate pooling kernel
    // (top-left, top-right, bottom-left, bottom-right) over the BF16 values.
    // Every M here is a multiple of the 256-pixel tile.
    static_assert(LG != 6 || COLS, "64-wide tiles pool from column strips");
    constexpr int VA = LG == 5 ? 2 : 1;
    constexpr int W = 1 << LG, Wo = W / 2;
    bf16x4 act[4][NB];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int row = m0 + tile_pixel<COLS>(wave, a, lane);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int64_t o = (int64_t)row * p.N + n0 + 16 * b + c4;
        const f32x4 z = acc[a][b] + bs[b];
        if (p.z) *reinterpret_cast<f32x4*>(p.z + o) = z;
        act[a][b] = to_bf16x4(f32x4{silu(z[0]), silu(z[1]), silu(z[2]), silu(z[3])});
        *reinterpret_cast<bf16x4*>(static_cast<__bf16*>(p.out) + o) = act[a][b];
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a & VA) continue;
      const int row = m0 + tile_pixel<COLS>(wave, a, lane);  // even image row and column
      const int img = row >> (2 * LG), yy = (row >> LG) & (W - 1), xx = row & (W - 1);
      const int64_t po = ((int64_t)img * Wo + (yy >> 1)) * Wo + (xx >> 1);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        f32x4 sum;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float tl = (float)act[a][b][v], bl = (float)act[a ^ VA][b][v];
          const float tr = __shfl_xor(tl, 1), br = __shfl_xor(bl, 1);
          sum[v] = 0.25f * (((tl + tr) + bl) + br);
        }
        if ((lane & 1) == 0)
          *reinterpret_cast<bf16x4*>(p.pool + po * p.N + n0 + 16 * b + c4) = to_bf16x4(sum);
      }
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = m0 + tile_pixel<COLS>(wave, a, lane);
    if (row >= p.M) continue;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t o = (int64_t)row * p.N + n0 + 16 * b + c4;
      if (EPI == EPI_SILU) {
        const f32x4 z = acc[a][b] + bs[b];
        if (p.z) *reinterpret_cast<f32x4*>(p.z + o) = z;
        const f32x4 act{silu(z[0]), silu(z[1]), silu(z[2]), silu(z[3])};
        *reinterpret_cast<bf16x4*>(static_cast<__bf16*>(p.out) + o) = to_bf16x4(act);
      } else {
        *reinterpret_cast<f32x4*>(static_cast<float*>(p.out) + o) = acc[a][b];
      }
    }
  }
}

// Input element type as a template integer (kernel names in traces then
// demangle plainly): TIN_BF16 for activations, TIN_F32 for gradients.
enum { TIN_BF16 = 0, TIN_F32 = 1 };
template <int TIN>
using InType = typename std::conditional<TIN == TIN_BF16, __bf16, float>::type;

template <int TIN, int IN, int BN, int EPI, int LG>
__global__ void __launch_bounds__(256) k_conv_halo(ConvArgs p) {
  using TIn = InType<TIN>;
  // weights staged in LDS for BN = 64; for BN = 32 (the one-chunk layers at
  // 64^2, which depend on occupancy) each wave reads them from L2, one tap ahead
  constexpr bool BLDS = BN >= 64;
  __shared__ __attribute__((aligned(16))) __bf16 As[HPMAX][CLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BLDS ? 9 : 1][BLDS ? BN : 1][CLDB];
  constexpr int NB = BN / 16;
  constexpr int BPIECES = 9 * BN * 4;  // 16-byte pieces of the chunk's weights
  constexpr int BSLOTS = (BPIECES + 255) / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * CBM, n0 = blockIdx.y * BN;
  // the image side is a template parameter, so that the tile geometry below
  // is constant and its divisions are multiplications
  constexpr int lg = LG, W = 1 << lg;
  const int ci = p.ci, K = 9 * ci;
  // tile geometry: G image slices of R rows x W columns, halo (R+2) x (W+2)
  constexpr int lgR = lg >= 4 ? 8 - lg : lg;  // rows per slice: 256 / W, or W for W = 8
  constexpr int R = 1 << lgR, lgRW = lgR + lg;
  constexpr int HW2 = W + 2, slice = (R + 2) * HW2;
  constexpr int G = CBM >> lgRW, HP = G * slice;
  const int img0 = m0 >> (2 * lg), y0 = (m0 >> lg) & (W - 1);
  // staging: 16-byte slots of CPQ channels, QPP slots per pixel and chunk
  constexpr int CPQ = 16 / (int)sizeof(TIn), LGQ = CPQ == 8 ? 2 : 3, QPP = 1 << LGQ;
  constexpr int NSLOT = (HPMAX * QPP + 255) / 256;
  const TIn* xin = static_cast<const TIn*>(p.x);
  const TIn* xco = static_cast<const TIn*>(p.xc);

  // source pixel of every staging slot (fixed over the channel chunks)
  int src[NSLOT];
#pragma unroll
  for (int i = 0; i < NSLOT; ++i) {
    const int idx = tid + 256 * i, px = idx >> LGQ;
    int s = -1;
    if (px < HP) {
      const int g = px / slice, rem = px - g * slice;
      const int hr = rem / HW2, hc = rem - hr * HW2;
      const int yy = y0 + hr - 1, xx = hc - 1;
      if (yy >= 0 && yy < W && xx >= 0 && xx < W) {
        const int m = (((img0 + g) << lg) + yy) * W + xx;
        if (m < p.M) s = m;
      }
    }
    src[i] = s;
  }
  // halo-tile pixel of each of this lane's 4 A-fragment rows at tap (0, 0)
  constexpr bool COLS = LG == 6;
  int hbase[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int o = tile_pixel<COLS>(wave, a, lane);
    const int g = o >> lgRW, r = (o >> lg) & (R - 1), x = o & (W - 1);
    hbase[a] = g * slice + r * HW2 + x;
  }

  f32x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const __bf16* wlane = p.wt + (int64_t)(n0 + (lane & 15)) * K + 8 * (lane >> 4);
  const int chunks = ci >> 5;
  // Staging registers of one chunk: the weights (BN = 64) and the halo tile.
  // With BF16 activations and BN = 64 the next chunk's loads are issued before the
  // current chunk's MFMAs and stored to LDS after them (register prefetch);
  // the FP32 input of the data gradient is loaded and stored in one step.
  constexpr bool PIPE = CPQ == 8 && BLDS;
  using AReg = typename std::conditional<CPQ == 8, bf16x8, f32x4>::type;
  AReg ar[NSLOT];
  bf16x8 br[BLDS ? BSLOTS : 1];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int i = 0; i < BSLOTS; ++i) {
      const int piece = tid + 256 * i;
      if (BLDS && piece < BPIECES) {
        const int tap = piece / (BN * 4), rem = piece - tap * (BN * 4);
        const int n = rem >> 2, part = rem & 3;
        br[BLDS ? i : 0] = *reinterpret_cast<const bf16x8*>(p.wt + (int64_t)(n0 + n) * K +
                                                            tap * ci + cc * 32 + part * 8);
      }
    }
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) {
      const int idx = tid + 256 * i, px = idx >> LGQ, q = idx & (QPP - 1);
      ar[i] = AReg{};
      const int s = src[i];
      if (px < HP && s >= 0) {
        const TIn* from;
        if (IN == IN_UPCAT && cc * 32 < p.c1) {
          const int im = s >> (2 * lg), yy = (s >> lg) & (W - 1), xx = s & (W - 1);
          const int sc = (((im << (lg - 1)) + (yy >> 1)) << (lg - 1)) + (xx >> 1);
          from = xco + (int64_t)sc * p.c1 + cc * 32 + CPQ * q;
        } else if (IN == IN_UPCAT) {
          from = xin + (int64_t)s * (ci - p.c1) + (cc * 32 - p.c1) + CPQ * q;
        } else {
          from = xin + (int64_t)s * ci + cc * 32 + CPQ * q;
        }
        ar[i] = *reinterpret_cast<const AReg*>(from);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < BSLOTS; ++i) {
      const int piece = tid + 256 * i;
      if (BLDS && piece < BPIECES) {
        const int tap = piece / (BN * 4), rem = piece - tap * (BN * 4);
        *reinterpret_cast<bf16x8*>(&Bs[BLDS ? tap : 0][BLDS ? rem >> 2 : 0][(rem & 3) * 8]) =
            br[BLDS ? i : 0];
      }
    }
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) {
      const int idx = tid + 256 * i, px = idx >> LGQ, q = idx & (QPP - 1);
      if (px < HP) {
        if constexpr (CPQ == 8)
          *reinterpret_cast<bf16x8*>(&As[px][8 * q]) = ar[i];
        else
          *reinterpret_cast<bf16x4*>(&As[px][4 * q]) = to_bf16x4(ar[i]);
      }
    }
  };
  if (PIPE) fetch(0);
  for (int cc = 0; cc < chunks; ++cc) {
    if (!PIPE) fetch(cc);
    store();
    bf16x8 bcur[NB];
    if (!BLDS) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        bcur[b] = *reinterpret_cast<const bf16x8*>(wlane + (int64_t)b * 16 * K + cc * 32);
    }
    __syncthreads();
    if (PIPE && cc + 1 < chunks) fetch(cc + 1);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int toff = (tap / 3) * HW2 + (tap % 3);
      bf16x8 bnext[NB];
      if (!BLDS && tap < 8) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bnext[b] = *reinterpret_cast<const bf16x8*>(wlane + (int64_t)b * 16 * K + (tap + 1) * ci +
                                                      cc * 32);
      }
      bf16x8 af[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        af[a] = *reinterpret_cast<const bf16x8*>(&As[hbase[a] + toff][8 * (lane >> 4)]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const bf16x8 bf =
            BLDS ? *reinterpret_cast<const bf16x8*>(
                       &Bs[BLDS ? tap : 0][BLDS ? b * 16 + (lane & 15) : 0][8 * (lane >> 4)])
                 : bcur[b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf, af[a], acc[a][b], 0, 0, 0);
      }
      if (!BLDS && tap < 8) {
#pragma unroll
        for (int b = 0; b < NB; ++b) bcur[b] = bnext[b];
      }
    }
    __syncthreads();
  }
  epilogue<NB, EPI, COLS, LG>(p, acc, m0, n0, wave, lane);
}

// First layer: CI (< 32) input channels, K = 9 CI <= 64 padded to 64; N = 32.
// The tile's input pixels plus a one-pixel halo (the geometry of
// k_conv_halo) are staged in LDS as FP32 with coalesced loads; each thread
// then assembles its pixel's 9 CI values (indices fixed at compile time) and
// writes its BF16 row of A with 16-byte stores.
template <int CI, int EPI>
__global__ void __launch_bounds__(256) k_conv_first(ConvArgs p) {
  static_assert(9 * CI <= 64, "first layer: 9 CI must fit in 64 columns");
  __shared__ float Xs[HPMAX][CI];
  __shared__ __attribute__((aligned(16))) __bf16 As[CBM][72];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[32][72];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * CBM;
  const int lg = p.lg, W = 1 << lg;
  const int lgR = lg >= 4 ? 8 - lg : lg, R = 1 << lgR, lgRW = lgR + lg;
  const int HW2 = W + 2, slice = (R + 2) * HW2, HP = (CBM >> lgRW) * slice;
  const int img0 = m0 >> (2 * lg), y0 = (m0 >> lg) & (W - 1);
  const float* x = static_cast<const float*>(p.x);
  // halo tile, one pixel per thread and pass
  for (int px = tid; px < HP; px += 256) {
    const int g = px / slice, rem = px - g * slice;
    const int hr = rem / HW2, hc = rem - hr * HW2;
    const int yy = y0 + hr - 1, xx = hc - 1;
    int m = -1;
    if (yy >= 0 && yy < W && xx >= 0 && xx < W) {
      m = (((img0 + g) << lg) + yy) * W + xx;
      if (m >= p.M) m = -1;
    }
#pragma unroll
    for (int c = 0; c < CI; ++c) Xs[px][c] = m >= 0 ? x[(int64_t)m * CI + c] : 0.f;
  }
  __syncthreads();
  // A: pixel o = tid of the tile, k = tap CI + c
  {
    const int o = tid;
    const int hb = (o >> lgRW) * slice + ((o >> lg) & (R - 1)) * HW2 + (o & (W - 1));
    float v[64];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int h = hb + (tap / 3) * HW2 + (tap % 3);
#pragma unroll
      for (int c = 0; c < CI; ++c) v[tap * CI + c] = Xs[h][c];
    }
#pragma unroll
    for (int k = 9 * CI; k < 64; ++k) v[k] = 0.f;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      bf16x8 b;
#pragma unroll
      for (int e = 0; e < 8; ++e) b[e] = (__bf16)v[8 * g + e];
      *reinterpret_cast<bf16x8*>(&As[tid][8 * g]) = b;
    }
  }
  // B: wt [32][64]
  {
    const int j = tid >> 3, part = tid & 7;
    *reinterpret_cast<bf16x8*>(&Bs[j][part * 8]) =
        *reinterpret_cast<const bf16x8*>(p.wt + (int64_t)j * 64 + part * 8);
  }
  __syncthreads();
  f32x4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    bf16x8 af[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      af[a] = *reinterpret_cast<const bf16x8*>(
          &As[wave * 64 + a * 16 + (lane & 15)][ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const bf16x8 bfr =
          *reinterpret_cast<const bf16x8*>(&Bs[b * 16 + (lane & 15)][ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr, af[a], acc[a][b], 0, 0, 0);
    }
  }
  epilogue<2, EPI>(p, acc, m0, 0, wave, lane);
}

template <int TIN, int IN, int BN, int EPI>
void launch_halo_bn(const ConvArgs& p, dim3 grid, hipStream_t st) {
  switch (p.lg) {
    case 3: hipLaunchKernelGGL((k_conv_halo<TIN, IN, BN, EPI, 3>), grid, dim3(256), 0, st, p); break;
    case 4: hipLaunchKernelGGL((k_conv_halo<TIN, IN, BN, EPI, 4>), grid, dim3(256), 0, st, p); break;
    case 5: hipLaunchKernelGGL((k_conv_halo<TIN, IN, BN, EPI, 5>), grid, dim3(256), 0, st, p); break;
    default: hipLaunchKernelGGL((k_conv_halo<TIN, IN, BN, EPI, 6>), grid, dim3(256), 0, st, p); break;
  }
}

// Callers have checked 3 <= lg <= 6 (halo_ok).
template <int TIN, int IN, int EPI>
hipError_t launch_halo(const ConvArgs& p, hipStream_t st) {
  const int bn = (EPI == EPI_HEAD) ? 32 : (p.N % 64 == 0) ? 64 : 32;
  dim3 grid((p.M + CBM - 1) / CBM, p.N / bn);
  if (bn == 64)
    launch_halo_bn<TIN, IN, 64, EPI>(p, grid, st);
  else
    launch_halo_bn<TIN, IN, 32, EPI>(p, grid, st);
  return hipGetLastError();
}

bool halo_ok(int M, int lg, int ci, int N) {
  return M > 0 && lg >= 3 && lg <= 6 && ci > 0 && ci % 32 == 0 && N > 0 && N % 32 == 0;
}

}  // namespace

hipError_t conv3_silu(const __bf16* x, int B, int lg, int ci, const __bf16* wt, const float* bias,
                      __bf16* act, float* z, int co, __bf16* pool, hipStream_t st) {
  ConvArgs p{x, nullptr, 0, B << (2 * lg), lg, ci, wt, bias, act, z, nullptr, nullptr, co, pool};
  if (!halo_ok(p.M, lg, ci, co) || !act || (pool && lg < 4)) return hipErrorInvalidValue;
  return launch_halo<TIN_BF16, IN_PLAIN, EPI_SILU>(p, st);
}

hipError_t conv3_upcat_silu(const __bf16* coarse, int c1, const __bf16* skip, int c2, int B,
                            int lg, const __bf16* wt, const float* bias, __bf16* act, float* z,
                            int co, hipStream_t st) {
  ConvArgs p{skip, coarse, c1, B << (2 * lg), lg, c1 + c2, wt, bias, act, z, nullptr, nullptr, co};
  if (!halo_ok(p.M, lg, p.ci, co) || c1 % 32 != 0 || lg < 4 || !act) return hipErrorInvalidValue;
  return launch_halo<TIN_BF16, IN_UPCAT, EPI_SILU>(p, st);
}

hipError_t conv3_silu_head(const __bf16* x, int B, int lg, int ci, const __bf16* wt,
                           const float* bias, const float* head, __bf16* act, float* z, float* y,
                           hipStream_t st) {
  ConvArgs p{x, nullptr, 0, B << (2 * lg), lg, ci, wt, bias, act, z, head, y, 32};
  if (!halo_ok(p.M, lg, ci, 32) || !y || !head) return hipErrorInvalidValue;
  return launch_halo<TIN_BF16, IN_PLAIN, EPI_HEAD>(p, st);
}

hipError_t conv3_plain(const float* x, int B, int lg, int ci, const __bf16* wt, float* out, int co,
                       hipStream_t st) {
  ConvArgs p{x, nullptr, 0, B << (2 * lg), lg, ci, wt, nullptr, out, nullptr, nullptr, nullptr, co};
  if (!halo_ok(p.M, lg, ci, co) || !out) return hipErrorInvalidValue;
  return launch_halo<TIN_F32, IN_PLAIN, EPI_PLAIN>(p, st);
}

hipError_t conv3_first_silu(const float* x, int B, int lg, int ci, const __bf16* wt,
                            const float* bias, __bf16* act, float* z, hipStream_t st) {
  ConvArgs p{x, nullptr, 0, B << (2 * lg), lg, ci, wt, bias, act, z, nullptr, nullptr, 32};
  if (p.M <= 0 || lg < 3 || lg > 6 || !act) return hipErrorInvalidValue;
  const dim3 grid((p.M + CBM - 1) / CBM);
  switch (ci) {  // the input channel counts the network uses
    case 5: hipLaunchKernelGGL((k_conv_first<5, EPI_SILU>), grid, dim3(256), 0, st, p); break;
    case 3: hipLaunchKernelGGL((k_conv_first<3, EPI_SILU>), grid, dim3(256), 0, st, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nn
}  // namespace dd
