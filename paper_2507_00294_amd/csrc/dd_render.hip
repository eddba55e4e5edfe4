// dd_render.hip -- visualisation of damage maps (dd_render_maps): psi maps
// rendered to 8-bit RGB images on the device, the counterpart of the
// paper's integrated live and offline 2-D views of the diffusion
// distribution (Sec. IV).  Any [n][h][w] array of psi values is accepted:
// the maps of dd_damage_map, the frames of dd_damage_sweep, the final maps
// of dd_batch_solve or dd_unet_predict.
//
// Per pixel, value v of map m with range [lo_m, hi_m]:
//   t = 0                         if not (v > lo_m) (also NaN, v <= 0 on a log scale)
//   t = 1                         if v >= hi_m
//   t = ln(v / lo_m) / ln(hi_m / lo_m)      (log scale)
//   t = (v - lo_m) / (hi_m - lo_m)          (linear scale)
// (evaluated as (ln v - ln lo_m) * (1 / (ln hi_m - ln lo_m)), resp. with the
// reciprocal of hi_m - lo_m, ln by ln_pos of dd_log.h)
//   colour = table[min(255, floor(256 t))]
// The table interpolates the colour-map anchors of dd.h linearly between
// anchor bins (FP64, rounded to the nearest integer).  With iso-lines, a
// pixel whose level min(L - 1, floor(L t)) differs from that of its right
// or lower neighbour in the same map is drawn white.  An automatic range
// takes hi_m = the largest finite value of map m and lo_m = max(hi_m
// 10^-decades, 2^-1022) (log) or 0 (linear); a map whose hi_m <= lo_m (no
// positive value) renders black.  A t that is not a number (a linear range
// so wide that hi - lo overflows) is taken as 0.
// HBM-bound: 8 bytes read and 3 written per pixel (the neighbours' values
// come from the same cache lines).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/dd.h"
#include "dd_log.h"
#include "dd_runtime.h"

namespace dd {
namespace {

// Colour-map anchors: (bin, r, g, b), bins 0 .. 255 increasing (the table of
// dd.h).
constexpr int kAnchors = 7;
constexpr int kAnchor[kAnchors][4] = {
    {0, 0, 0, 0},       {38, 32, 12, 96},  {90, 118, 24, 132}, {141, 200, 52, 84},
    {192, 244, 128, 32}, {230, 250, 208, 64}, {255, 255, 255, 232}};

// One table entry: the linear interpolation between the anchors around bin
// i, in FP64, rounded to the nearest integer (x >= 0, so x + 0.5 truncates
// to the rounding).
struct ColourTable {
  uint32_t rgb[256];
  constexpr ColourTable() : rgb() {
    for (int i = 0; i < 256; ++i) {
      int a = 0;
      while (a + 1 < kAnchors - 1 && kAnchor[a + 1][0] <= i) ++a;
      const int b0 = kAnchor[a][0], b1 = kAnchor[a + 1][0];
      uint32_t packed = 0;
      for (int c = 0; c < 3; ++c) {
        const double c0 = kAnchor[a][c + 1], c1 = kAnchor[a + 1][c + 1];
        const double x = c0 + (c1 - c0) * (double)(i - b0) / (double)(b1 - b0);
        packed |= (uint32_t)(int)(x + 0.5) << (8 * c);
      }
      rgb[i] = packed;
    }
  }
};
constexpr ColourTable kTable{};

struct RenderArgs {
  const double* psi;
  uint8_t* rgb;
  const double2* range;  // per map (lo, hi) of the automatic range, else null
  double lo, hi;         // explicit range
  int64_t npix, total;   // pixels per map, all pixels
  int32_t w, h;
  int32_t log_scale, levels;  // levels = 0: no iso-lines
  int32_t autor;               // k_render_map: automatic range
  ColourTable table;
};

// Largest finite value of each map (one block per map, fixed-order tree).
__global__ void __launch_bounds__(256) k_render_range(const double* __restrict__ psi, int64_t npix,
                                                      double fac, int32_t log_scale,
                                                      double2* __restrict__ range) {
  __shared__ double red[256];
  const int64_t m = blockIdx.x;
  const double* p = psi + m * npix;
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < npix; i += 256) {
    const double v = p[i];
    if (__builtin_isfinite(v) && v > mx) mx = v;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double hi = red[0];
    // a log range starts at the smallest normal double at the lowest
    const double lo = log_scale ? fmax(hi * fac, 2.2250738585072014e-308) : 0.0;
    range[m] = make_double2(lo, hi);
  }
}

// The scale of a range [lo, hi]: t = (ln v - ln lo) / (ln hi - ln lo) (log)
// or (v - lo) / (hi - lo) (linear), the quotient taken as a product with the
// reciprocal, ln from ln_pos; both kernels use these, so they agree bit for
// bit.
struct Scale {
  double lo, hi, base, inv;
  int log_scale;
};
__device__ __forceinline__ Scale make_scale(double lo, double hi, int log_scale) {
  Scale s{lo, hi, 0.0, 0.0, log_scale};
  s.base = log_scale ? ln_pos(lo) : lo;
  s.inv = 1.0 / ((log_scale ? ln_pos(hi) : hi) - s.base);
  return s;
}
__device__ __forceinline__ double scale_t(double v, const Scale& s) {
  if (!(v > s.lo)) return 0.0;
  if (v >= s.hi) return 1.0;
  const double t = ((s.log_scale ? ln_pos(v) : v) - s.base) * s.inv;
  return fmin(fmax(t, 0.0), 1.0);  // a t that is not a number (overflowed range) is 0
}
__device__ __forceinline__ int level_of(double t, int L) { return min(L - 1, (int)(t * L)); }

__global__ void __launch_bounds__(256) k_render(RenderArgs A) {
  __shared__ uint32_t tab[256];
  tab[threadIdx.x] = A.table.rgb[threadIdx.x];
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < A.total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / A.npix, q = e - m * A.npix;
    double lo = A.lo, hi = A.hi;
    if (A.range) {
      const double2 r = A.range[m];
      lo = r.x;
      hi = r.y;
    }
    uint32_t c;
    if (!(hi > lo)) {  // an automatic range over a map with no positive value
      c = tab[0];
    } else {
      const Scale sc = make_scale(lo, hi, A.log_scale);
      const double t = scale_t(A.psi[e], sc);
      c = tab[min(255, (int)(t * 256.0))];
      if (A.levels > 0) {
        const int x = (int)(q % A.w), y = (int)(q / A.w);
        const int lv = level_of(t, A.levels);
        bool edge = false;
        if (x + 1 < A.w) edge |= level_of(scale_t(A.psi[e + 1], sc), A.levels) != lv;
        if (y + 1 < A.h)
          edge |= level_of(scale_t(A.psi[e + A.w], sc), A.levels) != lv;
        if (edge) c = 0xFFFFFFu;
      }
    }
    uint8_t* o = A.rgb + 3 * e;
    o[0] = (uint8_t)(c & 0xFF);
    o[1] = (uint8_t)((c >> 8) & 0xFF);
    o[2] = (uint8_t)((c >> 16) & 0xFF);
  }
}

// Maps of at most kMapPixMax pixels, a multiple of 4, into a 4-byte aligned
// image: one block per map.  The automatic range (the same reduction as
// k_render_range), then each pixel's colour bin (kept in registers by the
// thread that colours it) and level (into LDS, for the neighbours), so that
// every pixel takes one logarithm (k_render takes three with iso-lines),
// then the colours, four pixels (12 bytes) per thread and step as three
// 4-byte stores.  The host sends here only psi arrays that start 16-byte
// aligned; a map holds a multiple of four values, so four pixels load as two
// 16-byte vectors.  Per pixel the arithmetic is k_render's, so both give the
// same image.  The iso-line test reads the neighbours' levels at clamped
// indices and selects: a short-circuit form of it compiled to code whose
// vertical comparison did not take effect.
constexpr int kMapPixMax = 16384;
constexpr int kMapSteps = kMapPixMax / (4 * 256);  // groups of four pixels per thread

__global__ void __launch_bounds__(256) k_render_map(RenderArgs A, double fac) {
  __shared__ uint32_t tab[256];
  __shared__ double red[256];
  __shared__ uint8_t s_lev[kMapPixMax];
  const int tid = threadIdx.x;
  const int npix = (int)A.npix, w = A.w, L = A.levels;
  const int64_t m = blockIdx.x;
  const double* p = A.psi + m * A.npix;
  tab[tid] = A.table.rgb[tid];
  double lo = A.lo, hi = A.hi;
  if (A.autor) {
    double mx = 0.0;
    for (int i = tid; i < npix; i += 256) {
      const double v = p[i];
      if (__builtin_isfinite(v) && v > mx) mx = v;
    }
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
      __syncthreads();
    }
    hi = red[0];
    lo = A.log_scale ? fmax(hi * fac, 2.2250738585072014e-308) : 0.0;
  }
  const bool blank = !(hi > lo);
  // the thread's pixels 4 g .. 4 g + 3, g = tid + 256 j: colour bins packed
  // four to a register, levels into LDS for the neighbours' tests
  uint32_t bins[kMapSteps];
  const Scale sc = make_scale(lo, hi, A.log_scale);
#pragma unroll
  for (int j = 0; j < kMapSteps; ++j) {
    const int g = tid + 256 * j;
    bins[j] = 0;
    if (blank || 4 * g >= npix) continue;
    const double2 v01 = *reinterpret_cast<const double2*>(p + 4 * g);
    const double2 v23 = *reinterpret_cast<const double2*>(p + 4 * g + 2);
    const double v[4] = {v01.x, v01.y, v23.x, v23.y};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double t = scale_t(v[k], sc);
      bins[j] |= (uint32_t)min(255, (int)(t * 256.0)) << (8 * k);
      if (L > 0) s_lev[4 * g + k] = (uint8_t)level_of(t, L);
    }
  }
  __syncthreads();
  uint32_t* out = reinterpret_cast<uint32_t*>(A.rgb + 3 * (m * A.npix));
#pragma unroll
  for (int j = 0; j < kMapSteps; ++j) {
    const int g = tid + 256 * j;
    if (4 * g >= npix) continue;
    uint32_t c[4];
    // coordinates of the group's first pixel, then stepped pixel by pixel
    int y = (4 * g) / w, x = 4 * g - y * w;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = 4 * g + k;
      c[k] = tab[blank ? 0 : (bins[j] >> (8 * k)) & 0xFFu];
      if (!blank && L > 0) {
        // neighbours read at clamped (in-range) indices, then selected
        const int lv = s_lev[i];
        const int lr = s_lev[min(i + 1, npix - 1)], ld = s_lev[min(i + w, npix - 1)];
        const int er = (x + 1 < w) ? (lr ^ lv) : 0;
        const int ed = (y + 1 < A.h) ? (ld ^ lv) : 0;
        c[k] = (er | ed) ? 0xFFFFFFu : c[k];
      }
      if (++x == w) {
        x = 0;
        ++y;
      }
    }
    // bytes r0 g0 b0 r1 | g1 b1 r2 g2 | b2 r3 g3 b3 (little endian)
    out[3 * g + 0] = (c[0] & 0xFFFFFFu) | (c[1] << 24);
    out[3 * g + 1] = ((c[1] >> 8) & 0xFFFFu) | ((c[2] & 0xFFFFu) << 16);
    out[3 * g + 2] = ((c[2] >> 16) & 0xFFu) | ((c[3] & 0xFFFFFFu) << 8);
  }
}

// Per-thread device buffer of the automatic ranges.
thread_local DevBuf g_range_buf;

}  // namespace
}  // namespace dd

using namespace dd;

dd_status dd_render_maps(const double* psi, int64_t n, int32_t w, int32_t h,
                         const dd_render_opts* opt, uint8_t* rgb, void* hip_stream) {
  if (!opt) return fail(DD_EINVAL, "NULL options");
  if (n < 0 || w < 1 || h < 1) return fail(DD_EINVAL, "need n >= 0 maps of w, h >= 1 pixels");
  if ((int64_t)w * h > (1LL << 40) / std::max<int64_t>(n, 1))
    return fail(DD_EINVAL, "too many pixels");
  if (n > 0 && (!psi || !rgb)) return fail(DD_EINVAL, "NULL array");
  if (opt->log_scale != 0 && opt->log_scale != 1) return fail(DD_EINVAL, "log_scale must be 0 or 1");
  if (opt->levels < 0 || opt->levels > 256) return fail(DD_EINVAL, "levels must be in [0, 256]");
  const bool autor = opt->lo == 0.0 && opt->hi == 0.0;
  if (autor) {
    if (opt->log_scale && !(std::isfinite(opt->decades) && opt->decades > 0 && opt->decades <= 300))
      return fail(DD_EINVAL, "decades must be in (0, 300]");
  } else {
    if (!(std::isfinite(opt->lo) && std::isfinite(opt->hi) && opt->hi > opt->lo))
      return fail(DD_EINVAL, "need finite lo < hi (or lo = hi = 0 for an automatic range)");
    if (opt->log_scale && !(opt->lo > 0)) return fail(DD_EINVAL, "a log scale needs lo > 0");
  }
  dd_status rc = ensure_device();
  if (rc != DD_OK) return rc;
  if (n == 0) return DD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t npix = (int64_t)w * h, total = npix * n;
  RenderArgs A{};
  A.psi = psi;
  A.rgb = rgb;
  A.lo = opt->lo;
  A.hi = opt->hi;
  A.npix = npix;
  A.total = total;
  A.w = w;
  A.h = h;
  A.log_scale = opt->log_scale;
  A.levels = opt->levels;
  A.table = kTable;
  if (npix <= kMapPixMax && npix % 4 == 0 && n <= 0x7fffffff &&
      reinterpret_cast<uintptr_t>(rgb) % 4 == 0 && reinterpret_cast<uintptr_t>(psi) % 16 == 0) {
    A.autor = autor ? 1 : 0;
    const double fac = autor ? std::pow(10.0, -opt->decades) : 0.0;
    hipLaunchKernelGGL(k_render_map, dim3((unsigned)n), dim3(256), 0, st, A, fac);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "render kernel launch");
    return DD_OK;
  }
  if (autor) {
    hipError_t e = g_range_buf.ensure(sizeof(double2) * (size_t)n);
    if (e != hipSuccess) return hip_fail(e, "device allocation");
    const double fac = std::pow(10.0, -opt->decades);
    if (n > 0x7fffffff) return fail(DD_EINVAL, "too many maps");
    hipLaunchKernelGGL(k_render_range, dim3((unsigned)n), dim3(256), 0, st, psi, npix, fac,
                       opt->log_scale, g_range_buf.as<double2>());
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "range kernel launch");
    A.range = g_range_buf.as<double2>();
  }
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_render, dim3(blocks), dim3(256), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "render kernel launch");
  return DD_OK;
}
