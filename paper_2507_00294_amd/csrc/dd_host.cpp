// dd_host.cpp -- host runtime of libdd: the C ABI of include/dd.h.
//
// Responsibilities: argument validation, scan-order generation, device
// buffers owned by a scan handle, work planning (near band / far region,
// series-degree segments, work items in longest-first order, partial slots)
// and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "dd_internal.h"
#include "dd_kernels.h"
#include "dd_runtime.h"

namespace dd {

// ---------------------------------------------------------------------------
// Errors.
static thread_local std::string g_err;

dd_status fail(dd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

dd_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(DD_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(DD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Allocation limit for tests of the out-of-memory path (DD_ALLOC_LIMIT_BYTES,
// applied to each single host or device allocation the library makes).
static size_t alloc_limit() {
  static size_t lim = [] {
    const char* e = getenv("DD_ALLOC_LIMIT_BYTES");
    if (!e || !*e) return std::numeric_limits<size_t>::max();
    return (size_t)strtoull(e, nullptr, 10);
  }();
  return lim;
}

bool host_alloc_ok(size_t bytes) { return bytes <= alloc_limit(); }

hipError_t dev_alloc(void** p, size_t bytes) {
  if (bytes > alloc_limit()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes ? bytes : 16);
}

// ---------------------------------------------------------------------------
// Device selection: one gfx950 device, the caller's current one.
dd_status ensure_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) return fail(DD_EDEVICE, "no HIP device available");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DD_EDEVICE, "hipGetDevice failed");
  static std::mutex mu;
  static std::map<int, int> ok;  // device -> 1 gfx950, 0 other
  std::lock_guard<std::mutex> lk(mu);
  auto it = ok.find(dev);
  if (it == ok.end()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return fail(DD_EDEVICE, "hipGetDeviceProperties failed");
    ok[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    it = ok.find(dev);
  }
  if (!it->second) return fail(DD_EDEVICE, "libdd is built for gfx950 only");
  return DD_OK;
}

// Gauss-Legendre rule on [0, 1] with n nodes by Newton iteration on P_n:
// x[i] = (1 - z_i) / 2, w[i] = half the weight of z_i on [-1, 1].
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

const GLNodes& gl_nodes() {
  static GLNodes g = [] {
    GLNodes r;
    gauss_legendre01(kGL, r.x, r.w);
    return r;
  }();
  return g;
}

// ---------------------------------------------------------------------------
// Scan orders.  SplitMix64 (Steele, Lea & Flood 2014), Lemire's bounded
// integers (2019) on its top 32 bits, Fisher-Yates from the last slot.
namespace {
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  uint32_t below(uint32_t n) {  // uniform in [0, n)
    uint64_t prod = (uint64_t)(uint32_t)(next() >> 32) * n;
    if ((uint32_t)prod < n) {
      const uint32_t floor_ = (0u - n) % n;
      while ((uint32_t)prod < floor_) prod = (uint64_t)(uint32_t)(next() >> 32) * n;
    }
    return (uint32_t)(prod >> 32);
  }
};
}  // namespace

static dd_status make_visits(const dd_scan_desc& d, std::vector<int32_t>& ids) {
  const int64_t n = (int64_t)d.nx * d.ny;
  switch (d.order) {
    case DD_RASTER:
      ids.resize(n);
      for (int64_t v = 0; v < n; ++v) ids[v] = (int32_t)v;
      return DD_OK;
    case DD_INTERLEAVED: {
      ids.clear();
      ids.reserve(n);
      const int s = d.stride;
      for (int oy = 0; oy < s; ++oy)
        for (int ox = 0; ox < s; ++ox)
          for (int row = oy; row < d.ny; row += s)
            for (int col = ox; col < d.nx; col += s) ids.push_back(row * d.nx + col);
      return DD_OK;
    }
    case DD_RANDOM: {
      ids.resize(n);
      for (int64_t v = 0; v < n; ++v) ids[v] = (int32_t)v;
      SplitMix64 g{d.seed};
      for (int64_t i = n - 1; i > 0; --i) std::swap(ids[i], ids[g.below((uint32_t)(i + 1))]);
      return DD_OK;
    }
    case DD_MULTIFRAME: {
      const int64_t total = n * d.frames;
      ids.resize(total);
      for (int64_t v = 0; v < total; ++v) ids[v] = (int32_t)(v % n);
      return DD_OK;
    }
    case DD_EXPLICIT:
      ids.assign(d.visits, d.visits + d.n_visits);
      return DD_OK;
  }
  return fail(DD_EINVAL, "unknown order %d", d.order);
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

static dd_status validate(const dd_scan_desc* d) {
  if (!d) return fail(DD_EINVAL, "desc is NULL");
  if (d->nx < 1 || d->ny < 1) return fail(DD_EINVAL, "nx and ny must be >= 1");
  if ((int64_t)d->nx * d->ny > (int64_t)1 << 30) return fail(DD_EINVAL, "probe grid too large");
  if (d->reserved != 0) return fail(DD_EINVAL, "reserved must be 0");
  if (!finite_pos(d->pitch_m)) return fail(DD_EINVAL, "pitch_m must be finite and > 0");
  if (!finite_pos(d->dwell_s)) return fail(DD_EINVAL, "dwell_s must be finite and > 0");
  if (!finite_pos(d->sigma_m)) return fail(DD_EINVAL, "sigma_m must be finite and > 0");
  if (!finite_pos(d->D_m2s)) return fail(DD_EINVAL, "D_m2s must be finite and > 0");
  if (!std::isfinite(d->Q0_us) || d->Q0_us < 0) return fail(DD_EINVAL, "Q0_us must be finite and >= 0");
  switch (d->order) {
    case DD_RASTER:
    case DD_RANDOM:
      break;
    case DD_INTERLEAVED:
      if (d->stride < 1) return fail(DD_EINVAL, "stride must be >= 1");
      break;
    case DD_MULTIFRAME:
      if (d->frames < 1) return fail(DD_EINVAL, "frames must be >= 1");
      if ((int64_t)d->nx * d->ny * d->frames > (int64_t)1 << 30)
        return fail(DD_EINVAL, "too many visits");
      break;
    case DD_EXPLICIT: {
      if (!d->visits || d->n_visits < 1) return fail(DD_EINVAL, "explicit visits missing");
      if (d->n_visits > (int64_t)1 << 30) return fail(DD_EINVAL, "too many visits");
      const int64_t n = (int64_t)d->nx * d->ny;
      for (int64_t v = 0; v < d->n_visits; ++v)
        if (d->visits[v] < 0 || d->visits[v] >= n) return fail(DD_EINVAL, "visit %lld out of range", (long long)v);
      break;
    }
    default:
      return fail(DD_EINVAL, "unknown order %d", d->order);
  }
  // Lattice coordinates and squared distances must stay exact in single
  // precision (|e|^2 + |p|^2 < 2^24).
  if (d->nx > 2048 || d->ny > 2048) return fail(DD_EINVAL, "probe grid side above 2048");
  return DD_OK;
}

// ---------------------------------------------------------------------------
// Lag-row closed forms on the host, used only for planning (c decides the
// near/far split and the series degree).
double row_c(double lam, double kappa, double s2) {
  const double db = 4.0 * kappa * std::min(lam, 1.0);
  const double b0 = s2 + 4.0 * kappa * std::max(lam - 1.0, 0.0);
  return db / (b0 * (b0 + db));
}

// Largest dx = a c at lag lam over the pairs that are not culled:
// min(a_max c, cull w), w = db / b0, since a <= cull b1 for those pairs and
// b1 c = w.
double row_dx_bound(double lam, double a_max, double cull, double kappa, double s2) {
  const double db = 4.0 * kappa * std::min(lam, 1.0);
  const double b0 = s2 + 4.0 * kappa * std::max(lam - 1.0, 0.0);
  return std::min(a_max * db / (b0 * (b0 + db)), cull * db / b0);
}

int degree_needed(double dx, bool mixed) {
  // smallest M with e^{2 dx} dx^{M+1} / (M+1)! below the precision's target
  const double tol = mixed ? 2e-8 : kTrunc64;
  const int mmax = mixed ? kM32 : kM64;
  if (dx <= 0) return 0;
  double term = std::exp(2 * dx);
  for (int M = 0; M <= mmax; ++M) {
    term *= dx / (M + 1);
    if (term <= tol) return M;
  }
  return mmax;
}

// First row n >= n_start (n >= 1) whose dx bound (row_dx_bound) is <= thr;
// the bound decreases for lags >= 1, so binary search applies.
int64_t first_row_below(double thr, double a_max, double cull, double f, double kappa, double s2,
                        int64_t n_start, int64_t n_end) {
  if (a_max <= 0) return n_start;
  auto ok = [&](int64_t n) {
    return row_dx_bound(f + (double)n, a_max, cull, kappa, s2) <= thr;
  };
  if (ok(n_start)) return n_start;
  int64_t lo = n_start, hi = std::max(n_end, n_start + 1);
  while (!ok(hi)) {
    lo = hi;
    hi = hi * 2 + 1;
    if (hi > ((int64_t)1 << 40)) return hi;
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (ok(mid))
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// Largest dx that the series of degree M covers: e^{2dx} dx^{M+1}/(M+1)! = tol
// (bisection), for M = 0 .. kMaxSeg; the same for every scan, computed once.
static const double* dx_cover(bool mixed) {
  struct Table {
    double v[kMaxSeg + 1];
    explicit Table(double tol) {
      for (int M = 0; M <= kMaxSeg; ++M) {
        double lo = 0, hi = 1.0;
        for (int it = 0; it < 80; ++it) {
          const double mid = 0.5 * (lo + hi);
          double t = std::exp(2 * mid);
          for (int k = 1; k <= M + 1; ++k) t *= mid / k;
          (t <= tol ? lo : hi) = mid;
        }
        v[M] = lo;
      }
    }
  };
  static const Table t32(2e-8), t64(kTrunc64);
  return mixed ? t32.v : t64.v;
}

// Degree bounds for the far region starting at row kf (aligned so that
// kf + k*align are the only segment starts).
DegreeBounds degree_bounds(double a_max, double f, double kappa, double s2, int64_t kf, int align,
                           bool mixed) {
  DegreeBounds b;
  b.plain = b.fold = 1 << 30;
  const int mmax = mixed ? kM32 : kM64;
  const double cull = mixed ? kCullX32 : kCullX64;
  const double dx0 = row_dx_bound(f + (double)kf, a_max, cull, kappa, s2);
  b.m_max = std::min(degree_needed(dx0, mixed), mmax);
  const double* cover = dx_cover(mixed);
  for (int M = 0; M <= kMaxSeg; ++M) b.b[M] = (int32_t)kf;
  for (int M = 0; M < b.m_max; ++M) {
    // first row whose dx bound degree M covers
    int64_t n = first_row_below(cover[M], a_max, cull, f, kappa, s2, kf, kf + 1);
    if (align > 1) n = kf + (n - kf + align - 1) / align * align;
    b.b[M] = (int32_t)std::min<int64_t>(n, (int64_t)1 << 30);
  }
  // make b nonincreasing in M (b[M] >= b[M+1])
  for (int M = b.m_max - 1; M >= 0; --M) b.b[M] = std::max(b.b[M], b.b[M + 1]);
  return b;
}

// First rows of the two lighter forms of the mixed arrival series (see
// DegreeBounds), for the far region from row kf, aligned like the degree
// segments.  y_max(n) = a_max log2(e) (rb1 + c) bounds a pair's exponent in
// both forms (RA = log2(e) (rb1 - c P_1/P_0) <= log2(e) (rb1 + c) since
// |P_1/P_0| < 1); the margin keeps fl(a rhi) and fl(a RA) below the powers
// of two that the error bounds assume.
void lean_bounds(DegreeBounds& b, double a_max, double kappa, double s2, int64_t kf, int align) {
  b.plain = b.fold = 1 << 30;
  if (a_max <= 0) return;
  auto ymax = [&](int64_t n) {
    const double lam = (double)n;
    const double db = 4.0 * kappa * std::min(lam, 1.0);
    const double b0 = s2 + 4.0 * kappa * std::max(lam - 1.0, 0.0);
    return a_max * 1.4426950408889634 * (1.0 / (b0 + db) + db / (b0 * (b0 + db)));
  };
  auto first_row = [&](double ylim, double dxlim) {  // both bounds fall with n
    auto ok = [&](int64_t n) {
      return ymax(n) <= ylim * (1.0 - 1e-6) &&
             row_dx_bound((double)n, a_max, kCullX32, kappa, s2) <= dxlim;
    };
    int64_t lo = kf, hi = kf;
    if (!ok(hi)) {
      while (!ok(hi)) {
        lo = hi;
        hi = hi * 2 + 1;
        if (hi > ((int64_t)1 << 30)) return (int64_t)1 << 30;
      }
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        (ok(mid) ? hi : lo) = mid;
      }
    }
    if (align > 1) hi = kf + (hi - kf + align - 1) / align * align;
    return std::min<int64_t>(hi, (int64_t)1 << 30);
  };
  const double* cover = dx_cover(true);
  b.fold = (int32_t)std::max<int64_t>(first_row(4.0, std::min(2e-4, cover[1])), b.b[1]);
  b.plain = (int32_t)std::max<int64_t>(first_row(8.0, cover[kMaxA]), b.b[kMaxA]);
  b.plain = std::min(b.plain, b.fold);
}

}  // namespace dd

using namespace dd;

// ---------------------------------------------------------------------------
// Scan handle.
dd_status dd_scan_create(const dd_scan_desc* desc, dd_scan** out) {
  if (!out) return fail(DD_EINVAL, "out is NULL");
  *out = nullptr;
  dd_status st = validate(desc);
  if (st != DD_OK) return st;
  int64_t V = desc->order == DD_EXPLICIT ? desc->n_visits
              : desc->order == DD_MULTIFRAME ? (int64_t)desc->nx * desc->ny * desc->frames
                                             : (int64_t)desc->nx * desc->ny;
  if (!host_alloc_ok((size_t)V * 24)) return fail(DD_ENOMEM, "host allocation over limit");
  dd_scan* s = new (std::nothrow) dd_scan();
  if (!s) return fail(DD_ENOMEM, "out of host memory");
  try {
    s->desc = *desc;
    s->desc.visits = nullptr;
    st = make_visits(*desc, s->ids);
    if (st != DD_OK) {
      delete s;
      return st;
    }
  } catch (const std::bad_alloc&) {
    delete s;
    return fail(DD_ENOMEM, "out of host memory");
  }
  s->V = (int64_t)s->ids.size();
  s->tau_v = desc->order == DD_MULTIFRAME ? desc->dwell_s / desc->frames : desc->dwell_s;
  s->kappa = desc->D_m2s * s->tau_v / (desc->pitch_m * desc->pitch_m);
  const double sh = desc->sigma_m / desc->pitch_m;
  s->s2 = 2.0 * sh * sh;
  s->pref = desc->Q0_us / (4.0 * M_PI * desc->D_m2s);  // Q0/(4 pi D) of Eqs. 1-4
  if (!(std::isfinite(s->kappa) && s->kappa > 0 && std::isfinite(s->s2) && s->s2 > 0 &&
        std::isfinite(s->pref))) {
    delete s;
    return fail(DD_EINVAL, "scan parameters out of the representable range");
  }
  *out = s;
  return DD_OK;
}

void dd_scan_destroy(dd_scan* s) {
  if (!s) return;
  s->release_device();
  delete s;
}

int64_t dd_scan_num_visits(const dd_scan* s) { return s ? s->V : -1; }

dd_status dd_scan_visits(const dd_scan* s, int32_t* out_host) {
  if (!s || !out_host) return fail(DD_EINVAL, "NULL argument");
  memcpy(out_host, s->ids.data(), sizeof(int32_t) * s->ids.size());
  return DD_OK;
}

const char* dd_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Kernel timing.
namespace {
struct ProfRec {
  std::string kernel;
  hipEvent_t a, b;
  double pairs, flops;
  bool done;
};
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
  std::map<std::string, dd_kernel_stats> tot;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
ProfState& prof() {
  static ProfState* p = new ProfState();
  return *p;
}
const char* const kKernelNames[] = {"arrival_far", "arrival_near", "map", "batch", "lag_rows",
                                    "reduce"};
}  // namespace

namespace dd {
ProfToken prof_begin(const char* kernel, hipStream_t st) {
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  ProfToken t;
  if (!P.on) return t;
  hipEvent_t a = P.get(), b = P.get();
  if (!a || !b) return t;
  if (hipEventRecord(a, st) != hipSuccess) return t;
  P.recs.push_back(ProfRec{kernel, a, b, 0, 0, false});
  t.slot = (int)P.recs.size() - 1;
  return t;
}
bool prof_on() {
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  return P.on;
}
void prof_end(ProfToken tok, hipStream_t st, double pairs, double flops) {
  if (tok.slot < 0) return;
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  if (tok.slot >= (int)P.recs.size()) return;
  ProfRec& r = P.recs[tok.slot];
  r.pairs = pairs;
  r.flops = flops;
  r.done = hipEventRecord(r.b, st) == hipSuccess;
}
}  // namespace dd

dd_status dd_profiling(int32_t enable) {
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  P.on = enable != 0;
  return DD_OK;
}

dd_status dd_profile_read(const char* kernel, dd_kernel_stats* out, int32_t reset) {
  if (!kernel || !out) return fail(DD_EINVAL, "NULL argument");
  bool known = false;
  for (const char* k : kKernelNames) known = known || strcmp(k, kernel) == 0;
  if (!known) return fail(DD_EINVAL, "unknown kernel name '%s'", kernel);
  ProfState& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  for (ProfRec& r : P.recs) {
    if (r.done) {
      if (hipEventSynchronize(r.b) != hipSuccess) return fail(DD_EDEVICE, "event synchronize failed");
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(DD_EDEVICE, "event time failed");
      dd_kernel_stats& t = P.tot[r.kernel];
      t.ms += ms;
      t.launches += 1;
      t.pairs += r.pairs;
      t.flops += r.flops;
    }
    P.pool.push_back(r.a);
    P.pool.push_back(r.b);
  }
  P.recs.clear();
  dd_kernel_stats z{0.0, 0, 0.0, 0.0};
  auto it = P.tot.find(kernel);
  *out = it == P.tot.end() ? z : it->second;
  if (reset) P.tot.erase(kernel);
  return DD_OK;
}
