// dd_tune.cpp -- autotuner of libdd's tile shapes.
//
// The parameters are the tile width of a work item (R evaluation points per
// lane: 64 R per wavefront) for the far region and for the near band, the
// number of lags per far work item, and the same width/length pair for maps.
// Each candidate is timed with HIP events on representative problems (the
// 512x512 random-order arrival query, a 128x128 final map) and the fastest is
// kept.  The winners go to a small JSON file that dd_tune_load reads back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "dd_runtime.h"

using namespace dd;

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Median time (ms) of `reps` runs of f after one warm-up run.
template <typename F>
dd_status time_ms(F&& f, hipStream_t st, int reps, double& out) {
  Timer t;
  std::vector<double> v;
  dd_status rc = f();
  if (rc != DD_OK) return rc;
  for (int k = 0; k < reps; ++k) {
    if (hipEventRecord(t.a, st) != hipSuccess) return fail(DD_EDEVICE, "event record failed");
    rc = f();
    if (rc != DD_OK) return rc;
    if (hipEventRecord(t.b, st) != hipSuccess) return fail(DD_EDEVICE, "event record failed");
    if (hipEventSynchronize(t.b) != hipSuccess) return fail(DD_EDEVICE, "event sync failed");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    v.push_back(ms);
  }
  std::sort(v.begin(), v.end());
  out = v[v.size() / 2];
  return DD_OK;
}

struct ScanGuard {
  dd_scan* s = nullptr;
  ~ScanGuard() { dd_scan_destroy(s); }
};

dd_status make_scan(int side, int order, uint64_t seed, double dwell, double sigma, double D,
                    ScanGuard& g) {
  dd_scan_desc d{};
  d.nx = d.ny = side;
  d.order = order;
  d.stride = 2;
  d.frames = 1;
  d.seed = seed;
  d.pitch_m = 1e-9;
  d.dwell_s = dwell;
  d.sigma_m = sigma;
  d.D_m2s = D;
  d.Q0_us = 1.0;
  return dd_scan_create(&d, &g.s);
}

bool write_cache(const char* path, const TuneParams& t, const double (&ms)[4]) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f,
          "{\n  \"arch\": \"gfx950\",\n  \"version\": 1,\n"
          "  \"arrival_mixed\": {\"R\": %d, \"RN\": %d, \"K\": %d, \"ms\": %.4f},\n"
          "  \"arrival_fp64\": {\"R\": %d, \"RN\": %d, \"K\": %d, \"ms\": %.4f},\n"
          "  \"map_mixed\": {\"R\": %d, \"K\": %d, \"ms\": %.4f},\n"
          "  \"map_fp64\": {\"R\": %d, \"K\": %d, \"ms\": %.4f}\n}\n",
          t.arr_R_mixed, t.arr_RN_mixed, t.arr_K_mixed, ms[0], t.arr_R_f64, t.arr_RN_f64,
          t.arr_K_f64, ms[1], t.map_R_mixed, t.map_K, ms[2], t.map_R_f64, t.map_K, ms[3]);
  return fclose(f) == 0;
}

// Finds "key": {...} and reads integer fields from it.
bool read_int(const std::string& txt, const char* obj, const char* field, int& out) {
  const std::string ko = std::string("\"") + obj + "\"";
  size_t p = txt.find(ko);
  if (p == std::string::npos) return false;
  const size_t open = txt.find('{', p), close = txt.find('}', p);
  if (open == std::string::npos || close == std::string::npos || open > close) return false;
  const std::string body = txt.substr(open, close - open);
  const std::string kf = std::string("\"") + field + "\"";
  size_t q = body.find(kf);
  if (q == std::string::npos) return false;
  q = body.find(':', q);
  if (q == std::string::npos) return false;
  char* end = nullptr;
  errno = 0;
  const long v = strtol(body.c_str() + q + 1, &end, 10);
  if (errno || end == body.c_str() + q + 1) return false;
  out = (int)v;
  return true;
}

bool valid(const TuneParams& t) {
  auto r_ok = [](int r) { return r == 2 || r == 4; };
  auto rm_ok = [](int r) { return r == 1 || r == 2 || r == 4; };
  auto k_ok = [](int k) { return k >= 64 && k <= (1 << 24); };
  return r_ok(t.arr_R_mixed) && r_ok(t.arr_R_f64) && r_ok(t.arr_RN_mixed) && r_ok(t.arr_RN_f64) &&
         k_ok(t.arr_K_mixed) && k_ok(t.arr_K_f64) && rm_ok(t.map_R_mixed) && rm_ok(t.map_R_f64) &&
         k_ok(t.map_K);
}

}  // namespace

dd_status dd_tune_load(const char* cache_path) {
  if (!cache_path) return fail(DD_EINVAL, "cache_path is NULL");
  FILE* f = fopen(cache_path, "r");
  if (!f) return fail(DD_EINVAL, "cannot open %s", cache_path);
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  if (txt.find("\"gfx950\"") == std::string::npos)
    return fail(DD_EINVAL, "%s is not a gfx950 tuning cache", cache_path);
  TuneParams t = tune();
  bool ok = read_int(txt, "arrival_mixed", "R", t.arr_R_mixed) &&
            read_int(txt, "arrival_mixed", "RN", t.arr_RN_mixed) &&
            read_int(txt, "arrival_mixed", "K", t.arr_K_mixed) &&
            read_int(txt, "arrival_fp64", "R", t.arr_R_f64) &&
            read_int(txt, "arrival_fp64", "RN", t.arr_RN_f64) &&
            read_int(txt, "arrival_fp64", "K", t.arr_K_f64) &&
            read_int(txt, "map_mixed", "R", t.map_R_mixed) &&
            read_int(txt, "map_mixed", "K", t.map_K) &&
            read_int(txt, "map_fp64", "R", t.map_R_f64);
  if (!ok || !valid(t)) return fail(DD_EINVAL, "malformed tuning cache %s", cache_path);
  tune() = t;
  return DD_OK;
}

dd_status dd_autotune(const char* cache_path) {
  std::string path = cache_path ? cache_path : "";
  if (path.empty()) {
    const char* e = getenv("DD_TUNE_CACHE");
    path = (e && *e) ? e : "dd_tune.json";
  }
  dd_status rc = ensure_device();
  if (rc != DD_OK) return rc;
  hipStream_t st = nullptr;
  if (hipStreamCreate(&st) != hipSuccess) return fail(DD_EDEVICE, "hipStreamCreate failed");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sg{st};
  const TuneParams saved = tune();
  TuneParams best = saved;
  double best_ms[4] = {0, 0, 0, 0};

  // Arrival: the 512x512 random scan (dwell 0.5 us, sigma 0.4 nm, D 1e-12).
  ScanGuard big;
  rc = make_scan(512, DD_RANDOM, 3, 0.5e-6, 0.4e-9, 1e-12, big);
  if (rc != DD_OK) return rc;
  double* out = nullptr;
  if (dev_alloc((void**)&out, sizeof(double) * 512 * 512) != hipSuccess)
    return fail(DD_ENOMEM, "device allocation failed");
  struct FreeGuard {
    double* p;
    ~FreeGuard() { (void)hipFree(p); }
  } fg{out};
  for (int mixed = 1; mixed >= 0; --mixed) {
    double bms = 1e30;
    for (int R : {2, 4})
      for (int RN : {2, 4})
        for (int K : {1024, 2048, 4096, 8192}) {
          TuneParams t = best;
          (mixed ? t.arr_R_mixed : t.arr_R_f64) = R;
          (mixed ? t.arr_RN_mixed : t.arr_RN_f64) = RN;
          (mixed ? t.arr_K_mixed : t.arr_K_f64) = K;
          tune() = t;
          double ms = 0;
          rc = time_ms(
              [&] {
                return dd_damage_at_probe_arrival(big.s, mixed ? DD_MIXED : DD_FP64, out, 1, st);
              },
              st, 3, ms);
          if (rc != DD_OK) {
            tune() = saved;
            return rc;
          }
          if (ms < bms) {
            bms = ms;
            best = t;
          }
        }
    best_ms[mixed ? 0 : 1] = bms;
  }
  // Maps: 128x128 final map of a 64x64 interleaved scan at 0.25 nm.
  ScanGuard mid;
  rc = make_scan(64, DD_INTERLEAVED, 0, 1e-6, 0.5e-9, 2.5e-13, mid);
  if (rc != DD_OK) {
    tune() = saved;
    return rc;
  }
  const dd_grid g{0.0, 0.0, 0.25e-9, 0.25e-9, 128, 128};
  const double t_end = 64.0 * 64.0 * 1e-6;
  double* mout = nullptr;
  if (dev_alloc((void**)&mout, sizeof(double) * 128 * 128) != hipSuccess) {
    tune() = saved;
    return fail(DD_ENOMEM, "device allocation failed");
  }
  FreeGuard fg2{mout};
  for (int mixed = 1; mixed >= 0; --mixed) {
    double bms = 1e30;
    for (int R : {1, 2, 4})
      for (int K : {1024, 4096, 16384}) {
        TuneParams t = best;
        (mixed ? t.map_R_mixed : t.map_R_f64) = R;
        if (mixed) t.map_K = K;
        if (!mixed && K != best.map_K) continue;
        tune() = t;
        double ms = 0;
        rc = time_ms([&] { return dd_damage_map(mid.s, &g, &t_end, 1, mixed ? DD_MIXED : DD_FP64,
                                                mout, 1, st); },
                     st, 3, ms);
        if (rc != DD_OK) {
          tune() = saved;
          return rc;
        }
        if (ms < bms) {
          bms = ms;
          best = t;
        }
      }
    best_ms[mixed ? 2 : 3] = bms;
  }
  tune() = best;
  if (!write_cache(path.c_str(), best, best_ms))
    return fail(DD_EINVAL, "cannot write %s", path.c_str());
  return DD_OK;
}
