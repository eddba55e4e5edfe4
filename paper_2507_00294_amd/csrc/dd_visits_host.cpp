// dd_visits_host.cpp -- the general visit list handle (dd_visits_*): every visit
// with its own position, start time and dwell (Sec. II, Eqs. 1-4 per visit,
// Eq. 6 over the visits started before the query time), in FP64 or with
// the near form in FP32 (mixed).
//
// Work planning.  Visits are kept in start order.  A launch serves one list
// or, for the batch calls, many: every tile names its list, whose
// descriptor (visits, order, output, grid and times, scaling) the kernels
// read.  Evaluation points go in tiles of 256 (one thread each); visits in
// chunks of K (a multiple of 256, at most 32 chunks per list).  A work item
// is one tile against one chunk, written to a partial-sum slot of its own,
// and the slots are summed in a fixed order, so results depend neither on
// scheduling nor on the other lists of a batch.  Items are dropped on the
// host when no pair can contribute, that is when
//   * the chunk's first start is at or after the tile's latest time
//     (nothing has started), or
//   * the bounding boxes of tile and chunk are so far apart that
//     a / b1 > 745 for every pair, with b1 taken at the largest lag
//     (the kernel would cull each pair; a margin of 1e-9 keeps host and
//     device roundings on the same side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <set>
#include <vector>

#include "../../include/dd.h"
#include "dd_runtime.h"
#include "dd_visits.h"

using namespace dd;

namespace {

struct Box {
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  void add(double x, double y) {
    x0 = std::min(x0, x);
    x1 = std::max(x1, x);
    y0 = std::min(y0, y);
    y1 = std::max(y1, y);
  }
};

// Smallest squared distance between two boxes, in units of sigma^2.
double box_a_min(const Box& p, const Box& q, double inv_sigma) {
  const double gx = std::max({0.0, q.x0 - p.x1, p.x0 - q.x1}) * inv_sigma;
  const double gy = std::max({0.0, q.y0 - p.y1, p.y0 - q.y1}) * inv_sigma;
  return gx * gx + gy * gy;
}

constexpr int64_t kGroupTiles = 4096;  // tiles per launch (partial sums <= 256 MiB)

#define VIS_HIP(call, what)                            \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, what);   \
  } while (0)

}  // namespace

struct dd_visits {
  int64_t n = 0;
  std::vector<double4> vis;   // (x, y, t0, dwell) in start order
  std::vector<int64_t> perm;  // start order -> caller's index
  double sigma = 0, D = 0, Q0 = 0, inv_sigma = 0, th4 = 0, pref = 0;
  int64_t K = 0;              // visits per chunk
  std::vector<Box> chunk_box;
  std::vector<double> chunk_t0;  // first start of each chunk

  int dev = -1;
  DevBuf d_vis, d_perm, tmp_out;

  void release_device() {
    for (DevBuf* b : {&d_vis, &d_perm, &tmp_out})
      b->release();
    dev = -1;
  }

  dd_status prepare(hipStream_t st) {
    dd_status rc = ensure_device();
    if (rc != DD_OK) return rc;
    int cur = 0;
    VIS_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (dev >= 0 && dev != cur) release_device();
    if (dev == cur) return DD_OK;
    VIS_HIP(d_vis.ensure(sizeof(double4) * n), "device allocation");
    VIS_HIP(d_perm.ensure(sizeof(int64_t) * n), "device allocation");
    VIS_HIP(hipMemcpyAsync(d_vis.p, vis.data(), sizeof(double4) * n, hipMemcpyHostToDevice, st),
            "host-to-device copy");
    VIS_HIP(hipMemcpyAsync(d_perm.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st),
            "host-to-device copy");
    VIS_HIP(hipStreamSynchronize(st), "stream synchronize");
    dev = cur;
    return DD_OK;
  }

  // Items of one tile (box, latest time) against every chunk that can
  // contribute, appended to `items`; returns the number of slots used.
  int32_t plan_tile(int32_t tile, const Box& box, double tmax, std::vector<VisItem>& items) const {
    int32_t slot = 0;
    const int64_t n_chunks = (int64_t)chunk_t0.size();
    for (int64_t c = 0; c < n_chunks && chunk_t0[c] < tmax; ++c) {
      const double b1_max = 2.0 + th4 * (tmax - chunk_t0[c]);
      if (box_a_min(box, chunk_box[c], inv_sigma) > 745.0 * (1.0 + 1e-9) * b1_max) continue;
      const int64_t v0 = c * K;
      items.push_back(VisItem{tile, slot++, v0, std::min(K, n - v0)});
    }
    return slot;
  }

  VisList desc(double* out, OutFlag fl, const double* times = nullptr,
               VisGrid grid = VisGrid{}) const {
    return VisList{d_vis.as<double4>(), d_perm.as<int64_t>(), out, times, grid,
                   inv_sigma, th4, pref, fl};
  }

  // Tiles of the arrival query (visits in start order), appended for list `list`.
  void arrival_tiles(int32_t list, std::vector<VisTile>& tiles) const {
    for (int64_t p0 = 0; p0 < n; p0 += kVisTile) {
      const int64_t p1 = std::min(n, p0 + kVisTile);
      tiles.push_back(VisTile{p0, 0, 0, vis[p1 - 1].z, (int32_t)(p1 - p0), 0, 0, list, 0, 0});
    }
  }
  Box tile_box(const VisTile& t) const {
    Box b;
    for (int64_t p = t.p0; p < t.p0 + t.n; ++p) b.add(vis[p].x, vis[p].y);
    return b;
  }

};

namespace {

// Per-thread launch tables of the visit-list queries (host vectors reused
// between calls, device buffers grown as needed).
// Pinned host memory of the launch tables, grown as needed.
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need) {
    if (need <= bytes && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    const size_t want = std::max(need, (size_t)1 << 20);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e == hipSuccess) bytes = want;
    return e;
  }
};

// A launch group's tables go to the device in one copy from pinned memory:
// [map times | list descriptors | tiles | items], each part 256-byte aligned.
// While a copy or launch may be in flight (`inflight`), the next group waits
// for the event recorded after the previous group's launches (`done`, on
// whatever stream those went to) before it rewrites the stage or regrows a
// device buffer.  A call ends with its stream synchronized (the non-finite
// check), which clears the flag; a call that failed half-way leaves it set,
// and the next group, on any stream, still waits.
struct VisScratch {
  std::vector<VisTile> h_tiles;
  std::vector<VisItem> h_items;
  std::vector<VisList> h_lists;
  std::vector<const double*> h_times;  // maps: each list's times (host) and count
  std::vector<int32_t> h_nt;
  HostStage stage;
  DevBuf d_stage, d_partial;
  bool inflight = false;
  hipEvent_t done = nullptr;  // after the last group's launches; kept until the process ends
  // non-finite flag of the thread's calls (see OutFlag), read at the end
  // of each call
  DevBuf flag;
  uint64_t seq = 0;
  unsigned long long* flag_host = nullptr;  // pinned, kept until the process ends
};
thread_local VisScratch g_vis;

// A fresh flag for a call; the word is cleared when first used and when
// the seq wraps.
dd_status call_flag(hipStream_t st, OutFlag& fl) {
  VisScratch& W = g_vis;
  if (!W.flag_host)
    VIS_HIP(hipHostMalloc((void**)&W.flag_host, 256, hipHostMallocDefault),
            "pinned host allocation");
  if (!W.flag.p || W.seq >= kFlagSeqMax) {
    VIS_HIP(W.flag.ensure(sizeof(unsigned long long)), "device allocation");
    *W.flag_host = 0;
    VIS_HIP(hipMemcpyAsync(W.flag.p, W.flag_host, sizeof(unsigned long long),
                           hipMemcpyHostToDevice, st),
            "host-to-device copy");
    VIS_HIP(hipStreamSynchronize(st), "stream synchronize");
    W.seq = 0;
  }
  fl = OutFlag{W.flag.as<unsigned long long>(), (unsigned long long)++W.seq, 0};
  return DD_OK;
}

// After a call's last launch: DD_EDEVICE naming the list and index of its
// first non-finite output (off[k]: flat offset of list k's output).
dd_status check_call_flag(const OutFlag& fl, const std::vector<int64_t>& off, hipStream_t st) {
  VisScratch& W = g_vis;
  VIS_HIP(hipMemcpyAsync(W.flag_host, fl.word, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         st),
          "device-to-host copy");
  VIS_HIP(hipStreamSynchronize(st), "stream synchronize");
  W.inflight = false;
  const unsigned long long w = *W.flag_host;
  constexpr unsigned long long lim = (1ull << kFlagIndexBits) - 1;
  if ((w >> kFlagIndexBits) != fl.seq) return DD_OK;
  const int64_t bad = (int64_t)(lim - (w & lim));
  const int32_t k = (int32_t)(std::upper_bound(off.begin(), off.end(), bad) - off.begin()) - 1;
  return fail(DD_EDEVICE, "list %d: non-finite output value at index %lld", k,
              (long long)(bad - off[k]));
}

// Items in launch order: the most recent visits relative to the tile's
// time first (the pairs of short lags take the costlier forms; started
// early, they overlap the rest instead of trailing it).  Only the schedule
// changes: every item keeps its slot, so the sums do not.
void order_items(dd_visits* const* lists) {
  VisScratch& W = g_vis;
  std::vector<std::pair<double, int64_t>> key(W.h_items.size());
  for (size_t i = 0; i < W.h_items.size(); ++i) {
    const VisItem& it = W.h_items[i];
    const VisTile& tile = W.h_tiles[it.tile];
    const dd_visits* v = lists[tile.list];
    key[i] = {tile.tmax - v->chunk_t0[it.v0 / v->K], (int64_t)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<VisItem> sorted(W.h_items.size());
  for (size_t i = 0; i < key.size(); ++i) sorted[i] = W.h_items[key[i].second];
  W.h_items.swap(sorted);
}

// Partial sums and reduce of the current tiles and items (one launch group),
// with the tables staged and copied in one transfer.
dd_status launch_group(bool map, bool mixed, hipStream_t st) {
  VisScratch& W = g_vis;
  if (W.inflight) {
    VIS_HIP(hipEventSynchronize(W.done), "event synchronize");
    W.inflight = false;
  }
  if (!W.done) VIS_HIP(hipEventCreateWithFlags(&W.done, hipEventDisableTiming), "event creation");
  int64_t pbase = 0;
  double pairs = 0;
  for (VisTile& t : W.h_tiles) {
    t.pbase = pbase;
    pbase += (int64_t)t.slots * kVisTile;
  }
  for (const VisItem& it : W.h_items) pairs += (double)W.h_tiles[it.tile].n * (double)it.nv;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t nl = W.h_lists.size();
  std::vector<size_t> t_off(nl, 0);
  size_t off = 0;
  if (map)
    for (size_t k = 0; k < nl; ++k) {
      t_off[k] = off;
      off = up(off + sizeof(double) * (size_t)W.h_nt[k]);
    }
  const size_t l_off = off;
  off = up(off + sizeof(VisList) * nl);
  const size_t ti_off = off;
  off = up(off + sizeof(VisTile) * W.h_tiles.size());
  const size_t it_off = off;
  off = up(off + sizeof(VisItem) * std::max<size_t>(W.h_items.size(), 1));
  VIS_HIP(W.stage.ensure(off), "pinned host allocation");
  VIS_HIP(W.d_stage.ensure(off), "device allocation");
  VIS_HIP(W.d_partial.ensure(sizeof(double) * std::max<int64_t>(pbase, 1)), "device allocation");
  char* h = static_cast<char*>(W.stage.p);
  char* d = static_cast<char*>(W.d_stage.p);
  for (size_t k = 0; k < nl; ++k) {
    VisList L = W.h_lists[k];
    if (map) {
      std::copy(W.h_times[k], W.h_times[k] + W.h_nt[k], reinterpret_cast<double*>(h + t_off[k]));
      L.times = reinterpret_cast<const double*>(d + t_off[k]);
    }
    reinterpret_cast<VisList*>(h + l_off)[k] = L;
  }
  std::copy(W.h_tiles.begin(), W.h_tiles.end(), reinterpret_cast<VisTile*>(h + ti_off));
  std::copy(W.h_items.begin(), W.h_items.end(), reinterpret_cast<VisItem*>(h + it_off));
  W.inflight = true;
  VIS_HIP(hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, st), "host-to-device copy");
  VIS_HIP(hipEventRecord(W.done, st), "event record");  // the stage is read; again after the launches
  const VisList* dl = reinterpret_cast<const VisList*>(d + l_off);
  const VisTile* dt = reinterpret_cast<const VisTile*>(d + ti_off);
  const VisItem* di = reinterpret_cast<const VisItem*>(d + it_off);
  const ProfToken tok = prof_begin("k_visit_pairs", st);
  VIS_HIP(launch_visit_pairs(map, mixed, dl, dt, di, (int64_t)W.h_items.size(),
                             W.d_partial.as<double>(), st),
          "k_visit_pairs launch");
  prof_end(tok, st, pairs, 0.0);
  VIS_HIP(launch_visit_reduce(map, dl, dt, (int64_t)W.h_tiles.size(), W.d_partial.as<double>(),
                              st),
          "k_visit_reduce launch");
  VIS_HIP(hipEventRecord(W.done, st), "event record");
  return DD_OK;
}

// Arrival queries of lists[k] into outs[k] (device), all in the same launch
// groups: each list's tiles and items are planned exactly as for a call of
// its own, so the results do not depend on the batch.
dd_status run_arrivals(dd_visits* const* lists, int32_t n, bool mixed, double* const* outs,
                       hipStream_t st) {
  VisScratch& W = g_vis;
  OutFlag fl;
  dd_status rc = call_flag(st, fl);
  if (rc != DD_OK) return rc;
  std::vector<int64_t> off(n, 0);
  W.h_lists.resize(n);
  for (int32_t k = 0; k < n; ++k) {
    if (k > 0) off[k] = off[k - 1] + lists[k - 1]->n;
    fl.base = off[k];
    W.h_lists[k] = lists[k]->desc(outs[k], fl);
  }
  std::vector<VisTile> all;
  for (int32_t k = 0; k < n; ++k) lists[k]->arrival_tiles(k, all);
  for (size_t g0 = 0; g0 < all.size(); g0 += kGroupTiles) {
    const size_t g1 = std::min(all.size(), g0 + (size_t)kGroupTiles);
    W.h_tiles.assign(all.begin() + g0, all.begin() + g1);
    W.h_items.clear();
    for (size_t t = 0; t < W.h_tiles.size(); ++t) {
      VisTile& tile = W.h_tiles[t];
      const dd_visits* v = lists[tile.list];
      tile.slots = v->plan_tile((int32_t)t, v->tile_box(tile), tile.tmax, W.h_items);
    }
    order_items(lists);
    rc = launch_group(false, mixed, st);
    if (rc != DD_OK) return rc;
  }
  return check_call_flag(fl, off, st);
}

// Map tiles of a w x h grid: blocks of tw = min(w, 16) columns and
// th = min(h, 256 / tw) rows (a narrow grid takes taller blocks), in
// row-major block order; a square block keeps the spread of distances from
// a visit to the tile's pixels small.
struct MapTiling {
  int32_t w, h, tw, th, bx, by;
  explicit MapTiling(const dd_grid& g)
      : w(g.w), h(g.h), tw(std::min(g.w, 16)), th(std::min(g.h, kVisTile / std::min(g.w, 16))),
        bx((g.w + tw - 1) / tw), by((g.h + th - 1) / th) {}
  int64_t count() const { return (int64_t)bx * by; }
  // top-left pixel and size of block b
  void block(int64_t b, int32_t& u0, int32_t& v0, int32_t& cw, int32_t& ch) const {
    u0 = (int32_t)(b % bx) * tw;
    v0 = (int32_t)(b / bx) * th;
    cw = std::min(tw, w - u0);
    ch = std::min(th, h - v0);
  }
};

// Maps of lists[k] on grids[k] at times t_s[k][0 .. n_t[k]) into outs[k]
// (device), all in the same launch groups; each list's tiles and items are
// planned exactly as for a call of its own (tiles time by time, blocks in
// order), so the results do not depend on the batch.
dd_status run_maps(dd_visits* const* lists, int32_t n, const dd_grid* grids,
                   const double* const* t_s, const int32_t* n_t, bool mixed, double* const* outs,
                   hipStream_t st) {
  VisScratch& W = g_vis;
  std::vector<int64_t> npix(n), per(n), off(n, 0);
  std::vector<std::vector<Box>> boxes(n);
  std::vector<MapTiling> tiling;
  OutFlag fl;
  dd_status rc0 = call_flag(st, fl);
  if (rc0 != DD_OK) return rc0;
  W.h_lists.resize(n);
  W.h_times.resize(n);
  W.h_nt.resize(n);
  for (int32_t k = 0; k < n; ++k) {
    const dd_grid* g = &grids[k];
    dd_visits* v = lists[k];
    tiling.emplace_back(*g);
    npix[k] = (int64_t)g->w * g->h;
    per[k] = tiling[k].count();  // tiles per time
    if (k > 0) off[k] = off[k - 1] + (int64_t)n_t[k - 1] * npix[k - 1];
    fl.base = off[k];
    // times: set to the staged copy by launch_group
    W.h_lists[k] = v->desc(outs[k], fl, nullptr,
                           VisGrid{g->x0_m, g->y0_m, g->dx_m, g->dy_m, g->w, 0});
    W.h_times[k] = t_s[k];
    W.h_nt[k] = n_t[k];
    // pixel boxes of the tiles (the same at every time)
    boxes[k].resize(per[k]);
    for (int64_t b = 0; b < per[k]; ++b) {
      int32_t u0, v0, cw, ch;
      tiling[k].block(b, u0, v0, cw, ch);
      boxes[k][b].add(g->x0_m + (double)u0 * g->dx_m, g->y0_m + (double)v0 * g->dy_m);
      boxes[k][b].add(g->x0_m + (double)(u0 + cw - 1) * g->dx_m,
                      g->y0_m + (double)(v0 + ch - 1) * g->dy_m);
    }
  }
  dd_status rc = DD_OK;
  int32_t k = 0;
  int64_t local = 0;  // next tile of list k
  while (k < n) {
    W.h_tiles.clear();
    W.h_items.clear();
    while ((int64_t)W.h_tiles.size() < kGroupTiles && k < n) {
      const int64_t m = local / per[k], b = local % per[k];
      int32_t u0, v0, cw, ch;
      tiling[k].block(b, u0, v0, cw, ch);
      const int64_t p0 = (int64_t)v0 * grids[k].w + u0;
      const double t = t_s[k][m];
      VisTile tile{p0, 0, m * npix[k] + p0, t, cw * ch, (int32_t)m, 0, k, cw, 0};
      tile.slots = lists[k]->plan_tile((int32_t)W.h_tiles.size(), boxes[k][b], t, W.h_items);
      W.h_tiles.push_back(tile);
      if (++local == per[k] * n_t[k]) {
        ++k;
        local = 0;
      }
    }
    order_items(lists);
    rc = launch_group(true, mixed, st);
    if (rc != DD_OK) return rc;
  }
  return check_call_flag(fl, off, st);
}

dd_status check_map_args(const dd_grid* g, const double* t_s, int32_t n_t) {
  if (!g || !t_s) return fail(DD_EINVAL, "NULL argument");
  if (n_t < 1) return fail(DD_EINVAL, "n_t must be >= 1");
  if (g->w < 1 || g->h < 1) return fail(DD_EINVAL, "grid w and h must be >= 1");
  if ((int64_t)g->w * g->h > (1LL << 30)) return fail(DD_EINVAL, "grid too large");
  for (double x : {g->x0_m, g->y0_m, g->dx_m, g->dy_m})
    if (!std::isfinite(x)) return fail(DD_EINVAL, "grid values must be finite");
  for (int32_t m = 0; m < n_t; ++m)
    if (!std::isfinite(t_s[m])) return fail(DD_EINVAL, "time %d not finite", m);
  return DD_OK;
}

}  // namespace

extern "C" {

dd_status dd_visits_create(int64_t n, const double* x_m, const double* y_m, const double* t0_s,
                           const double* dwell_s, double sigma_m, double D_m2s, double Q0_us,
                           dd_visits** out) {
  if (!out) return fail(DD_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1) return fail(DD_EINVAL, "a visit list needs at least one visit");
  if (!x_m || !y_m || !t0_s || !dwell_s) return fail(DD_EINVAL, "NULL argument");
  if (n > (int64_t)1 << 31) return fail(DD_EINVAL, "at most 2^31 visits");
  if (!(std::isfinite(sigma_m) && sigma_m > 0)) return fail(DD_EINVAL, "sigma must be > 0");
  if (!(std::isfinite(D_m2s) && D_m2s > 0)) return fail(DD_EINVAL, "D must be > 0");
  if (!(std::isfinite(Q0_us) && Q0_us >= 0)) return fail(DD_EINVAL, "Q0 must be >= 0");
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(x_m[i]) || !std::isfinite(y_m[i]))
      return fail(DD_EINVAL, "visit %lld: position not finite", (long long)i);
    if (!std::isfinite(t0_s[i])) return fail(DD_EINVAL, "visit %lld: start not finite", (long long)i);
    if (!(std::isfinite(dwell_s[i]) && dwell_s[i] > 0))
      return fail(DD_EINVAL, "visit %lld: dwell must be finite and > 0", (long long)i);
  }
  if (!host_alloc_ok(sizeof(double4) * (size_t)n)) return fail(DD_ENOMEM, "host allocation");
  dd_visits* v = new (std::nothrow) dd_visits;
  if (!v) return fail(DD_ENOMEM, "host allocation");
  try {
    v->n = n;
    v->perm.resize(n);
    std::iota(v->perm.begin(), v->perm.end(), (int64_t)0);
    std::stable_sort(v->perm.begin(), v->perm.end(),
                     [&](int64_t a, int64_t b) { return t0_s[a] < t0_s[b]; });
    v->vis.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t k = v->perm[i];
      v->vis[i] = make_double4(x_m[k], y_m[k], t0_s[k], dwell_s[k]);
    }
    v->K = std::max<int64_t>(512, ((n + kVisMaxSlots - 1) / kVisMaxSlots + kVisStage - 1) /
                                      kVisStage * kVisStage);
    for (int64_t c0 = 0; c0 < n; c0 += v->K) {
      Box b;
      for (int64_t i = c0; i < std::min(n, c0 + v->K); ++i) b.add(v->vis[i].x, v->vis[i].y);
      v->chunk_box.push_back(b);
      v->chunk_t0.push_back(v->vis[c0].z);
    }
  } catch (const std::bad_alloc&) {
    delete v;
    return fail(DD_ENOMEM, "host allocation");
  }
  v->sigma = sigma_m;
  v->D = D_m2s;
  v->Q0 = Q0_us;
  v->inv_sigma = 1.0 / sigma_m;
  v->th4 = 4.0 * D_m2s / (sigma_m * sigma_m);
  v->pref = Q0_us / (4.0 * M_PI * D_m2s);
  *out = v;
  return DD_OK;
}

void dd_visits_destroy(dd_visits* v) {
  if (!v) return;
  v->release_device();
  delete v;
}

int64_t dd_visits_count(const dd_visits* v) { return v ? v->n : -1; }

dd_status dd_visits_arrival(dd_visits* v, dd_precision p, double* out, int32_t out_on_device,
                            void* hip_stream) {
  if (!v || !out) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  const bool mixed = p == DD_MIXED;
  hipStream_t st = (hipStream_t)hip_stream;
  dd_status rc = v->prepare(st);
  if (rc != DD_OK) return rc;
  if (out_on_device) return run_arrivals(&v, 1, mixed, &out, st);
  VIS_HIP(v->tmp_out.ensure(sizeof(double) * v->n), "device allocation");
  double* tmp = v->tmp_out.as<double>();
  rc = run_arrivals(&v, 1, mixed, &tmp, st);
  if (rc != DD_OK) return rc;
  VIS_HIP(hipMemcpyAsync(out, v->tmp_out.p, sizeof(double) * v->n, hipMemcpyDeviceToHost, st),
          "device-to-host copy");
  VIS_HIP(hipStreamSynchronize(st), "stream synchronize");
  return DD_OK;
}

dd_status dd_visits_map(dd_visits* v, const dd_grid* g, const double* t_s, int32_t n_t,
                        dd_precision p, double* out, int32_t out_on_device, void* hip_stream) {
  if (!v || !out) return fail(DD_EINVAL, "NULL argument");
  return dd_visits_batch_map(&v, 1, g, &t_s, &n_t, p, &out, out_on_device, hip_stream);
}

dd_status dd_visits_batch_map(dd_visits* const* lists, int32_t n, const dd_grid* grids,
                              const double* const* t_s, const int32_t* n_t, dd_precision p,
                              double* const* outs, int32_t out_on_device, void* hip_stream) {
  if (!lists || !grids || !t_s || !n_t || !outs || n < 1)
    return fail(DD_EINVAL, "NULL argument or n < 1");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  std::set<const dd_visits*> seen;
  for (int32_t k = 0; k < n; ++k) {
    if (!lists[k] || !outs[k]) return fail(DD_EINVAL, "list or output %d is NULL", k);
    if (!seen.insert(lists[k]).second)
      return fail(DD_EINVAL, "list %d appears twice (a list holds one set of map times)", k);
    dd_status rc = check_map_args(&grids[k], t_s[k], n_t[k]);
    if (rc != DD_OK) return rc;
  }
  const bool mixed = p == DD_MIXED;
  hipStream_t st = (hipStream_t)hip_stream;
  for (int32_t k = 0; k < n; ++k) {
    dd_status rc = lists[k]->prepare(st);
    if (rc != DD_OK) return rc;
  }
  if (out_on_device) return run_maps(lists, n, grids, t_s, n_t, mixed, outs, st);
  // host outputs: one device buffer for all maps, then a copy per list
  std::vector<int64_t> off(n + 1, 0);
  for (int32_t k = 0; k < n; ++k)
    off[k + 1] = off[k] + (int64_t)n_t[k] * grids[k].w * grids[k].h;
  DevBuf tmp;
  VIS_HIP(tmp.ensure(sizeof(double) * off[n]), "device allocation");
  std::vector<double*> douts(n);
  for (int32_t k = 0; k < n; ++k) douts[k] = tmp.as<double>() + off[k];
  dd_status rc = run_maps(lists, n, grids, t_s, n_t, mixed, douts.data(), st);
  if (rc == DD_OK) {
    for (int32_t k = 0; k < n && rc == DD_OK; ++k) {
      hipError_t e = hipMemcpyAsync(outs[k], douts[k], sizeof(double) * (off[k + 1] - off[k]),
                                    hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) rc = hip_fail(e, "device-to-host copy");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == DD_OK && e != hipSuccess) rc = hip_fail(e, "stream synchronize");
  }
  tmp.release();
  return rc;
}

dd_status dd_visits_batch_arrival(dd_visits* const* lists, int32_t n, dd_precision p,
                                  double* const* outs, int32_t out_on_device, void* hip_stream) {
  if (!lists || !outs || n < 1) return fail(DD_EINVAL, "NULL argument or n < 1");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  for (int32_t k = 0; k < n; ++k)
    if (!lists[k] || !outs[k]) return fail(DD_EINVAL, "list or output %d is NULL", k);
  const bool mixed = p == DD_MIXED;
  hipStream_t st = (hipStream_t)hip_stream;
  for (int32_t k = 0; k < n; ++k) {
    dd_status rc = lists[k]->prepare(st);
    if (rc != DD_OK) return rc;
  }
  if (out_on_device) return run_arrivals(lists, n, mixed, outs, st);
  // host outputs: one device buffer for all lists, then a copy per list
  std::vector<int64_t> off(n + 1, 0);
  for (int32_t k = 0; k < n; ++k) off[k + 1] = off[k] + lists[k]->n;
  DevBuf tmp;
  VIS_HIP(tmp.ensure(sizeof(double) * off[n]), "device allocation");
  std::vector<double*> douts(n);
  for (int32_t k = 0; k < n; ++k) douts[k] = tmp.as<double>() + off[k];
  dd_status rc = run_arrivals(lists, n, mixed, douts.data(), st);
  if (rc == DD_OK) {
    for (int32_t k = 0; k < n && rc == DD_OK; ++k) {
      hipError_t e = hipMemcpyAsync(outs[k], douts[k], sizeof(double) * lists[k]->n,
                                    hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) rc = hip_fail(e, "device-to-host copy");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == DD_OK && e != hipSuccess) rc = hip_fail(e, "stream synchronize");
  }
  tmp.release();
  return rc;
}

}  // extern "C"
