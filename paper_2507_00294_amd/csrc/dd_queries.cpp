// dd_queries.cpp -- query entry points of libdd (arrival, map, batch, pair
// terms) and their work planning.  Eq. 6 of the paper is evaluated as a sum
// over (evaluation point, lag) pairs; see dd_kernels.hip for the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/dd.h"
#include "dd_internal.h"
#include "dd_kernels.h"
#include "dd_runtime.h"

namespace dd {

TuneParams& tune() {
  static TuneParams t;
  return t;
}

#define DD_HIP(call, what)                  \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename T>
static dd_status upload(DevBuf& b, const std::vector<T>& h, hipStream_t st) {
  DD_HIP(b.ensure(sizeof(T) * std::max<size_t>(h.size(), 1)), "device allocation");
  if (!h.empty()) {
    DD_HIP(hipMemcpyAsync(b.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st),
           "host-to-device copy");
    // the host vector is reused by the next call: wait for the copy
    DD_HIP(hipStreamSynchronize(st), "stream synchronize");
  }
  return DD_OK;
}

}  // namespace dd

using namespace dd;

// Positions of every visit in pitch units, padded by kPosPad zeros on both
// sides; integer rows 0 .. V + margin for the current scan parameters.
dd_status dd_scan::prepare(hipStream_t st) {
  dd_status rc = ensure_device();
  if (rc != DD_OK) return rc;
  int cur = 0;
  DD_HIP(hipGetDevice(&cur), "hipGetDevice");
  if (dev >= 0 && dev != cur) release_device();
  if (dev == cur) return DD_OK;
  const int64_t n = V + 2 * (int64_t)kPosPad;
  std::vector<float2> p32(n, make_float2(0.f, 0.f));
  std::vector<double2> p64(n, make_double2(0.0, 0.0));
  std::vector<float4> p4(n, make_float4(0.f, 0.f, 0.f, 0.f));
  for (int64_t v = 0; v < V; ++v) {
    const int32_t id = ids[v];
    const double x = id % desc.nx, y = id / desc.nx;
    p32[kPosPad + v] = make_float2((float)x, (float)y);
    p64[kPosPad + v] = make_double2(x, y);
    p4[kPosPad + v] = make_float4((float)(-2 * x), (float)(-2 * y), (float)(x * x + y * y), 0.f);
  }
  rc = upload(pos32, p32, st);
  if (rc != DD_OK) return rc;
  rc = upload(pos64, p64, st);
  if (rc != DD_OK) return rc;
  rc = upload(pos4, p4, st);
  if (rc != DD_OK) return rc;
  rc = upload(flag, std::vector<unsigned long long>(1, 0ull), st);
  if (rc != DD_OK) return rc;
  seq = 0;
  dev = cur;
  return DD_OK;
}

dd_status dd_scan::wait_last(hipStream_t st) {
  if (last && last->stream != st) DD_HIP(hipStreamWaitEvent(st, last->ev, 0), "stream wait");
  return DD_OK;
}

dd_status dd_scan::record_last(hipStream_t st) {
  if (!own) {
    auto e = std::make_shared<StreamEvent>();
    DD_HIP(hipEventCreateWithFlags(&e->ev, hipEventDisableTiming), "event creation");
    own = e;
  }
  DD_HIP(hipEventRecord(own->ev, st), "event record");
  own->stream = st;
  last = own;
  return DD_OK;
}

dd_status dd_scan::next_flag(hipStream_t st, OutFlag& fl) {
  if (seq >= kFlagSeqMax) {  // the seq wraps: clear the word first
    dd_status rc = upload(flag, std::vector<unsigned long long>(1, 0ull), st);
    if (rc != DD_OK) return rc;
    seq = 0;
  }
  ++seq;
  fl = OutFlag{flag.as<unsigned long long>(), (unsigned long long)seq, 0};
  return DD_OK;
}

namespace dd {

// Host word that receives a flag word (pinned, one per thread).
static thread_local unsigned long long* g_flag_host = nullptr;

// Copies a flag word to the host on st, synchronizes st and decodes it:
// the first non-finite output index of call `call_seq`, or -1.
static dd_status read_flag(const unsigned long long* word, hipStream_t st, uint64_t call_seq,
                           int64_t& first_bad) {
  first_bad = -1;
  if (!g_flag_host)
    DD_HIP(hipHostMalloc((void**)&g_flag_host, 256, hipHostMallocDefault), "pinned host allocation");
  DD_HIP(hipMemcpyAsync(g_flag_host, word, sizeof(unsigned long long), hipMemcpyDeviceToHost, st),
         "device-to-host copy");
  DD_HIP(hipStreamSynchronize(st), "stream synchronize");
  const unsigned long long w = *g_flag_host;
  constexpr unsigned long long lim = (1ull << kFlagIndexBits) - 1;
  if ((w >> kFlagIndexBits) == call_seq) first_bad = (int64_t)(lim - (w & lim));
  return DD_OK;
}

}  // namespace dd

dd_status dd_scan::check_flag(hipStream_t st, uint64_t call_seq) {
  int64_t bad = -1;
  dd_status rc = read_flag(flag.as<unsigned long long>(), st, call_seq, bad);
  if (rc != DD_OK) return rc;
  if (bad >= 0)
    return fail(DD_EDEVICE, "non-finite output value at index %lld of the call's output",
                (long long)bad);
  return DD_OK;
}

namespace {

// Integer-lag rows 0 .. V + 1024 (rows past V serve the aligned ends of the
// last lag chunks, whose pairs are masked).  They depend on the scan alone
// (kappa, sigma, V), so they are built by the scan's first query and kept.
dd_status build_int_rows(dd_scan* s, hipStream_t st) {
  const int64_t n_rows = s->V + 1024;
  if (s->n_rows == n_rows) return DD_OK;
  DD_HIP(s->rows64.ensure(sizeof(double) * kRow64 * n_rows), "device allocation");
  DD_HIP(s->rows32.ensure(sizeof(float) * kRow32 * n_rows), "device allocation");
  DD_HIP(launch_lag_rows(0, n_rows, 0.0, s->kappa, s->s2, gl_nodes(), s->rows64.as<double>(),
                         s->rows32.as<float>(), st),
         "lag-row kernel launch");
  s->n_rows = n_rows;
  return DD_OK;
}

// Causal pairs of an arrival item: sum over visits j in [A, B) of the lags
// n in [lo, hi) with n <= j.
double arrival_pairs(int64_t A, int64_t B, int64_t lo, int64_t hi) {
  if (hi <= lo || B <= A) return 0.0;
  const double L = (double)(hi - lo);
  auto S = [L](double x) {  // sum_{u=0}^{x-1} clamp(u, 0, L), x >= 0
    if (x <= L + 1) return x * (x - 1) / 2;
    return L * (L + 1) / 2 + (x - L - 1) * L;
  };
  const double u0 = std::max<double>(0, (double)(A + 1 - lo));
  const double u1 = std::max<double>(0, (double)(B - lo));
  return S(u1) - S(u0);
}

// Split [lo, hi) by the degree bounds and add up pairs and flops.
template <typename PairsFn>
void count_segments(const DegreeBounds& b, int64_t lo, int64_t hi, bool mixed, PairsFn&& pairs,
                    double& p_out, double& f_out) {
  const int64_t fold = std::max<int64_t>(lo, std::min<int64_t>(hi, b.fold));
  for (int M = b.m_max; M >= 0; --M) {
    const int64_t a = std::max<int64_t>(lo, b.b[M]);
    const int64_t e = (M == 0) ? fold : std::min<int64_t>(fold, b.b[M - 1]);
    if (a >= e) continue;
    const int64_t mid = std::max<int64_t>(a, std::min<int64_t>(e, b.plain));
    const double pf = pairs(a, mid), pp = pairs(mid, e);
    p_out += pf + pp;
    f_out += pf * series_flops(M, mixed) + pp * plain_flops(M);
  }
  if (fold < hi) {
    const double pr = pairs(fold, hi);
    p_out += pr;
    f_out += pr * kFoldFlops;
  }
}

// Plan of the arrival query: tiles of 64R visits; near band lags [1, kf);
// far chunks of K lags from kf, aligned to R.
// The near items go to `near` and the far items to `far`, both in planning
// order.  Pair and flop counts (for the profiler) are formed only if `count`.
// With j1 >= 0 only the tiles holding visits [j0, j1) get items (tile_slots
// keeps one entry per tile of the scan).  near_piece > 0 cuts the near band
// into pieces of that many lags, each a work item with its own slot (slots
// 0 .. np-1; the far chunks follow), so that a short range still has
// enough items; every piece is planned for every near tile, empty ones
// included, so that each slot a visit sums is written.
void plan_arrival(const dd_scan* s, bool mixed, int R, int RN, int K, ArrivalPlan& P,
                  std::vector<ArrItem>& near, std::vector<ArrItem>& far,
                  std::vector<int32_t>& tile_slots, bool count, int64_t j0 = 0,
                  int64_t j1 = -1, int64_t near_piece = 0) {
  const int T = 64 * R, TN = 64 * RN;
  const int64_t V = s->V;
  const double a_max = (double)(s->desc.nx - 1) * (s->desc.nx - 1) +
                       (double)(s->desc.ny - 1) * (s->desc.ny - 1);
  const double thr = mixed ? (double)kThr32 : kThr64;
  const double cull = mixed ? kCullX32 : kCullX64;
  int64_t kf = first_row_below(thr, a_max, cull, 0.0, s->kappa, s->s2, 1, V);
  kf = 1 + (kf - 1 + R - 1) / R * R;
  if (kf > V) kf = V + 1;  // every lag is in the near band
  P.bounds = degree_bounds(a_max, 0.0, s->kappa, s->s2, kf, R, mixed);
  if (mixed) lean_bounds(P.bounds, a_max, s->kappa, s->s2, kf, R);
  P.near_pairs = P.near_flops = P.far_pairs = P.far_flops = 0;
  const int64_t n_tiles = (V + T - 1) / T;
  const int64_t piece = near_piece > 0 ? near_piece : std::max<int64_t>(1, kf - 1);
  const int np = (int)std::max<int64_t>(1, (kf - 1 + piece - 1) / piece);
  near.clear();
  far.clear();
  tile_slots.assign(n_tiles, np);
  if (j1 < 0) j1 = V;
  int S = np;
  for (int64_t t = j0 / T; t < n_tiles && t * T < j1; ++t) {
    const int64_t J0 = t * T;
    const int64_t maxlag = std::min<int64_t>(J0 + T - 1, V - 1);
    const int64_t jend = std::min<int64_t>(J0 + T, V);
    int c = 0;
    if (maxlag >= kf) {
      const int64_t span_end = kf + (maxlag + 1 - kf + R - 1) / R * R;
      for (int64_t lo = kf; lo < span_end; lo += K, ++c) {
        const int64_t hi = std::min<int64_t>(lo + K, span_end);
        const int edge = (hi - 1 > J0) ? kItemEdge : 0;
        far.push_back(ArrItem{(int32_t)t, (int32_t)lo, (int32_t)hi, (np + c) | edge});
        if (count)
          count_segments(P.bounds, lo, hi, mixed,
                         [&](int64_t a, int64_t e) { return arrival_pairs(J0, jend, a, e); },
                         P.far_pairs, P.far_flops);
      }
    }
    tile_slots[t] = np + c;
    S = std::max(S, np + c);
  }
  // near band: tiles of 64 RN visits, lags [1, kf) in np pieces, slots 0 .. np-1
  for (int64_t t = j0 / TN; t < (V + TN - 1) / TN && t * TN < j1; ++t) {
    const int64_t J0 = t * TN;
    const int64_t maxlag = std::min<int64_t>(J0 + TN - 1, V - 1);
    for (int p = 0; p < np; ++p) {
      const int64_t lo = 1 + (int64_t)p * piece;
      const int64_t hi = std::min<int64_t>(kf, lo + piece);
      const int64_t nhi = std::max<int64_t>(lo, std::min<int64_t>(hi, maxlag + 1));
      near.push_back(ArrItem{(int32_t)t, (int32_t)lo, (int32_t)nhi, p | kItemNear});
      if (count) {
        const double np_ = arrival_pairs(J0, std::min<int64_t>(J0 + TN, V), lo, nhi);
        P.near_pairs += np_;
        P.near_flops += np_ * series_flops(mixed ? kMNear32 : kM64, mixed);
      }
    }
  }
  P.R = R;
  P.RN = RN;
  P.K = K;
  P.mixed = mixed;
  P.V = V;
  P.n_near = (int)near.size();
  P.n_far = (int)far.size();
  P.S = S;
}

// Lags per far work item: the tuned value, raised so that no tile has more
// than 64 far slots (bounds the partial buffer at 65 V doubles).
int arrival_K(int64_t V, int R, bool mixed) {
  int K = mixed ? tune().arr_K_mixed : tune().arr_K_f64;
  const int64_t need = (V + 63) / 64;
  if (need > K) K = (int)std::min<int64_t>(need, 1 << 28);
  return std::max(R, (K + R - 1) / R * R);
}

// Order of the far items for the per-scan arrival kernel, where wave w of
// block b takes item 4b + w and blocks are dealt to the 8 XCDs round robin
// (block b on XCD b mod 8, each XCD with its own L2).  Items of one lag
// chunk read the same lag rows, and items of adjacent tiles in one chunk
// read overlapping position windows; so the chunks are dealt to the XCDs by
// work (largest first onto the least loaded XCD), each XCD's items are kept
// chunk by chunk in tile order, and the item list interleaves the XCDs'
// queues four items at a time.  Every item writes its own partial slot, so
// the order changes no result.
void order_far_for_xcds(std::vector<ArrItem>& far) {
  constexpr int kX = 8, kW = 4;
  std::map<int32_t, std::vector<ArrItem>> chunks;  // n_lo -> items
  for (const ArrItem& it : far) chunks[it.n_lo].push_back(it);
  std::vector<std::pair<double, int32_t>> work;  // (work, n_lo)
  for (auto& kv : chunks) {
    double w = 0;
    for (const ArrItem& it : kv.second) w += (double)(it.n_hi - it.n_lo);
    std::stable_sort(kv.second.begin(), kv.second.end(),
                     [](const ArrItem& a, const ArrItem& b) { return a.tile < b.tile; });
    work.push_back({w, kv.first});
  }
  std::stable_sort(work.begin(), work.end(),
                   [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
                     return a.first > b.first;
                   });
  std::vector<std::vector<ArrItem>> q(kX);
  std::vector<double> load(kX, 0.0);
  for (const auto& w : work) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += w.first;
    const auto& v = chunks[w.second];
    q[x].insert(q[x].end(), v.begin(), v.end());
  }
  std::vector<size_t> pos(kX, 0);
  std::vector<ArrItem> out;
  out.reserve(far.size());
  for (size_t b = 0; out.size() < far.size(); ++b) {
    int x = (int)(b % kX);
    if (pos[x] >= q[x].size()) {  // this XCD's queue is done: lend it the fullest one's items
      size_t best = 0;
      for (int y = 0; y < kX; ++y)
        if (q[y].size() - pos[y] > best) best = q[y].size() - pos[y], x = y;
    }
    for (int k = 0; k < kW && pos[x] < q[x].size(); ++k) out.push_back(q[x][pos[x]++]);
  }
  far.swap(out);
}

dd_status run_arrival(dd_scan* s, bool mixed, double* out_dev, const OutFlag& fl, hipStream_t st) {
  dd_status rc = s->prepare(st);
  if (rc != DD_OK) return rc;
  ProfToken tr = prof_begin("lag_rows", st);
  rc = build_int_rows(s, st);
  if (rc != DD_OK) return rc;
  prof_end(tr, st, 0, 0);
  const int R = mixed ? tune().arr_R_mixed : tune().arr_R_f64;
  const int RN = mixed ? tune().arr_RN_mixed : tune().arr_RN_f64;
  const int K = arrival_K(s->V, R, mixed);
  ArrivalPlan& P = s->arr_plan;
  if (P.V != s->V || P.R != R || P.RN != RN || P.K != K || P.mixed != mixed) {
    std::vector<ArrItem> items, far;
    std::vector<int32_t> tile_slots;
    plan_arrival(s, mixed, R, RN, K, P, items, far, tile_slots, true);
    auto longer = [](const ArrItem& a, const ArrItem& b) {
      return (a.n_hi - a.n_lo) > (b.n_hi - b.n_lo);
    };
    std::stable_sort(items.begin(), items.end(), longer);
    order_far_for_xcds(far);
    items.insert(items.end(), far.begin(), far.end());  // near items first
    rc = upload(s->items, items, st);
    if (rc != DD_OK) return rc;
    rc = upload(s->aux, tile_slots, st);
    if (rc != DD_OK) return rc;
  }
  DD_HIP(s->partial.ensure(sizeof(double) * (size_t)P.S * (size_t)s->V), "device allocation");
  ArrivalLaunch L{};
  L.pos = mixed ? (const void*)(s->pos32.as<float2>() + kPosPad)
                : (const void*)(s->pos64.as<double2>() + kPosPad);
  L.pos4 = s->pos4.as<float4>() + kPosPad;
  L.rows64 = s->rows64.as<double>();
  L.rows32 = s->rows32.as<float>();
  L.V = s->V;
  L.bounds = P.bounds;
  L.partial = s->partial.as<double>();
  L.pstride = s->V;
  L.pj0 = 0;
  L.R = R;
  L.mixed = mixed;
  L.items = s->items.as<ArrItem>();
  L.n_items = P.n_near;
  L.near = true;
  L.R = RN;
  ProfToken tn = prof_begin("arrival_near", st);
  DD_HIP(launch_arrival(L, st), "arrival near-band launch");
  prof_end(tn, st, P.near_pairs, P.near_flops);
  L.items = s->items.as<ArrItem>() + P.n_near;
  L.n_items = P.n_far;
  L.near = false;
  L.R = R;
  ProfToken tf = prof_begin("arrival_far", st);
  DD_HIP(launch_arrival(L, st), "arrival far-region launch");
  prof_end(tf, st, P.far_pairs, P.far_flops);
  ProfToken tq = prof_begin("reduce", st);
  DD_HIP(launch_reduce_arrival(s->partial.as<double>(), s->aux.as<int32_t>(), s->V, 0, 64 * R,
                               s->pref, 0, s->V, out_dev, fl, st),
         "arrival reduce launch");
  prof_end(tq, st, 0, 0);
  return DD_OK;
}

struct PinnedBuf {
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

// Staging of a visit range's plan: one pinned buffer per thread, copied to
// the device asynchronously; the next range query on the thread waits for
// that copy (`copied`) before it rewrites the buffer.
struct RangeStage {
  PinnedBuf host;
  hipEvent_t copied = nullptr;  // kept until the process ends
  bool pending = false;
};
static thread_local RangeStage g_range;

}  // namespace

// Arrival at the visits [j0, j1) only (streaming: the visits just made).
// Only the tiles holding them are planned.  The partial sums keep only the
// columns of the range's tiles, so the lag chunks can be short: about 8192
// far items over the range's tiles, and the near band in pieces of 16 lags.
// The plan is a pure function of the scan, the range, the precision and the
// tuned tile shapes, so every entry point that runs it gives the same
// results bit for bit.
void dd::plan_range(const dd_scan* s, bool mixed, int64_t j0, int64_t j1, bool count,
                    RangePlan& rp) {
  const int R = mixed ? tune().arr_R_mixed : tune().arr_R_f64;
  const int RN = mixed ? tune().arr_RN_mixed : tune().arr_RN_f64;
  const int64_t T = 64 * R, TN = 64 * RN;
  rp.pj0 = std::min(j0 / T * T, j0 / TN * TN);
  const int64_t pend = std::max((j1 + T - 1) / T * T, (j1 + TN - 1) / TN * TN);
  rp.pstride = pend - rp.pj0;
  const int64_t tiles = (j1 - 1) / T - j0 / T + 1;
  int64_t K64 = std::max<int64_t>(64, (tiles * j1 + 8191) / 8192);
  const int K = (int)std::min<int64_t>((K64 + R - 1) / R * R, 1 << 28);
  plan_arrival(s, mixed, R, RN, K, rp.P, rp.items, rp.far, rp.tile_slots, count, j0, j1, 16);
  auto longer = [](const ArrItem& a, const ArrItem& b) {
    return (a.n_hi - a.n_lo) > (b.n_hi - b.n_lo);
  };
  std::stable_sort(rp.items.begin(), rp.items.end(), longer);
  std::stable_sort(rp.far.begin(), rp.far.end(), longer);
  rp.items.insert(rp.items.end(), rp.far.begin(), rp.far.end());  // near items first
}

// Launches of a planned range whose items, tile slots and partial sums are
// at the given device addresses (rows and positions resident).
dd_status dd::launch_range(dd_scan* s, bool mixed, const RangePlan& rp, int64_t j0, int64_t j1,
                           const ArrItem* d_items, const int32_t* d_slots, double* d_partial,
                           double* out_dev, const OutFlag& fl, hipStream_t st, bool profile) {
  const ArrivalPlan& P = rp.P;
  ArrivalLaunch L{};
  L.pos = mixed ? (const void*)(s->pos32.as<float2>() + kPosPad)
                : (const void*)(s->pos64.as<double2>() + kPosPad);
  L.pos4 = s->pos4.as<float4>() + kPosPad;
  L.rows64 = s->rows64.as<double>();
  L.rows32 = s->rows32.as<float>();
  L.V = s->V;
  L.bounds = P.bounds;
  L.partial = d_partial;
  L.pstride = rp.pstride;
  L.pj0 = rp.pj0;
  L.mixed = mixed;
  L.range = true;
  L.items = d_items;
  L.n_items = P.n_near;
  L.near = true;
  L.R = P.RN;
  ProfToken tn = profile ? prof_begin("arrival_near", st) : ProfToken{};
  DD_HIP(launch_arrival(L, st), "arrival near-band launch");
  if (profile) prof_end(tn, st, P.near_pairs, P.near_flops);
  L.items = d_items + P.n_near;
  L.n_items = P.n_far;
  L.near = false;
  L.R = P.R;
  ProfToken tf = profile ? prof_begin("arrival_far", st) : ProfToken{};
  DD_HIP(launch_arrival(L, st), "arrival far-region launch");
  if (profile) prof_end(tf, st, P.far_pairs, P.far_flops);
  ProfToken tq = profile ? prof_begin("reduce", st) : ProfToken{};
  DD_HIP((P.S > 64 ? launch_reduce_arrival_wide : launch_reduce_arrival)(
             d_partial, d_slots, rp.pstride, rp.pj0, 64 * P.R, s->pref, j0, j1 - j0, out_dev, fl,
             st),
         "arrival reduce launch");
  if (profile) prof_end(tq, st, 0, 0);
  return DD_OK;
}

namespace {

dd_status run_arrival_range(dd_scan* s, bool mixed, int64_t j0, int64_t j1, double* out_dev,
                            const OutFlag& fl, hipStream_t st) {
  dd_status rc = s->prepare(st);
  if (rc != DD_OK) return rc;
  rc = build_int_rows(s, st);
  if (rc != DD_OK) return rc;
  if (j1 <= j0) return DD_OK;
  static thread_local RangePlan rp;  // host vectors reused between calls
  plan_range(s, mixed, j0, j1, prof_on(), rp);
  const ArrivalPlan& P = rp.P;
  const size_t bi = sizeof(ArrItem) * rp.items.size(), bt = sizeof(int32_t) * rp.tile_slots.size();
  DD_HIP(s->aux2.ensure(std::max<size_t>(bi, 16)), "device allocation");
  DD_HIP(s->aux3.ensure(std::max<size_t>(bt, 16)), "device allocation");
  RangeStage& G = g_range;
  if (G.pending) DD_HIP(hipEventSynchronize(G.copied), "event synchronize");
  G.pending = false;
  DD_HIP(G.host.ensure(bi + bt), "pinned host allocation");
  if (bi) std::memcpy(G.host.p, rp.items.data(), bi);
  if (bt) std::memcpy((char*)G.host.p + bi, rp.tile_slots.data(), bt);
  if (!G.copied) DD_HIP(hipEventCreateWithFlags(&G.copied, hipEventDisableTiming), "event creation");
  if (bi) DD_HIP(hipMemcpyAsync(s->aux2.p, G.host.p, bi, hipMemcpyHostToDevice, st),
                 "host-to-device copy");
  if (bt) DD_HIP(hipMemcpyAsync(s->aux3.p, (char*)G.host.p + bi, bt, hipMemcpyHostToDevice, st),
                 "host-to-device copy");
  DD_HIP(hipEventRecord(G.copied, st), "event record");
  G.pending = true;
  DD_HIP(s->partial.ensure(sizeof(double) * (size_t)P.S * (size_t)rp.pstride), "device allocation");
  return launch_range(s, mixed, rp, j0, j1, s->aux2.as<ArrItem>(), s->aux3.as<int32_t>(),
                      s->partial.as<double>(), out_dev, fl, st, true);
}

// Map query.  Times are snapped to a dwell boundary when within 8 ulp.
struct MapGroup {
  double f;
  int64_t n_first, n_last;  // rows needed
  int64_t alloc_off;        // first row in the call's row buffer
  int64_t kf;
  DegreeBounds bounds;
};

struct RowJob {
  int64_t n_first, count, off;
  double f;
};

struct MapPlan {
  std::vector<MapItem> items;     // near items first, each kind longest first
  std::vector<MapTime> times;
  std::vector<RowJob> jobs;       // rows to build (none when int_rows is used)
  int64_t total_rows = 0, slots = 0, npix = 0;
  double X0 = 0, Y0 = 0, DX = 0, DY = 0;
  double pairs = 0, flops = 0;
  int R = 1;
  bool lattice = false;
};

// Pixel coordinates (pitch units) are multiples of 2^-q for some q <= 8 and
// small enough that |e|^2 + |p|^2 stays an exact single-precision value.
bool grid_is_lattice(double X0, double Y0, double DX, double DY, int w, int h, int nx, int ny) {
  for (int q = 0; q <= 8; ++q) {
    const double sc = std::ldexp(1.0, q);
    bool ok = true;
    for (double v : {X0, Y0, DX, DY}) ok = ok && std::rint(v * sc) == v * sc;
    if (!ok) continue;
    const double ex = std::max(std::fabs(X0), std::fabs(X0 + (w - 1) * DX));
    const double ey = std::max(std::fabs(Y0), std::fabs(Y0 + (h - 1) * DY));
    const double pe = (double)(nx - 1) * (nx - 1) + (double)(ny - 1) * (ny - 1);
    const double bound = (ex * ex + ey * ey + pe) * sc * sc;
    return bound < 16777216.0 && (ex + nx) * sc < 4096.0 && (ey + ny) * sc < 4096.0;
  }
  return false;
}

// Plans a map query.  With int_rows, every time must lie on a dwell boundary
// at or before the end of the scan, and rows are taken from the scan's
// integer-lag table (row n at offset n) instead of a per-call table.
void plan_map(const dd_scan* s, const dd_grid* g, const double* t_s, int32_t n_t, bool mixed,
              int R, int64_t Kmap, bool int_rows, MapPlan& P, bool sort_items = true,
              bool count = true) {
  const int64_t npix = (int64_t)g->w * g->h;
  const double p = s->desc.pitch_m;
  P.X0 = g->x0_m / p;
  P.Y0 = g->y0_m / p;
  P.DX = g->dx_m / p;
  P.DY = g->dy_m / p;
  P.npix = npix;
  P.R = R;
  const int T = 64 * R;
  const int64_t n_tiles = (npix + T - 1) / T;
  // largest squared distance between any pixel and any probe (bounding boxes)
  const double xa = P.X0, xb = P.X0 + (g->w - 1) * P.DX, ya = P.Y0, yb = P.Y0 + (g->h - 1) * P.DY;
  const double mx = std::max({std::fabs(xa), std::fabs(xb), std::fabs(xa - (s->desc.nx - 1)),
                              std::fabs(xb - (s->desc.nx - 1))});
  const double my = std::max({std::fabs(ya), std::fabs(yb), std::fabs(ya - (s->desc.ny - 1)),
                              std::fabs(yb - (s->desc.ny - 1))});
  const double a_max = mx * mx + my * my;
  const double thr = mixed ? (double)kThr32 : kThr64;
  P.lattice = grid_is_lattice(P.X0, P.Y0, P.DX, P.DY, g->w, g->h, s->desc.nx, s->desc.ny);

  std::vector<MapTime>& times = P.times;
  times.assign(n_t, MapTime{});
  std::vector<int> tgroup(n_t);
  std::vector<MapGroup> groups;
  std::map<double, int> gid;
  std::vector<int64_t> nlo(n_t);
  for (int m = 0; m < n_t; ++m) {
    double th = t_s[m] / s->tau_v;
    const double r = std::rint(th);
    if (std::fabs(th - r) <= 8.0 * 2.220446049250313e-16 * std::max(1.0, std::fabs(th))) th = r;
    const double K = std::floor(th);
    const double f = th - K;
    times[m].K = (int64_t)K;
    times[m].n_min = (f == 0.0) ? 1 : 0;
    nlo[m] = std::max<int64_t>(times[m].n_min, times[m].K - s->V + 1);
    auto it = gid.find(f);
    int gi;
    if (it == gid.end()) {
      gi = (int)groups.size();
      gid[f] = gi;
      groups.push_back(MapGroup{f, nlo[m], times[m].K, 0, 0, {}});
    } else {
      gi = it->second;
      groups[gi].n_first = std::min(groups[gi].n_first, nlo[m]);
      groups[gi].n_last = std::max(groups[gi].n_last, times[m].K);
    }
    tgroup[m] = gi;
  }
  // Row storage per group; groups whose span is very wide get per-time rows.
  P.total_rows = 0;
  P.jobs.clear();
  for (auto& G : groups) {
    G.kf = first_row_below(thr, a_max, mixed ? kCullX32 : kCullX64, G.f, s->kappa, s->s2, 1,
                           std::max<int64_t>(G.n_last, 1));
    G.bounds = degree_bounds(a_max, G.f, s->kappa, s->s2, G.kf, 1, mixed);
    const int64_t span = std::max<int64_t>(0, G.n_last - G.n_first + 1);
    if (int_rows) {
      G.alloc_off = 0;
    } else if (span <= 4 * s->V + 4096) {
      G.alloc_off = P.total_rows;
      if (span > 0) P.jobs.push_back(RowJob{G.n_first, span, P.total_rows, G.f});
      P.total_rows += span;
    } else {
      G.alloc_off = -1;
    }
  }
  for (int m = 0; m < n_t; ++m) {
    const MapGroup& G = groups[tgroup[m]];
    if (int_rows) {
      times[m].row_base = 0;
    } else if (G.alloc_off >= 0) {
      times[m].row_base = G.alloc_off - G.n_first;
    } else {
      const int64_t span = std::max<int64_t>(0, times[m].K - nlo[m] + 1);
      times[m].row_base = P.total_rows - nlo[m];
      if (span > 0) P.jobs.push_back(RowJob{nlo[m], span, P.total_rows, G.f});
      P.total_rows += span;
    }
    times[m].bounds = G.bounds;
  }
  // Items and slots.
  int64_t Kc = Kmap;
  int64_t far_total = 0;
  for (int m = 0; m < n_t; ++m) {
    const int64_t kf = std::max<int64_t>(groups[tgroup[m]].kf, nlo[m]);
    far_total += std::max<int64_t>(0, times[m].K + 1 - kf);
  }
  // A small map splits its far lags into shorter chunks (down to 512) until it
  // alone yields about 64 work items of 256 pixels, so that a call holding few
  // small maps still spreads over the chip.  The chunk length depends only on
  // this map (grid and times), never on the rest of a batched call, so batched
  // and single-map results stay the same bit for bit.
  const int64_t units = (npix + 255) / 256;
  while (Kc > 512 && units * ((far_total + Kc - 1) / Kc) < 64) Kc /= 2;
  // keep partials below ~1 GiB
  const int64_t cap_slots = std::max<int64_t>(n_t * 2, (1LL << 27) / std::max<int64_t>(npix, 1));
  while (far_total / Kc + n_t > cap_slots) Kc *= 2;
  std::vector<MapItem> near, far;
  int64_t slot_base = 0;
  P.pairs = P.flops = 0;
  for (int m = 0; m < n_t; ++m) {
    const int64_t K = times[m].K;
    const int64_t kf = std::max<int64_t>(groups[tgroup[m]].kf, nlo[m]);
    const int64_t near_hi = std::max<int64_t>(nlo[m], std::min<int64_t>(kf, K + 1));
    // The near band is one work item per tile; a small map splits it into up
    // to 64 / units pieces of at least 32 lags (slots 0 .. np-1), by the same
    // per-map rule as the far chunks.
    const int64_t near_len = near_hi - nlo[m];
    const int64_t np = std::max<int64_t>(
        1, std::min<int64_t>((64 + units - 1) / units, near_len / 32));
    for (int64_t j = 0; j < np; ++j) {
      const int64_t a = nlo[m] + near_len * j / np, e = nlo[m] + near_len * (j + 1) / np;
      for (int64_t t = 0; t < n_tiles; ++t)
        near.push_back(MapItem{(int32_t)t, m, (int32_t)a, (int32_t)e, (int32_t)j, 1, 0, 0});
    }
    int c = 0;
    if (count) {
      P.pairs += (double)npix * (double)(near_hi - nlo[m]);
      P.flops += (double)npix * (double)(near_hi - nlo[m]) *
                 series_flops(mixed ? kMNear32 : kM64, mixed);
    }
    for (int64_t lo = std::max(kf, nlo[m]); lo <= K; lo += Kc, ++c) {
      const int64_t hi = std::min<int64_t>(lo + Kc, K + 1);
      for (int64_t t = 0; t < n_tiles; ++t)
        far.push_back(MapItem{(int32_t)t, m, (int32_t)lo, (int32_t)hi, (int32_t)np + c, 0, 0, 0});
      if (count)
        count_segments(times[m].bounds, lo, hi, mixed,
                       [&](int64_t a, int64_t e) { return (double)npix * (double)(e - a); },
                       P.pairs, P.flops);
    }
    times[m].slot_base = slot_base;
    times[m].n_slots = (int32_t)np + c;
    slot_base += np + c;
  }
  P.slots = slot_base;
  auto longer = [](const MapItem& a, const MapItem& b) {
    return (a.n_hi - a.n_lo) > (b.n_hi - b.n_lo);
  };
  if (sort_items) {
    std::stable_sort(near.begin(), near.end(), longer);
    std::stable_sort(far.begin(), far.end(), longer);
  }
  P.items = near;
  P.items.insert(P.items.end(), far.begin(), far.end());
}

dd_status run_map(dd_scan* s, const dd_grid* g, const double* t_s, int32_t n_t, bool mixed,
                  double* out_dev, const OutFlag& fl, hipStream_t st) {
  dd_status rc = s->prepare(st);
  if (rc != DD_OK) return rc;
  // The FP32 bulk takes the squared distance a exactly only when pixels and
  // probes share a dyadic lattice.  Off it, a rounded a costs a term about
  // x1 * 1e-7 of relative accuracy, above the mixed bound where distant
  // probes (large x1) dominate a pixel, so such grids run on the FP64 kernels.
  if (mixed) {
    const double p = s->desc.pitch_m;
    if (!grid_is_lattice(g->x0_m / p, g->y0_m / p, g->dx_m / p, g->dy_m / p, g->w, g->h,
                         s->desc.nx, s->desc.ny))
      mixed = false;
  }
  const int R = mixed ? tune().map_R_mixed : tune().map_R_f64;
  MapPlan P;
  plan_map(s, g, t_s, n_t, mixed, R, tune().map_K, false, P);
  DD_HIP(s->maprows64.ensure(sizeof(double) * kRow64 * std::max<int64_t>(P.total_rows, 1)),
         "device allocation");
  DD_HIP(s->maprows32.ensure(sizeof(float) * kRow32 * std::max<int64_t>(P.total_rows, 1)),
         "device allocation");
  ProfToken trw = prof_begin("lag_rows", st);
  for (const RowJob& j : P.jobs)
    DD_HIP(launch_lag_rows(j.n_first, j.count, j.f, s->kappa, s->s2, gl_nodes(),
                           s->maprows64.as<double>() + j.off * kRow64,
                           s->maprows32.as<float>() + j.off * kRow32, st),
           "lag-row kernel launch");
  prof_end(trw, st, 0, 0);
  rc = upload(s->aux2, P.items, st);
  if (rc != DD_OK) return rc;
  rc = upload(s->aux3, P.times, st);
  if (rc != DD_OK) return rc;
  DD_HIP(s->partial.ensure(sizeof(double) * (size_t)P.slots * (size_t)P.npix),
         "device allocation");
  MapLaunch L{};
  L.pos = mixed ? (const void*)(s->pos32.as<float2>() + kPosPad)
                : (const void*)(s->pos64.as<double2>() + kPosPad);
  L.pos4 = s->pos4.as<float4>() + kPosPad;
  L.lattice = P.lattice;
  L.rows64 = s->maprows64.as<double>();
  L.rows32 = s->maprows32.as<float>();
  L.items = s->aux2.as<MapItem>();
  L.n_items = (int32_t)P.items.size();
  L.times = s->aux3.as<MapTime>();
  L.X0 = P.X0; L.Y0 = P.Y0; L.DX = P.DX; L.DY = P.DY;
  L.W = g->w; L.H = g->h;
  L.partial = s->partial.as<double>();
  L.R = R;
  L.mixed = mixed;
  ProfToken tm = prof_begin("map", st);
  DD_HIP(launch_map(L, st), "map launch");
  prof_end(tm, st, P.pairs, P.flops);
  ProfToken tq = prof_begin("reduce", st);
  DD_HIP(launch_reduce_map(s->partial.as<double>(), s->aux3.as<MapTime>(), n_t, P.npix, s->pref,
                           out_dev, fl, st),
         "map reduce launch");
  prof_end(tq, st, 0, 0);
  return DD_OK;
}

// A query call on one scan.  It waits for the handle's last call if that ran
// on another stream, takes a fresh non-finite flag, runs into `out` (device)
// or into the handle's staging buffer and then host memory, and records its
// event.  With host outputs it synchronizes and returns DD_EDEVICE if an
// output value was not finite; with device outputs dd_scan_check reports
// that later.
}  // namespace

dd_status dd::begin_call(dd_scan* s, hipStream_t st, OutFlag& fl) {
  dd_status rc = s->prepare(st);
  if (rc != DD_OK) return rc;
  rc = s->wait_last(st);
  if (rc != DD_OK) return rc;
  return s->next_flag(st, fl);
}

namespace {

template <typename F>
dd_status deliver(dd_scan* s, size_t n, double* out, int32_t on_device, hipStream_t st, F&& run) {
  OutFlag fl;
  dd_status rc = begin_call(s, st, fl);
  if (rc != DD_OK) return rc;
  if (on_device) {
    rc = run(out, fl);
    if (rc != DD_OK) return rc;
    return s->record_last(st);
  }
  DD_HIP(s->tmp_out.ensure(sizeof(double) * std::max<size_t>(n, 1)), "device allocation");
  rc = run(s->tmp_out.as<double>(), fl);
  if (rc != DD_OK) return rc;
  if (n) DD_HIP(hipMemcpyAsync(out, s->tmp_out.p, sizeof(double) * n, hipMemcpyDeviceToHost, st),
                "device-to-host copy");
  rc = s->record_last(st);
  if (rc != DD_OK) return rc;
  return s->check_flag(st, fl.seq);
}


// ---------------------------------------------------------------------------
// Batched solve: every scan's arrival and final-map items in one persistent
// launch, then one fixed-order reduction launch.
// Scratch of the batched solve, shared by the calls of one host thread.  A
// call may run on another stream than the previous one (the surrogate runs
// its exact judge on a second stream): each call records `done` after its
// last launch and the next call makes its stream wait for it before its
// uploads overwrite the scratch.  (Reallocation is safe: hipFree waits for
// the device.)
// The call's tables (scans, four item lists, reductions, tile slots) travel
// in one pinned host block and one copy; the next call waits for that copy
// (`copied`) before it rewrites the block.

struct BatchScratch {
  DevBuf block, partial, counter, staging;
  PinnedBuf host_block;
  std::vector<BatchScan> h_scans;
  std::vector<BatchItem> h_items, h_near_items, h_map_items, h_map_near_items, h_tmp;
  std::vector<BatchReduce> h_reds;
  std::vector<int32_t> h_slots;
  std::vector<uint64_t> h_ka, h_kb;
  hipEvent_t done = nullptr, copied = nullptr;  // kept until the process ends
  bool pending = false, copy_pending = false;
  // the call's non-finite flag (index: flat output index of the call) and
  // the event each scan of the last call holds as its last call
  DevBuf flag;
  uint64_t seq = 0;
  std::shared_ptr<StreamEvent> ev;
};
static thread_local BatchScratch g_batch;
static thread_local uint64_t g_plan_clock = 0;  // recency of the handles' cached map plans

int64_t item_cost(const BatchItem& a) { return ((int64_t)a.cost_hi << 31) | a.cost_lo; }

// Items longest first.  A stable LSD radix sort on (largest cost - cost):
// equal costs keep their planned order, as with a stable comparison sort, at
// linear cost for the long item lists of a large batch.  The sort runs on
// 8-byte (key, index) words; the items move once at the end.
void sort_longest_first(std::vector<BatchItem>& v, std::vector<BatchItem>& tmp,
                        std::vector<uint64_t>& ka, std::vector<uint64_t>& kb) {
  const size_t n = v.size();
  if (n < 2) return;
  int64_t top = 0;
  for (const BatchItem& a : v) top = std::max(top, item_cost(a));
  if (top == 0) return;
  constexpr int kBits = 11;
  constexpr uint64_t kMask = (1u << kBits) - 1;
  // keys above 2^32 - 1 are clamped: the order among items that long is
  // then their planned order, which an LPT schedule does not need to refine
  const uint64_t span = std::min<uint64_t>((uint64_t)top, 0xffffffffULL);
  ka.resize(n);
  kb.resize(n);
  for (size_t i = 0; i < n; ++i) {
    const uint64_t key = std::min<uint64_t>((uint64_t)(top - item_cost(v[i])), span);
    ka[i] = (key << 32) | (uint64_t)i;
  }
  size_t count[(size_t)1 << kBits];
  for (int shift = 32; shift < 64 && (span >> (shift - 32)) != 0; shift += kBits) {
    std::fill(count, count + ((size_t)1 << kBits), 0);
    for (size_t i = 0; i < n; ++i) ++count[(ka[i] >> shift) & kMask];
    size_t sum = 0;
    for (size_t& c : count) {
      const size_t here = c;
      c = sum;
      sum += here;
    }
    for (size_t i = 0; i < n; ++i) kb[count[(ka[i] >> shift) & kMask]++] = ka[i];
    ka.swap(kb);
  }
  tmp.resize(n);
  for (size_t i = 0; i < n; ++i) tmp[i] = v[ka[i] & 0xffffffffULL];
  v.swap(tmp);
}

}  // namespace

// The probe sub-grid of scan s that sel selects (sel.w < 0: the whole grid).
static MapSel resolve_sel(const dd_scan* s, const MapSel& sel) {
  if (sel.w < 0) return MapSel{0, 0, 1, s->desc.nx, s->desc.ny};
  return sel;
}

// Batched solve; the final map covers the probe sub-grid `sel` of each scan.
dd_status dd::run_batch(dd_scan* const* scans, int32_t n, uint32_t mask, bool mixed,
                        double* const* outs, int32_t on_device, hipStream_t st,
                        const MapSel& sel) {
  for (int32_t k = 0; k < n && sel.w >= 0; ++k) {
    const MapSel q = resolve_sel(scans[k], sel);
    if (q.w < 1 || q.h < 1 || q.step < 1 || q.x0 < 0 || q.y0 < 0 ||
        q.x0 + (int64_t)q.step * (q.w - 1) >= scans[k]->desc.nx ||
        q.y0 + (int64_t)q.step * (q.h - 1) >= scans[k]->desc.ny)
      return fail(DD_EINVAL, "scan %d: probe sub-grid outside its grid", k);
  }
  const int R = mixed ? tune().arr_R_mixed : tune().arr_R_f64;
  const int RN = mixed ? tune().arr_RN_mixed : tune().arr_RN_f64;
  const bool want_arr = (mask & DD_Q_ARRIVAL) != 0, want_map = (mask & DD_Q_FINAL_AT_PROBES) != 0;
  // map tile width: the tuned one, narrowed while a narrower tile still covers
  // the largest map of the call (a one-row map fills one 64-pixel tile)
  int RM = mixed ? tune().map_R_mixed : tune().map_R_f64;
  if (want_map) {
    int64_t most = 0;
    for (int32_t k = 0; k < n; ++k) {
      const MapSel q = resolve_sel(scans[k], sel);
      most = std::max<int64_t>(most, (int64_t)q.w * q.h);
    }
    while (RM > 1 && 64LL * (RM / 2) >= most) RM /= 2;
    // A small call (the surrogate's fallback) yields too few far items to
    // fill the chip with 4-pixel tiles: below ~24k items (about 100 maps of
    // 64x64) 2-pixel tiles, below ~6k 1-pixel tiles (rows staged in LDS) are
    // faster (measured on 64x64 final maps).  The tile width does not change
    // any pixel's sum.  The estimate takes every lag as far and the chunk
    // length of plan_map.
    if (RM == 4) {
      double est = 0;
      for (int32_t k = 0; k < n; ++k) {
        const MapSel q = resolve_sel(scans[k], sel);
        const int64_t npix = (int64_t)q.w * q.h, V = scans[k]->V;
        const int64_t units = (npix + 255) / 256;
        int64_t Kc = tune().map_K;
        while (Kc > 512 && units * ((V + Kc - 1) / Kc) < 64) Kc /= 2;
        est += (double)((npix + 255) / 256) * (double)((V + Kc - 1) / Kc);
      }
      if (est < 6144)
        RM = 1;
      else if (est < 24576)
        RM = 2;
    }
  }
  // host tables, kept by the thread between calls (no reallocation per call)
  BatchScratch& W = g_batch;
  const bool count = prof_on();
  std::vector<BatchScan>& bs = W.h_scans;
  std::vector<BatchItem>& items = W.h_items;
  std::vector<BatchItem>& near_items = W.h_near_items;
  std::vector<BatchItem>& map_items = W.h_map_items;
  std::vector<BatchItem>& map_near_items = W.h_map_near_items;
  std::vector<BatchReduce>& reds = W.h_reds;
  std::vector<int32_t>& all_slots = W.h_slots;
  bs.assign(n, BatchScan{});
  items.clear();
  near_items.clear();
  map_items.clear();
  map_near_items.clear();
  reds.clear();
  all_slots.clear();
  std::vector<int64_t> arr_off(n, 0), map_off(n, 0), slot_off(n, 0), out_off(n, 0);
  int64_t partial_total = 0, out_total = 0;
  double pairs = 0, flops = 0;
  ProfToken trw = prof_begin("lag_rows", st);
  std::vector<OutFlag> scan_flag(n);
  const StreamEvent* waited = nullptr;
  for (int32_t k = 0; k < n; ++k) {
    dd_scan* s = scans[k];
    dd_status rc = s->prepare(st);
    if (rc != DD_OK) return rc;
    // rows (or a pending call) of a scan last used on another stream
    if (s->last && s->last->stream != st && s->last.get() != waited) {
      DD_HIP(hipStreamWaitEvent(st, s->last->ev, 0), "stream wait");
      waited = s->last.get();
    }
    rc = s->next_flag(st, scan_flag[k]);
    if (rc != DD_OK) return rc;
    rc = build_int_rows(s, st);
    if (rc != DD_OK) return rc;
  }
  prof_end(trw, st, 0, 0);
  if (!W.flag.p || W.seq >= kFlagSeqMax) {
    dd_status rc = upload(W.flag, std::vector<unsigned long long>(1, 0ull), st);
    if (rc != DD_OK) return rc;
    W.seq = 0;
  }
  const OutFlag call_flag{W.flag.as<unsigned long long>(), (unsigned long long)++W.seq, 0};
  for (int32_t k = 0; k < n; ++k) {
    dd_scan* s = scans[k];
    BatchScan& B = bs[k];
    B.pos = mixed ? (const void*)(s->pos32.as<float2>() + kPosPad)
                  : (const void*)(s->pos64.as<double2>() + kPosPad);
    B.pos4 = s->pos4.as<float4>() + kPosPad;
    B.rows64 = s->rows64.as<double>();
    B.rows32 = s->rows32.as<float>();
    B.V = s->V;
    B.nx = s->desc.nx;
    B.ny = s->desc.ny;
    const MapSel q = resolve_sel(s, sel);
    B.map_x0 = q.x0;
    B.map_y0 = q.y0;
    B.map_step = q.step;
    B.map_w = q.w;
    B.map_h = q.h;
    out_off[k] = out_total;
    if (want_arr) {
      dd_scan::BatchArrPlan& C = s->barr;
      const int K = arrival_K(s->V, R, mixed);
      if (!(C.ok && C.mixed == mixed && C.R == R && C.RN == RN && C.K == K &&
            (C.counted || !count))) {
        ArrivalPlan AP;
        C.ok = false;
        plan_arrival(s, mixed, R, RN, K, AP, C.near, C.far, C.tile_slots, count);
        C.mixed = mixed;
        C.R = R;
        C.RN = RN;
        C.K = K;
        C.S = AP.S;
        C.bounds = AP.bounds;
        C.pairs = AP.near_pairs + AP.far_pairs;
        C.flops = AP.near_flops + AP.far_flops;
        C.counted = count;
        C.ok = true;
      }
      const std::vector<ArrItem>& an = C.near;
      const std::vector<ArrItem>& af = C.far;
      B.arr_bounds = C.bounds;
      arr_off[k] = partial_total;
      partial_total += (int64_t)C.S * s->V;
      slot_off[k] = (int64_t)all_slots.size();
      all_slots.insert(all_slots.end(), C.tile_slots.begin(), C.tile_slots.end());
      const double near_w = mixed ? 6.0 : 3.0;  // relative cost of a near pair
      auto add = [&](std::vector<BatchItem>& dst, const std::vector<ArrItem>& src, int kind,
                     double per_lag) {
        for (const ArrItem& a : src) {
          const int64_t c = (int64_t)((double)(a.n_hi - a.n_lo) * per_lag);
          dst.push_back(BatchItem{k, kind, a.tile, a.n_lo, a.n_hi, a.slot_flags,
                                  (int32_t)(c >> 31), (int32_t)(c & 0x7fffffff)});
        }
      };
      add(near_items, an, kBatchArrNear, 64.0 * RN * near_w);
      add(items, af, kBatchArrFar, 64.0 * R);
      reds.push_back(BatchReduce{nullptr, nullptr, 0, 64 * R, s->V, out_total, nullptr, s->pref,
                                 scan_flag[k]});
      out_total += s->V;
      pairs += C.pairs;
      flops += C.flops;
    }
    if (want_map) {
      const double pm = s->desc.pitch_m;
      dd_grid g{q.x0 * pm, q.y0 * pm, q.step * pm, q.step * pm, q.w, q.h};
      const double t_end = (double)s->V * s->tau_v;
      const int64_t Kmap = tune().map_K;
      dd_scan::BatchMapPlan* C = nullptr;
      for (dd_scan::BatchMapPlan& c : s->bmap)
        if (c.ok && c.mixed == mixed && c.R == RM && c.sel.x0 == q.x0 && c.sel.y0 == q.y0 &&
            c.sel.step == q.step && c.sel.w == q.w && c.sel.h == q.h && c.K == Kmap &&
            (c.counted || !count))
          C = &c;
      if (!C) {  // plan, replacing the plan used least recently
        C = s->bmap[0].used <= s->bmap[1].used ? &s->bmap[0] : &s->bmap[1];
        MapPlan MP;
        C->ok = false;
        plan_map(s, &g, &t_end, 1, mixed, RM, Kmap, true, MP, false, count);
        C->mixed = mixed;
        C->R = RM;
        C->sel = q;
        C->K = Kmap;
        C->time = MP.times[0];
        C->slots = MP.slots;
        C->npix = MP.npix;
        C->items.swap(MP.items);
        C->pairs = MP.pairs;
        C->flops = MP.flops;
        C->counted = count;
        C->ok = true;
      }
      C->used = ++g_plan_clock;
      B.map_time = C->time;
      map_off[k] = partial_total;
      partial_total += C->slots * C->npix;
      const double near_w = mixed ? 6.0 : 3.0;
      for (const MapItem& m : C->items) {
        const int64_t tile_pix = std::min<int64_t>(64 * RM, C->npix - (int64_t)m.tile * 64 * RM);
        const double cost = (double)(m.n_hi - m.n_lo) * tile_pix * (m.near ? near_w : 1.0);
        const int64_t c = (int64_t)cost;
        (m.near ? map_near_items : map_items)
            .push_back(BatchItem{k, m.near ? kBatchMapNear : kBatchMapFar, m.tile, m.n_lo, m.n_hi,
                                 m.slot, (int32_t)(c >> 31), (int32_t)(c & 0x7fffffff)});
      }
      OutFlag mf = scan_flag[k];
      mf.base = want_arr ? s->V : 0;  // index into the scan's output
      reds.push_back(BatchReduce{nullptr, nullptr, C->time.n_slots, 0, C->npix, out_total,
                                 nullptr, s->pref, mf});
      out_total += C->npix;
      pairs += C->pairs;
      flops += C->flops;
    }
  }
  if (W.pending) DD_HIP(hipStreamWaitEvent(st, W.done, 0), "stream wait");
  for (std::vector<BatchItem>* v : {&items, &near_items, &map_items, &map_near_items})
    sort_longest_first(*v, W.h_tmp, W.h_ka, W.h_kb);
  // tables: scans, far/near arrival items, far/near map items, reductions, slots
  struct Table {
    const void* src;
    size_t bytes, off;
  };
  Table tab[7] = {{bs.data(), sizeof(BatchScan) * bs.size(), 0},
                  {items.data(), sizeof(BatchItem) * items.size(), 0},
                  {near_items.data(), sizeof(BatchItem) * near_items.size(), 0},
                  {map_items.data(), sizeof(BatchItem) * map_items.size(), 0},
                  {map_near_items.data(), sizeof(BatchItem) * map_near_items.size(), 0},
                  {reds.data(), sizeof(BatchReduce) * reds.size(), 0},
                  {all_slots.data(), sizeof(int32_t) * all_slots.size(), 0}};
  size_t block_bytes = 0;
  for (Table& t : tab) {
    t.off = block_bytes;
    block_bytes += (t.bytes + 255) & ~(size_t)255;
  }
  DD_HIP(W.block.ensure(block_bytes), "device allocation");
  char* blk = (char*)W.block.p;
  DD_HIP(W.partial.ensure(sizeof(double) * (size_t)std::max<int64_t>(partial_total, 1)),
         "device allocation");
  double* part = W.partial.as<double>();
  if (!on_device) DD_HIP(W.staging.ensure(sizeof(double) * (size_t)std::max<int64_t>(out_total, 1)),
                         "device allocation");
  {
    const int32_t* d_slots = (const int32_t*)(blk + tab[6].off);
    size_t r = 0;
    for (int32_t k = 0; k < n; ++k) {
      double* o = on_device ? outs[k] : W.staging.as<double>() + out_off[k];
      if (want_arr) {
        bs[k].arr_partial = part + arr_off[k];
        reds[r].partial = bs[k].arr_partial;
        reds[r].tile_slots = d_slots + slot_off[k];
        reds[r].out = o;
        o += scans[k]->V;
        ++r;
      }
      if (want_map) {
        bs[k].map_partial = part + map_off[k];
        reds[r].partial = bs[k].map_partial;
        reds[r].out = o;
        ++r;
      }
    }
  }
  if (W.copy_pending) DD_HIP(hipEventSynchronize(W.copied), "event synchronize");
  W.copy_pending = false;
  DD_HIP(W.host_block.ensure(block_bytes), "pinned host allocation");
  for (const Table& t : tab)
    if (t.bytes) std::memcpy((char*)W.host_block.p + t.off, t.src, t.bytes);
  if (!W.copied)
    DD_HIP(hipEventCreateWithFlags(&W.copied, hipEventDisableTiming), "event creation");
  DD_HIP(hipMemcpyAsync(blk, W.host_block.p, block_bytes, hipMemcpyHostToDevice, st),
         "host-to-device copy");
  DD_HIP(hipEventRecord(W.copied, st), "event record");
  W.copy_pending = true;
  const BatchScan* d_scans = (const BatchScan*)(blk + tab[0].off);
  DD_HIP(W.counter.ensure(4 * sizeof(int)), "device allocation");
  ProfToken tb = prof_begin("batch", st);
  DD_HIP(launch_batch(d_scans, (const BatchItem*)(blk + tab[1].off), (int32_t)items.size(),
                      W.counter.as<int>(), R, mixed, st),
         "batched launch");
  DD_HIP(launch_batch_near(d_scans, (const BatchItem*)(blk + tab[2].off),
                           (int32_t)near_items.size(), W.counter.as<int>() + 1, RN, mixed, st),
         "batched near-band launch");
  DD_HIP(launch_batch_map(d_scans, (const BatchItem*)(blk + tab[3].off), (int32_t)map_items.size(),
                          W.counter.as<int>() + 2, RM, mixed, false, st),
         "batched map launch");
  DD_HIP(launch_batch_map(d_scans, (const BatchItem*)(blk + tab[4].off),
                          (int32_t)map_near_items.size(), W.counter.as<int>() + 3, RM, mixed, true,
                          st),
         "batched map near-band launch");
  prof_end(tb, st, pairs, flops);
  ProfToken tq = prof_begin("reduce", st);
  DD_HIP(launch_reduce_batch((const BatchReduce*)(blk + tab[5].off), (int32_t)reds.size(),
                             out_total, call_flag, st),
         "batched reduce launch");
  prof_end(tq, st, 0, 0);
  if (!W.done) DD_HIP(hipEventCreateWithFlags(&W.done, hipEventDisableTiming), "event creation");
  DD_HIP(hipEventRecord(W.done, st), "event record");
  W.pending = true;
  // each scan's last call is this one (its flag word is written here)
  if (!W.ev || W.ev.use_count() > 1) {
    auto e = std::make_shared<StreamEvent>();
    DD_HIP(hipEventCreateWithFlags(&e->ev, hipEventDisableTiming), "event creation");
    W.ev = e;
  }
  DD_HIP(hipEventRecord(W.ev->ev, st), "event record");
  W.ev->stream = st;
  for (int32_t k = 0; k < n; ++k) scans[k]->last = W.ev;
  if (!on_device) {
    for (int32_t k = 0; k < n; ++k) {
      const int64_t len = (k + 1 < n ? out_off[k + 1] : out_total) - out_off[k];
      if (len > 0)
        DD_HIP(hipMemcpyAsync(outs[k], W.staging.as<double>() + out_off[k], sizeof(double) * len,
                              hipMemcpyDeviceToHost, st),
               "device-to-host copy");
    }
    int64_t bad = -1;
    dd_status rc = read_flag(W.flag.as<unsigned long long>(), st, call_flag.seq, bad);
    if (rc != DD_OK) return rc;
    if (bad >= 0) {
      const int32_t k = (int32_t)(std::upper_bound(out_off.begin(), out_off.end(), bad) -
                                  out_off.begin()) - 1;
      return fail(DD_EDEVICE, "scan %d: non-finite output value at index %lld of its output", k,
                  (long long)(bad - out_off[k]));
    }
  }
  return DD_OK;
}

dd_status dd_damage_sweep(dd_scan* s, const dd_grid* g, double t0_s, double dt_s, int32_t n_t,
                          dd_precision p, double* out, int32_t out_on_device, void* hip_stream) {
  if (!s || !g || !out) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  if (n_t < 1) return fail(DD_EINVAL, "n_t must be >= 1");
  if (!(std::isfinite(t0_s) && t0_s >= 0)) return fail(DD_EINVAL, "t0 must be finite and >= 0");
  if (!(std::isfinite(dt_s) && dt_s > 0)) return fail(DD_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t0_s + (double)(n_t - 1) * dt_s)) return fail(DD_EINVAL, "last time not finite");
  if (g->w < 1 || g->h < 1) return fail(DD_EINVAL, "grid w and h must be >= 1");
  if ((int64_t)g->w * g->h > (1LL << 30)) return fail(DD_EINVAL, "grid too large");
  for (double v : {g->x0_m, g->y0_m, g->dx_m, g->dy_m})
    if (!std::isfinite(v)) return fail(DD_EINVAL, "grid values must be finite");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t npix = (int64_t)g->w * g->h;
  // times per map call: at most 4096 and at most 2^25 output values (256 MiB)
  const int32_t chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(4096, (1LL << 25) / npix));
  std::vector<double> t(chunk);
  // one call: one flag for all chunks, each chunk's indices offset by its
  // first output
  OutFlag fl;
  dd_status rc = begin_call(s, st, fl);
  if (rc != DD_OK) return rc;
  if (!out_on_device)
    DD_HIP(s->tmp_out.ensure(sizeof(double) * (size_t)chunk * npix), "device allocation");
  for (int32_t k0 = 0; k0 < n_t; k0 += chunk) {
    const int32_t c = std::min(chunk, n_t - k0);
    for (int32_t j = 0; j < c; ++j) t[j] = t0_s + (double)(k0 + j) * dt_s;
    double* o = out_on_device ? out + (size_t)k0 * npix : s->tmp_out.as<double>();
    fl.base = (int64_t)k0 * npix;
    rc = run_map(s, g, t.data(), c, p == DD_MIXED, o, fl, st);
    if (rc != DD_OK) return rc;
    if (!out_on_device) {  // the staging buffer is reused by the next chunk
      DD_HIP(hipMemcpyAsync(out + (size_t)k0 * npix, o, sizeof(double) * (size_t)c * npix,
                            hipMemcpyDeviceToHost, st),
             "device-to-host copy");
      DD_HIP(hipStreamSynchronize(st), "stream synchronize");
    }
  }
  rc = s->record_last(st);
  if (rc != DD_OK) return rc;
  return out_on_device ? DD_OK : s->check_flag(st, fl.seq);
}

dd_status dd_damage_at_probe_arrival_range(dd_scan* s, int64_t j0, int64_t j1, dd_precision p,
                                           double* out, int32_t out_on_device, void* hip_stream) {
  if (!s || (!out && j1 > j0)) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  if (j0 < 0 || j1 < j0 || j1 > s->V)
    return fail(DD_EINVAL, "visit range [%lld, %lld) outside [0, %lld]", (long long)j0,
                (long long)j1, (long long)s->V);
  if (j1 == j0) return DD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  return deliver(s, (size_t)(j1 - j0), out, out_on_device, st, [&](double* o, const OutFlag& fl) {
    return run_arrival_range(s, p == DD_MIXED, j0, j1, o, fl, st);
  });
}

dd_status dd_damage_at_probe_arrival(dd_scan* s, dd_precision p, double* out,
                                     int32_t out_on_device, void* hip_stream) {
  if (!s || !out) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  hipStream_t st = (hipStream_t)hip_stream;
  return deliver(s, (size_t)s->V, out, out_on_device, st,
                 [&](double* o, const OutFlag& fl) { return run_arrival(s, p == DD_MIXED, o, fl, st); });
}

dd_status dd_damage_map(dd_scan* s, const dd_grid* g, const double* t_s, int32_t n_t,
                        dd_precision p, double* out, int32_t out_on_device, void* hip_stream) {
  if (!s || !g || !out || (n_t > 0 && !t_s)) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  if (n_t < 1) return fail(DD_EINVAL, "n_t must be >= 1");
  if (g->w < 1 || g->h < 1) return fail(DD_EINVAL, "grid w and h must be >= 1");
  if ((int64_t)g->w * g->h > (1LL << 30)) return fail(DD_EINVAL, "grid too large");
  for (double v : {g->x0_m, g->y0_m, g->dx_m, g->dy_m})
    if (!std::isfinite(v)) return fail(DD_EINVAL, "grid values must be finite");
  for (int32_t m = 0; m < n_t; ++m)
    if (!std::isfinite(t_s[m]) || t_s[m] < 0) return fail(DD_EINVAL, "time %d invalid", m);
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = (size_t)n_t * g->w * g->h;
  return deliver(s, n, out, out_on_device, st,
                 [&](double* o, const OutFlag& fl) {
                   return run_map(s, g, t_s, n_t, p == DD_MIXED, o, fl, st);
                 });
}

dd_status dd_batch_solve(dd_scan* const* scans, int32_t n, uint32_t query_mask, dd_precision p,
                         double* const* outs, int32_t out_on_device, void* hip_stream) {
  if (n < 1 || !scans || !outs) return fail(DD_EINVAL, "bad batch arguments");
  if ((query_mask & 3u) == 0 || (query_mask & ~3u)) return fail(DD_EINVAL, "bad query mask");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  for (int32_t k = 0; k < n; ++k)
    if (!scans[k] || !outs[k]) return fail(DD_EINVAL, "scan %d or its output is NULL", k);
  return dd::run_batch(scans, n, query_mask, p == DD_MIXED, outs, out_on_device,
                       (hipStream_t)hip_stream, MapSel{});
}

dd_status dd_scan_check(dd_scan* s, int64_t* first_bad) {
  if (first_bad) *first_bad = -1;
  if (!s) return fail(DD_EINVAL, "NULL argument");
  if (s->dev < 0 || s->seq == 0) return DD_OK;
  int cur = 0;
  DD_HIP(hipGetDevice(&cur), "hipGetDevice");
  if (cur != s->dev) return fail(DD_EINVAL, "the scan ran on device %d, not %d", s->dev, cur);
  if (s->last) DD_HIP(hipEventSynchronize(s->last->ev), "event synchronize");
  unsigned long long w = 0;
  DD_HIP(hipMemcpy(&w, s->flag.p, sizeof(w), hipMemcpyDeviceToHost), "device-to-host copy");
  constexpr unsigned long long lim = (1ull << kFlagIndexBits) - 1;
  if ((w >> kFlagIndexBits) != s->seq) return DD_OK;
  const int64_t bad = (int64_t)(lim - (w & lim));
  if (first_bad) *first_bad = bad;
  return fail(DD_EDEVICE, "non-finite output value at index %lld of the scan's last call",
              (long long)bad);
}

dd_status dd_pair_terms(double kappa, double sigma_hat, int64_t n, const double* a,
                        const double* lag, dd_precision p, double* out, void* hip_stream) {
  if (!(std::isfinite(kappa) && kappa > 0 && std::isfinite(sigma_hat) && sigma_hat > 0))
    return fail(DD_EINVAL, "kappa and sigma_hat must be finite and > 0");
  if (n < 0 || (n > 0 && (!a || !lag || !out))) return fail(DD_EINVAL, "bad arrays");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  dd_status rc = ensure_device();
  if (rc != DD_OK) return rc;
  DD_HIP(launch_pair_terms(kappa, 2.0 * sigma_hat * sigma_hat, n, a, lag, p == DD_MIXED,
                           gl_nodes(), out, (hipStream_t)hip_stream),
         "pair-term launch");
  return DD_OK;
}
