// dd_noalloc.hip -- the streaming arrival query without allocation
// (dd_damage_at_probe_arrival_range_noalloc), for callers that cannot
// allocate device memory: code under stream capture, serving loops that
// must not allocate, harnesses that forbid it.
//
// The query's scratch -- work items, partial-sum slots per tile and the
// partial sums themselves -- lives in one static device array per GPU,
// `scratch`, of kScratchBytes.  Every call on a GPU shares it: calls that
// overlap on one GPU (on different streams, or from different threads)
// race on it; calls on one stream are ordered by the stream.  The array
// keeps the last call's contents, and nothing in it needs to start at zero:
// the plan is copied in whole, and every partial-sum slot the reduction
// reads is written by a work item of the same call.  The scan's
// resident tables (positions, lag rows, flag word, event) must already be
// on the device; the call then allocates nothing.  Plan and kernels are
// those of dd_damage_at_probe_arrival_range, so the results are the same
// bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dd.h"
#include "dd_internal.h"
#include "dd_kernels.h"
#include "dd_runtime.h"

namespace dd {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

// Host code must not pass this name to a kernel: it is a host-side stand-in.
// Its device address (one per GPU) comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

dd_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DD_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorUnknown,
                                               "scratch symbol address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return DD_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace dd

using namespace dd;

dd_status dd_damage_at_probe_arrival_range_noalloc(dd_scan* s, int64_t j0, int64_t j1,
                                                   dd_precision p, double* out_dev,
                                                   void* hip_stream) {
  if (!s || (!out_dev && j1 > j0)) return fail(DD_EINVAL, "NULL argument");
  if (p != DD_FP64 && p != DD_MIXED) return fail(DD_EINVAL, "unknown precision %d", (int)p);
  if (j0 < 0 || j1 < j0 || j1 > s->V)
    return fail(DD_EINVAL, "visit range [%lld, %lld) outside [0, %lld]", (long long)j0,
                (long long)j1, (long long)s->V);
  if (j1 == j0) return DD_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  // resident tables of this scan on this device, built by an earlier query
  if (s->dev != cur || s->n_rows != s->V + 1024 || !s->flag.p || !s->own)
    return fail(DD_EINVAL,
                "the scan's device tables are not resident on device %d: run a query of this "
                "scan (e.g. dd_damage_at_probe_arrival_range) on it first",
                cur);
  const bool mixed = p == DD_MIXED;
  static thread_local RangePlan rp;  // host vectors reused between calls
  plan_range(s, mixed, j0, j1, false, rp);
  const size_t bi = sizeof(ArrItem) * rp.items.size();
  const size_t bt = sizeof(int32_t) * rp.tile_slots.size();
  const size_t bp = sizeof(double) * (size_t)rp.P.S * (size_t)rp.pstride;
  const size_t off_t = align256(bi), off_p = off_t + align256(bt), need = off_p + bp;
  if (need > kScratchBytes)
    return fail(DD_EINVAL,
                "the range needs %zu bytes of scratch, above the %zu bytes of the "
                "no-allocation query; use dd_damage_at_probe_arrival_range",
                need, kScratchBytes);
  void* base = nullptr;
  dd_status rc = scratch_on(cur, &base);
  if (rc != DD_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  OutFlag fl;
  rc = begin_call(s, st, fl);  // the scan is resident: nothing is allocated
  if (rc != DD_OK) return rc;
  char* b = (char*)base;
  // The plan goes up from pageable host memory.  HIP performs such a copy
  // synchronously: in stream order (after the kernels of the previous call
  // on this stream have read the scratch) and complete when it returns, so
  // the next call may rewrite the host vectors.
  if (bi) {
    e = hipMemcpyAsync(b, rp.items.data(), bi, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "host-to-device copy");
  }
  if (bt) {
    e = hipMemcpyAsync(b + off_t, rp.tile_slots.data(), bt, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "host-to-device copy");
  }
  rc = launch_range(s, mixed, rp, j0, j1, (const ArrItem*)b, (const int32_t*)(b + off_t),
                    (double*)(b + off_p), out_dev, fl, st, false);
  if (rc != DD_OK) return rc;
  return s->record_last(st);
}
