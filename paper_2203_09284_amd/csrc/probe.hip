// Gather-rate probe: the time of the sweep's memory gathers with nothing else
// around them.
//
// The sweep of Eq. 1 reads, for every in-edge, the contribution of its source
// at the source's gather slot.  On a graph without id locality those reads
// land on random cache lines, and their rate on this device, not HBM's
// streaming rate, is what bounds the sweep.  This kernel performs exactly
// those reads (the plan's in-edge slots in its bin order, skipping the
// slots the sweep serves from its LDS copy) and sums them, on the sweep's
// grid, eight loads in flight per lane: no rank update, no list bounds, no
// writes but one value per thread.  Mode 1 draws as many slots uniformly
// from [0, n) instead (a counter-based SplitMix64 mix of the edge index,
// Steele, Lea and Flood 2014), the device's rate for random lines that no
// cache holds.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

using namespace fpr;

namespace {

constexpr int kProbeBlock = 512;
constexpr int kProbeLoads = 8;

__device__ __forceinline__ uint32_t mix_slot(uint64_t e, uint32_t n) {
  uint64_t z = e + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (uint32_t)(((z >> 32) * (uint64_t)n) >> 32);  // in [0, n)
}

template <typename T>
__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const T *a, const int32_t *idx, int64_t m, int hot,
                                                              int uniform, uint32_t n, double *out) {
  const int64_t step = (int64_t)gridDim.x * kProbeBlock * kProbeLoads;
  double acc = 0.0;
  for (int64_t e0 = (int64_t)blockIdx.x * kProbeBlock * kProbeLoads + threadIdx.x; e0 < m; e0 += step) {
    int32_t s[kProbeLoads];
#pragma unroll
    for (int k = 0; k < kProbeLoads; ++k) {
      const int64_t e = e0 + (int64_t)k * kProbeBlock;
      s[k] = e >= m ? -1 : uniform ? (int32_t)mix_slot((uint64_t)e, n) : idx[e];
    }
    T v[kProbeLoads];
#pragma unroll
    for (int k = 0; k < kProbeLoads; ++k) v[k] = s[k] >= hot ? a[s[k]] : (T)0;
#pragma unroll
    for (int k = 0; k < kProbeLoads; ++k) acc += (double)v[k];
  }
  out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = acc;
}

template <typename T>
int probe_impl(pr_graph *g, int uniform, int reps, double *best_us, double *mean_us) {
  const DevPlan &P = g->fwd;
  const int64_t limit = kHotBytes / (int64_t)sizeof(T);
  const int64_t hot64 = uniform ? 0 : g->popts.hot_slots < 0 ? limit : std::min<int64_t>(g->popts.hot_slots, limit);
  const int hot = (int)std::min<int64_t>(hot64, g->n);
  const int grid = std::max(1, g->grid);
  T *arr = nullptr;
  double *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = PR_OK;
  auto fail = [&](hipError_t e) { rc = pr_fail(PR_EDEVICE, "pr_probe_gathers: %s", hipGetErrorString(e)); };
  hipError_t e;
  if (hipMalloc((void **)&arr, sizeof(T) * (size_t)g->n) != hipSuccess ||
      hipMalloc((void **)&out, sizeof(double) * (size_t)grid * kProbeBlock) != hipSuccess) {
    (void)hipGetLastError();
    rc = pr_fail(PR_ENOMEM, "pr_probe_gathers: no device memory for %lld values", (long long)g->n);
  } else if ((e = hipMemsetAsync(arr, 0, sizeof(T) * (size_t)g->n, g->work)) != hipSuccess ||
             (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    fail(e);
  } else {
    double best = 1e300, sum = 0.0;
    // one untimed launch, then `reps` timed ones
    for (int r = 0; r <= reps && rc == PR_OK; ++r) {
      (void)hipEventRecord(e0, g->work);
      k_probe_gather<T><<<grid, kProbeBlock, 0, g->work>>>(arr, P.idx, P.m, hot, uniform, (uint32_t)g->n, out);
      (void)hipEventRecord(e1, g->work);
      if ((e = hipGetLastError()) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
        fail(e);
        break;
      }
      float ms = 0.0f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        fail(e);
        break;
      }
      if (r > 0) {
        best = std::min(best, 1e3 * (double)ms);
        sum += 1e3 * (double)ms;
      }
    }
    if (rc == PR_OK) {
      *best_us = best;
      if (mean_us) *mean_us = sum / reps;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(g->work);
  if (arr) (void)hipFree(arr);
  if (out) (void)hipFree(out);
  return rc;
}

}  // namespace

extern "C" int pr_probe_gathers(pr_graph *g, int precision, int mode, int reps, double *best_us, double *mean_us,
                                void *stream) {
  pr_clear_error();
  if (!g) return pr_fail(PR_EINVAL, "graph is NULL");
  if (precision != PR_FP64 && precision != PR_FP32) return pr_fail(PR_EINVAL, "bad precision %d", precision);
  if (mode != 0 && mode != 1) return pr_fail(PR_EINVAL, "pr_probe_gathers: mode %d is not 0 or 1", mode);
  if (reps < 1 || reps > 1000) return pr_fail(PR_EINVAL, "pr_probe_gathers: reps=%d outside [1, 1000]", reps);
  if (!best_us) return pr_fail(PR_EINVAL, "pr_probe_gathers: best_us is NULL");
  if (g->n > (int64_t)INT32_MAX) return pr_fail(PR_EINVAL, "pr_probe_gathers: n exceeds the 32-bit slot range");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  // the caller's stream is joined to the work stream around the probe
  hipStream_t user = (hipStream_t)stream;
  (void)hipEventRecord(g->ev_in, user);
  (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  const int rc = precision == PR_FP32 ? probe_impl<float>(g, mode, reps, best_us, mean_us)
                                      : probe_impl<double>(g, mode, reps, best_us, mean_us);
  (void)hipEventRecord(g->ev_out, g->work);
  (void)hipStreamWaitEvent(user, g->ev_out, 0);
  return rc;
}
