// Device helpers shared by the sweep, batched and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fpr {
namespace dev {

// ------------------------------------------------------------ arithmetic --

// Per-lane sum: plain FP64, or FP32 with Neumaier compensation.
template <typename T>
struct LaneSum;

template <>
struct LaneSum<double> {
  double s = 0.0;
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ double value() const { return s; }
  __device__ __forceinline__ LaneSum shfl_up(int off) const {
    LaneSum r;
    r.s = __shfl_up(s, off, 64);
    return r;
  }
  // this = earlier + this
  __device__ __forceinline__ void add_before(const LaneSum &earlier) { s = earlier.s + s; }
  // this = this + later
  __device__ __forceinline__ void combine_with(const LaneSum &later) { s = s + later.s; }
  // butterfly over the lpr-lane group (lpr a power of two, uniform in the wavefront)
  __device__ __forceinline__ void group_reduce(int lpr) {
    for (int off = lpr >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  }
};

template <>
struct LaneSum<float> {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float v) {
#pragma clang fp contract(off)
    float t = s + v;
    if (fabsf(s) >= fabsf(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s + (double)c; }
  __device__ __forceinline__ LaneSum shfl_up(int off) const {
    LaneSum r;
    r.s = __shfl_up(s, off, 64);
    r.c = __shfl_up(c, off, 64);
    return r;
  }
  __device__ __forceinline__ void add_before(const LaneSum &earlier) {
    LaneSum e = earlier;
    e.combine(s, c);
    *this = e;
  }
  __device__ __forceinline__ void combine_with(const LaneSum &later) { combine(later.s, later.c); }
  // TwoSum of the leading parts, compensations added
  __device__ __forceinline__ void combine(float s2, float c2) {
#pragma clang fp contract(off)
    float t = s + s2;
    float bp = t - s;
    float err = (s - (t - bp)) + (s2 - bp);
    c = c + c2 + err;
    s = t;
  }
  __device__ __forceinline__ void group_reduce(int lpr) {
    for (int off = lpr >> 1; off > 0; off >>= 1) {
      float s2 = __shfl_xor(s, off, 64);
      float c2 = __shfl_xor(c, off, 64);
      combine(s2, c2);
    }
  }
};

// Reductions carried per thread through a work item.
struct Red {
  double chg = 0.0;   // sum (or max) of |x' - x|
  double dang = 0.0;  // new dangling mass
  double tot = 0.0;   // new total mass
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace dev
}  // namespace fpr
