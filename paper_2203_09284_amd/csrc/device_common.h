// Device helpers shared by the sweep, batched and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fpr {
namespace dev {

// ------------------------------------------------------- cross-lane moves --
//
// DPP moves (a VALU operand modifier, no LDS round trip, unlike __shfl_*,
// which becomes ds_bpermute).  Lanes without a source, and rows outside the
// row mask, read 0.  Controls: row_shr:n shifts within rows of 16 lanes,
// row_bcast:15 / :31 broadcast lane 15 of each row (lane 31) to the next rows,
// wave_shr:1 shifts the whole wavefront by one lane.
enum : int {
  kDppRowShr1 = 0x111,
  kDppRowShr2 = 0x112,
  kDppRowShr4 = 0x114,
  kDppRowShr8 = 0x118,
  kDppWaveShr1 = 0x138,
  kDppRowBcast15 = 0x142,
  kDppRowBcast31 = 0x143
};

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, true);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(v)));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL, ROW_MASK>((int)b);
  const int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive prefix sum of an int over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp_i<kDppRowShr1>(x);
  x += dpp_i<kDppRowShr2>(x);
  x += dpp_i<kDppRowShr4>(x);
  x += dpp_i<kDppRowShr8>(x);
  x += dpp_i<kDppRowBcast15, 0xa>(x);
  x += dpp_i<kDppRowBcast31, 0xc>(x);
  return x;
}

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
  template <int CTRL, int ROW_MASK = 0xf>
  __device__ __forceinline__ LaneSum dpp() const {
    LaneSum r;
    r.s = dpp_d<CTRL, ROW_MASK>(s);
    return r;
  }
  // sum over the lpr-lane group (lpr a power of two, uniform in the
  // wavefront): the whole wavefront by a DPP scan read at lane 63, smaller
  // groups by a butterfly
  __device__ __forceinline__ void group_reduce(int lpr) {
    if (lpr == 64) {
      s += dpp_d<kDppRowShr1>(s);
      s += dpp_d<kDppRowShr2>(s);
      s += dpp_d<kDppRowShr4>(s);
      s += dpp_d<kDppRowShr8>(s);
      s += dpp_d<kDppRowBcast15, 0xa>(s);
      s += dpp_d<kDppRowBcast31, 0xc>(s);
      s = readlane_d(s, 63);
      return;
    }
    for (int off = lpr >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  }
};

// FPR_NAIVE_SUM=1 builds a variant of the library whose FP32 sums are plain
// (no compensation term): a test compares its error against the compensated
// build's on a graph where a lane adds many terms far below its running sum.
#ifndef FPR_NAIVE_SUM
#define FPR_NAIVE_SUM 0
#endif

template <>
struct LaneSum<float> {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float v) {
#pragma clang fp contract(off)
    if constexpr (FPR_NAIVE_SUM) {
      s = s + v;
      return;
    }
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
    if constexpr (FPR_NAIVE_SUM) {
      s = s + s2;
      return;
    }
    float t = s + s2;
    float bp = t - s;
    float err = (s - (t - bp)) + (s2 - bp);
    c = c + c2 + err;
    s = t;
  }
  template <int CTRL, int ROW_MASK = 0xf>
  __device__ __forceinline__ LaneSum dpp() const {
    LaneSum r;
    r.s = dpp_f<CTRL, ROW_MASK>(s);
    r.c = dpp_f<CTRL, ROW_MASK>(c);
    return r;
  }
  template <int CTRL, int ROW_MASK = 0xf>
  __device__ __forceinline__ void scan_step() {
    LaneSum e = dpp<CTRL, ROW_MASK>();
    e.combine(s, c);
    *this = e;
  }
  __device__ __forceinline__ void group_reduce(int lpr) {
    if (lpr == 64) {
      scan_step<kDppRowShr1>();
      scan_step<kDppRowShr2>();
      scan_step<kDppRowShr4>();
      scan_step<kDppRowShr8>();
      scan_step<kDppRowBcast15, 0xa>();
      scan_step<kDppRowBcast31, 0xc>();
      s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s), 63));
      c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c), 63));
      return;
    }
    for (int off = lpr >> 1; off > 0; off >>= 1) {
      float s2 = __shfl_xor(s, off, 64);
      float c2 = __shfl_xor(c, off, 64);
      combine(s2, c2);
    }
  }
};

// Segmented inclusive scan over the 64 lanes: lane l ends with the sum of
// lanes k..l, k the last lane <= l whose flag is set (lane 0 if none).
template <typename T, int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_scan_step(LaneSum<T> &v, int &f) {
  LaneSum<T> p = v.template dpp<CTRL, ROW_MASK>();
  const int pf = dpp_i<CTRL, ROW_MASK>(f);
  p.combine_with(v);
  if (!f) v = p;
  f |= pf;
}
template <typename T>
__device__ __forceinline__ void seg_scan(LaneSum<T> &v, bool flag) {
  int f = flag ? 1 : 0;
  seg_scan_step<T, kDppRowShr1, 0xf>(v, f);
  seg_scan_step<T, kDppRowShr2, 0xf>(v, f);
  seg_scan_step<T, kDppRowShr4, 0xf>(v, f);
  seg_scan_step<T, kDppRowShr8, 0xf>(v, f);
  seg_scan_step<T, kDppRowBcast15, 0xa>(v, f);
  seg_scan_step<T, kDppRowBcast31, 0xc>(v, f);
}

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
