// Batched personalized PageRank: k teleport vectors, one-hot on seeds[j],
//     X[:, j] = (1-d) e_{seed_j} + d (P X[:, j] + D_j / n)   (Eq. 1 with a personalised teleport),
// solved as one multi-column Jacobi pull per sweep.
//
// Layout.  A launch advances T columns (T a multiple of 4, at most 64: the
// tile width).  Ranks and contributions are vertex-major: the T values of a
// vertex are one row of 4T bytes (256 bytes at T = 64), so an in-edge costs
// one row read, made by the 16 lanes of a lane group with 16-byte loads.  A
// wavefront is four such groups; lane j of a group holds columns 4j..4j+3
// (lanes with 4j >= T stay idle).
//
// Work (the plan's batched list).  Short and empty rows come in runs; each
// run is walked by one lane group, row by row: a group loads 16 gather slots
// at once (a lane each) and broadcasts them across its 16 lanes by DPP, with
// 8 row reads in flight per lane.  A long row is one item: the four groups sum one quarter of its list
// each.  A hub is split into `chunk`-edge items of the same kind, whose sums
// the finalize kernel adds in chunk order.  None of this depends on T, and
// every column is summed in the same order whatever the tile width, so the
// results do not depend on it.
//
// Arithmetic.  Ranks and contributions are FP32; sums use Kahan
// compensation per lane and TwoSum when quarters combine (in quarter order).
// Per-column residuals and dangling mass are summed in 64-bit fixed point
// (2^-60 units), exact and order-free, then read as FP64.
// A column whose L1 residual drops below tol is frozen: its values stop
// changing and its sweep count is recorded.  A launch's sweeps stop once all
// its columns are frozen.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "internal.h"

using namespace fpr;
using namespace fpr::dev;

namespace {

// Rows streamed once per sweep (the ranks, read and written; the new
// contribution rows, written) go through non-temporal loads and stores, so
// they do not push the gathered contribution rows of popular sources out of
// L2.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load(const float4 *p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store(float4 *p, const float4 &v) {
  const nt_f4 t = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(t, reinterpret_cast<nt_f4 *>(p));
}


constexpr int kVBlock = 512;          // threads per workgroup of the sweep
constexpr int kVWaves = kVBlock / 64;
constexpr int kVMaxT = 64;            // columns per launch at most
constexpr int kVFin = 256;            // threads per workgroup of the finalize kernel (one per column)

struct VState {
  double D[kVMaxT];      // dangling mass per column of the current iterate
  double resid[kVMaxT];  // last L1 change per column
  int done[kVMaxT];      // column frozen
  int iters[kVMaxT];     // sweeps until the column froze (or so far)
  double tol;
  int max_iter;
  int pad;
};

struct VArgs {
  const uint32_t *rows;
  const uint32_t *rowpos;
  const uint32_t *rptr;
  const int32_t *idx;
  const int4 *items;
  const int2 *vrun;
  const int4 *hsplit;
  const uint32_t *gpos;
  const double *inv_w;
  const int32_t *seeds;  // [T], -1 for padding columns
  float4 *x;             // [n][Q] vertex order (the kernels take it from io)
  const IoPtrs *io;      // io->x: where x lives (the caller's X when one launch holds all k columns)
  float4 *c0;            // [n][Q] gather-layout order
  float4 *c1;
  double *hpart;         // [n_chunks][T]
  unsigned long long *wg_part;  // [2][T][n_wg]: change and dangling mass per column and workgroup
                                // (fixed point, kFix units)
  VState *st;
  double d;
  double inv_n;
  int64_t n;
  int n_items;
  int n_split;
  int n_wg;    // workgroups of the sweep launch
  int ipg;     // consecutive items a wavefront takes at a time
  int chunk;
  int T;    // columns of this launch
  int Q;    // T / 4: float4 per row
  int par;  // sweep parity: 0 reads c0 and writes c1
};

// Compensated FP32 sum of one column: Kahan's update (the running low part c
// joins each term before the term joins s; the sum is s + c).  The terms of a
// PageRank sum all have one sign, where Kahan's error bound holds in any
// order; the update takes four operations per term against eight for the
// magnitude-tested form of LaneSum, which counts here: 64 columns per in-edge.
// Partial sums combine by TwoSum of their leading parts, compensations added.
struct KSum {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float v) {
#pragma clang fp contract(off)
    if constexpr (FPR_NAIVE_SUM) {
      s = s + v;
      return;
    }
    const float y = v + c;
    const float t = s + y;
    c = y - (t - s);
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s + (double)c; }
  __device__ __forceinline__ void combine_with(const KSum &l) {
#pragma clang fp contract(off)
    if constexpr (FPR_NAIVE_SUM) {
      s = s + l.s;
      return;
    }
    const float t = s + l.s;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (l.s - bp);
    c = c + l.c + err;
    s = t;
  }
};

struct Sum4 {
  KSum v[4];
  __device__ __forceinline__ void add(const float4 &a) {
    v[0].add(a.x);
    v[1].add(a.y);
    v[2].add(a.z);
    v[3].add(a.w);
  }
  __device__ __forceinline__ void combine_with(const Sum4 &l) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q].combine_with(l.v[q]);
  }
  // the sums held by lane `src` (every lane of the wavefront takes part)
  __device__ __forceinline__ Sum4 from_lane(int src) const {
    Sum4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r.v[q].s = __shfl(v[q].s, src, 64);
      r.v[q].c = __shfl(v[q].c, src, 64);
    }
    return r;
  }
};

// Per-column change and dangling mass.  Within a work item they are summed
// in FP64 in a fixed order (each group over its rows, then the four groups in
// order), so an item's sums do not depend on which wavefront ran it; each
// item's sum is then rounded once to 64-bit fixed point (kFix = 2^60 units per
// 1.0) and the items are added as integers, whose sums do not depend on their
// order.  So the totals, and the dangling mass every column's next sweep adds,
// are the same bits whatever the launch shape.  Both totals stay below 4
// (sums of |x' - x| and of x over a column whose values sum to 1), far inside
// the 64-bit range.
constexpr double kFix = 1152921504606846976.0;  // 2^60
__device__ __forceinline__ unsigned long long to_fix(double v) {
  return (unsigned long long)__double2ll_rn(v * kFix);
}

struct VRed {
  double chg[4] = {0.0, 0.0, 0.0, 0.0};
  double dang[4] = {0.0, 0.0, 0.0, 0.0};
};


// Lane view of a launch.  A row of Q float4 (T = 4Q columns) is read by a
// group of LPR >= Q lanes (lane j holds columns 4j..4j+3); four groups form a
// quad-slot, which runs one work item at a time (its four runs, or the four
// quarters of a long row); a wavefront holds 16 / LPR quad-slots.
struct VCtx {
  const float4 *cin;
  float4 *cout;
  int g, j;   // group within the quad-slot, lane within the group
  int base;   // first lane of the quad-slot
  int qs;     // quad-slot within the wavefront
  bool act;
  bool frozen[4];
  int seed[4];
  double dterm[4];
};

template <int LPR>
__device__ __forceinline__ VCtx make_vctx(const VArgs &a) {
  VCtx C;
  const int lane = threadIdx.x & 63;
  C.j = lane % LPR;
  C.g = (lane / LPR) & 3;
  C.qs = lane / (4 * LPR);
  C.base = C.qs * 4 * LPR;
  C.act = C.j < a.Q;
  C.cin = a.par ? a.c1 : a.c0;
  C.cout = a.par ? a.c0 : a.c1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = 4 * C.j + q;
    C.seed[q] = C.act ? a.seeds[col] : -1;
    C.frozen[q] = !C.act || C.seed[q] < 0 || a.st->done[col] != 0;
    C.dterm[q] = C.act ? a.st->D[col] * a.inv_n : 0.0;
  }
  return C;
}

// Lane `src` of the caller's group of LPR lanes (DPP: row broadcasts for
// groups of 16 and 8 lanes, quad permutes for 4 and 2; a group of one lane is
// the lane itself).
template <int LPR, int SRC>
__device__ __forceinline__ int group_bcast(int v) {
  if constexpr (LPR == 16) {
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + SRC, 0xf, 0xf, true);
  } else if constexpr (LPR == 8) {
    const int lo = __builtin_amdgcn_update_dpp(0, v, 0x150 + SRC, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, v, 0x150 + 8 + SRC, 0xf, 0xf, true);
    return (threadIdx.x & 8) ? hi : lo;
  } else if constexpr (LPR == 4) {
    return __builtin_amdgcn_update_dpp(0, v, SRC | (SRC << 2) | (SRC << 4) | (SRC << 6), 0xf, 0xf, true);
  } else if constexpr (LPR == 2) {
    return __builtin_amdgcn_update_dpp(0, v, SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6), 0xf, 0xf,
                                       true);
  } else {
    return v;
  }
}

// A group's 16 gather slots: lane j holds slots j, j + LPR, ... (16 / LPR of
// them); slot b is at lane b % LPR, register b / LPR.
template <int LPR>
struct Slots16 {
  int v[16 / LPR];
  template <int B>
  __device__ __forceinline__ int get() const {
    return group_bcast<LPR, B % LPR>(v[B / LPR]);
  }
};

template <int LPR>
__device__ __forceinline__ void load_slots(const VArgs &a, const VCtx &C, uint32_t e, uint32_t e1, Slots16<LPR> &sl) {
#pragma unroll
  for (int r = 0; r < 16 / LPR; ++r) {
    const uint32_t at = e + C.j + r * LPR;
    sl.v[r] = at < e1 ? a.idx[at] : 0;
  }
}

template <int LPR, int B0>
__device__ __forceinline__ void read8(const VArgs &a, const VCtx &C, const Slots16<LPR> &sl, int cnt, float4 *v) {
  int s[kBatch];
  s[0] = sl.template get<B0 + 0>();
  s[1] = sl.template get<B0 + 1>();
  s[2] = sl.template get<B0 + 2>();
  s[3] = sl.template get<B0 + 3>();
  s[4] = sl.template get<B0 + 4>();
  s[5] = sl.template get<B0 + 5>();
  s[6] = sl.template get<B0 + 6>();
  s[7] = sl.template get<B0 + 7>();
#pragma unroll
  for (int b = 0; b < kBatch; ++b)
    v[b] = (B0 + b < cnt && C.act) ? C.cin[(size_t)s[b] * a.Q + C.j] : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Adds the rows of cnt <= 16 in-edges, in list order, whose gather slots the
// group holds in `sl`; 8 row reads in flight per lane.
template <int LPR>
__device__ __forceinline__ void chunk16(const VArgs &a, const VCtx &C, const Slots16<LPR> &sl, int cnt, Sum4 &acc) {
  float4 v[kBatch];
  read8<LPR, 0>(a, C, sl, cnt, v);
#pragma unroll
  for (int b = 0; b < kBatch; ++b)
    if (b < cnt) acc.add(v[b]);
  if (cnt > kBatch) {
    read8<LPR, kBatch>(a, C, sl, cnt, v);
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
      if (kBatch + b < cnt) acc.add(v[b]);
  }
}

// Sum over the in-edges [e0, e1) in list order.
template <int LPR>
__device__ __forceinline__ void range_sum(const VArgs &a, const VCtx &C, uint32_t e0, uint32_t e1, Sum4 &acc) {
  for (uint32_t e = e0; e < e1; e += 16) {
    Slots16<LPR> sl;
    load_slots<LPR>(a, C, e, e1, sl);
    chunk16<LPR>(a, C, sl, (int)min(16u, e1 - e), acc);
  }
}

__device__ __forceinline__ float comp(const float4 &v, int q) {
  return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}

// Update of vertex u (gather slot `slot`, 1/W_u = iw, old row xo) from its
// column sums s[4]; frozen columns keep their values.
__device__ __forceinline__ void vupdate(const VArgs &a, const VCtx &C, uint32_t u, uint32_t slot, double iw,
                                        const float4 &xo, const double *s, VRed &red) {
  float xn[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float old = comp(xo, q);
    if (C.frozen[q]) {
      xn[q] = old;
    } else {
      const double tele = ((int)u == C.seed[q]) ? (1.0 - a.d) : 0.0;
      xn[q] = (float)(tele + a.d * (s[q] + C.dterm[q]));
      red.chg[q] += fabs((double)xn[q] - (double)old);
    }
  }
  nt_store(&a.x[(size_t)u * a.Q + C.j], make_float4(xn[0], xn[1], xn[2], xn[3]));
  if (iw != 0.0) {
    nt_store(&C.cout[(size_t)slot * a.Q + C.j],
             make_float4((float)((double)xn[0] * iw), (float)((double)xn[1] * iw),
                         (float)((double)xn[2] * iw), (float)((double)xn[3] * iw)));
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) red.dang[q] += (double)xn[q];
  }
}

// A run of rows [r0, r1), walked by one lane group.  The next row's bounds,
// vertex and slot, and the current row's update operands, load while the
// current row's rows are read; the next row's first 16 gather slots load
// while the current row is updated.
template <int LPR>
__device__ __forceinline__ void run_rows(const VArgs &a, const VCtx &C, int r0, int r1, VRed &red) {
  uint32_t e0 = a.rptr[r0], e1 = a.rptr[r0 + 1];
  uint32_t u = a.rows[r0], slot = a.rowpos[r0];
  Slots16<LPR> sl;
  load_slots<LPR>(a, C, e0, e1, sl);
  for (int r = r0; r < r1; ++r) {
    const bool more = r + 1 < r1;
    const uint32_t ne1 = more ? a.rptr[r + 2] : e1;
    const uint32_t nu = more ? a.rows[r + 1] : 0u;
    const uint32_t nslot = more ? a.rowpos[r + 1] : 0u;
    const double iw = a.inv_w[u];
    const float4 xo = C.act ? nt_load(&a.x[(size_t)u * a.Q + C.j]) : make_float4(0.f, 0.f, 0.f, 0.f);
    Sum4 acc;
    for (uint32_t e = e0; e < e1; e += 16) {
      if (e != e0) load_slots<LPR>(a, C, e, e1, sl);
      chunk16<LPR>(a, C, sl, (int)min(16u, e1 - e), acc);
    }
    load_slots<LPR>(a, C, e1, more ? ne1 : e1, sl);
    double s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = acc.v[q].value();
    if (C.act) vupdate(a, C, u, slot, iw, xo, s, red);
    e0 = e1;
    e1 = ne1;
    u = nu;
    slot = nslot;
  }
}

// The four groups of a quad-slot sum one quarter each of [e0, e1); group 0
// ends with the whole sum (quarters combined in order).
template <int LPR>
__device__ __forceinline__ Sum4 quarter_sum(const VArgs &a, const VCtx &C, uint32_t e0, uint32_t e1) {
  const uint32_t L = e1 - e0;
  const uint32_t q0 = e0 + (uint32_t)(((uint64_t)L * C.g) / 4);
  const uint32_t q1 = e0 + (uint32_t)(((uint64_t)L * (C.g + 1)) / 4);
  Sum4 acc;
  range_sum<LPR>(a, C, q0, q1, acc);
  Sum4 tot = acc;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const Sum4 o = acc.from_lane(C.base + C.j + LPR * k);
    tot.combine_with(o);
  }
  return tot;
}

// Ends a work item: its per-column sums (the quad-slot's four groups in
// order), rounded to fixed point, into the workgroup's totals in LDS
// (integer atomics: the order of the adds does not matter).
template <int LPR>
__device__ __forceinline__ void fold_item(const VCtx &C, VRed &red, unsigned long long (*tot)[kVMaxT]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double ch = red.chg[q], dg = red.dang[q];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      ch += __shfl(red.chg[q], C.base + C.j + LPR * k, 64);
      dg += __shfl(red.dang[q], C.base + C.j + LPR * k, 64);
    }
    if (C.g == 0 && C.act) {
      atomicAdd(&tot[0][4 * C.j + q], to_fix(ch));
      atomicAdd(&tot[1][4 * C.j + q], to_fix(dg));
    }
    red.chg[q] = 0.0;
    red.dang[q] = 0.0;
  }
}

template <int LPR>
__global__ __launch_bounds__(kVBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_vsweep(VArgs a0) {
  constexpr int NQS = 16 / LPR;  // quad-slots per wavefront
  __shared__ unsigned long long s_tot[2][kVMaxT];
  VArgs a = a0;
  a.x = static_cast<float4 *>(a0.io->x);
  const VCtx C = make_vctx<LPR>(a);
  // every group holds the same columns: the vote is uniform over the workgroup
  const bool all_frozen = C.frozen[0] && C.frozen[1] && C.frozen[2] && C.frozen[3];
  if (__ballot(!all_frozen) == 0ull) return;
  if (threadIdx.x < 2 * kVMaxT) s_tot[threadIdx.x / kVMaxT][threadIdx.x % kVMaxT] = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  // each quad-slot takes items as a wavefront of its own would
  const int vw = (int)(blockIdx.x * kVWaves + wave) * NQS + C.qs;
  const int nvw = a.n_wg * kVWaves * NQS;
  VRed red;
  for (int first = vw * a.ipg; first < a.n_items; first += nvw * a.ipg) {
    const int last = min(first + a.ipg, a.n_items);
    for (int item = first; item < last; ++item) {
      const int4 wi = a.items[item];
      if (wi.x == kVQuad) {
        if (C.g < wi.z) {
          const int2 rr = a.vrun[wi.y + C.g];
          run_rows<LPR>(a, C, rr.x, rr.y, red);
        }
      } else if (wi.x == kVLong) {
        const int r = wi.y;
        const uint32_t u = a.rows[r];
        const uint32_t slot = a.rowpos[r];
        const double iw = a.inv_w[u];
        const float4 xo = (C.g == 0 && C.act) ? nt_load(&a.x[(size_t)u * a.Q + C.j]) : make_float4(0.f, 0.f, 0.f, 0.f);
        const Sum4 tot = quarter_sum<LPR>(a, C, a.rptr[r], a.rptr[r + 1]);
        if (C.g == 0 && C.act) {
          double s[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) s[q] = tot.v[q].value();
          vupdate(a, C, u, slot, iw, xo, s, red);
        }
      } else {  // kHeavy: chunk wi.z of hub row wi.y, partial sums to hpart[wi.w + wi.z]
        const uint32_t rb = a.rptr[wi.y], re = a.rptr[wi.y + 1];
        const uint32_t c0 = rb + (uint32_t)wi.z * (uint32_t)a.chunk;
        const uint32_t c1 = min(re, c0 + (uint32_t)a.chunk);
        const Sum4 tot = quarter_sum<LPR>(a, C, c0, c1);
        if (C.g == 0 && C.act) {
          double *hp = a.hpart + (size_t)(wi.w + wi.z) * a.T + 4 * C.j;
#pragma unroll
          for (int q = 0; q < 4; ++q) hp[q] = tot.v[q].value();
        }
      }
      fold_item<LPR>(C, red, s_tot);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * a.T) {
    const int kind = threadIdx.x / a.T, col = threadIdx.x % a.T;
    a.wg_part[((size_t)kind * a.T + col) * a.n_wg + blockIdx.x] = s_tot[kind][col];
  }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kVFin) void k_vfinal(VArgs a0) {
  __shared__ unsigned long long s_red[2][kVFin / 64];
  VArgs a = a0;
  a.x = static_cast<float4 *>(a0.io->x);
  const int col = blockIdx.x;
  VState *st = a.st;
  if (st->done[col]) return;
  const int seed = a.seeds[col];
  const double dterm = st->D[col] * a.inv_n;
  float *xf = reinterpret_cast<float *>(a.x);
  float *cf = reinterpret_cast<float *>(a.par ? a.c0 : a.c1);
  unsigned long long chg = 0, dang = 0;
  for (int i = threadIdx.x; i < a.n_wg; i += kVFin) {
    chg += a.wg_part[(size_t)col * a.n_wg + i];
    dang += a.wg_part[((size_t)a.T + col) * a.n_wg + i];
  }
  for (int h = threadIdx.x; h < a.n_split; h += kVFin) {
    const int4 hs = a.hsplit[h];
    const uint32_t u = a.rows[hs.x];
    const uint32_t slot = a.rowpos[hs.x];
    // chunk sums in chunk order, eight loads in flight (a zero past the end
    // leaves the sum unchanged)
    double s = 0.0;
    for (int k0 = 0; k0 < hs.z; k0 += 8) {
      double pt[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) pt[k] = k0 + k < hs.z ? a.hpart[(size_t)(hs.y + k0 + k) * a.T + col] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) s += pt[k];
    }
    const float old = xf[(size_t)u * a.T + col];
    const double tele = ((int)u == seed) ? (1.0 - a.d) : 0.0;
    const float xn = (float)(tele + a.d * (s + dterm));
    chg += to_fix(fabs((double)xn - (double)old));
    xf[(size_t)u * a.T + col] = xn;
    const double iw = a.inv_w[u];
    if (iw != 0.0) cf[(size_t)slot * a.T + col] = (float)((double)xn * iw);
    else dang += to_fix((double)xn);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  chg = wave_sum_u64(chg);
  dang = wave_sum_u64(dang);
  if (lane == 0) {
    s_red[0][wave] = chg;
    s_red[1][wave] = dang;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long chs = s_red[0][0], dgs = s_red[1][0];
    for (int w = 1; w < kVFin / 64; ++w) {
      chs += s_red[0][w];
      dgs += s_red[1][w];
    }
    const double ch = (double)chs / kFix, dg = (double)dgs / kFix;
    const int it = st->iters[col] + 1;
    st->iters[col] = it;
    st->resid[col] = ch;
    st->D[col] = dg;
    if (!(ch >= st->tol) || it >= st->max_iter) st->done[col] = 1;
  }
}

// x = 0 and c (the first sweep's input) = 0, as float4 rows.
__global__ __launch_bounds__(kBlock) void k_vzero(float4 *x, float4 *c, int64_t count) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) {
    x[i] = z;
    c[i] = z;
  }
}

// One thread per column: the one-hot start x = e_seed, its contribution, and
// the column's state.
__global__ void k_vseed(VArgs a, double tol, int max_iter) {
  const int col = threadIdx.x;
  VState *st = a.st;
  if (col == 0) {
    st->tol = tol;
    st->max_iter = max_iter;
  }
  if (col >= a.T) return;
  const int seed = a.seeds[col];
  double D = 0.0;
  if (seed >= 0) {
    reinterpret_cast<float *>(a.x)[(size_t)seed * a.T + col] = 1.0f;
    const double iw = a.inv_w[seed];
    if (iw != 0.0) reinterpret_cast<float *>(a.c0)[(size_t)a.gpos[seed] * a.T + col] = (float)(1.0 * iw);
    else D = 1.0;
  }
  st->D[col] = D;
  st->resid[col] = INFINITY;
  st->done[col] = seed >= 0 ? 0 : 1;
  st->iters[col] = 0;
}

// The launch's columns into the caller's row-major X[n][k].
__global__ __launch_bounds__(kBlock) void k_vout(VArgs a, float *X, int k, int col0) {
  const float *xf = reinterpret_cast<const float *>(a.x);
  const int64_t count = a.n * a.T;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) {
    const int64_t u = i / a.T;
    const int c = (int)(i - u * a.T);
    if (col0 + c < k) X[u * k + col0 + c] = xf[i];
  }
}

__global__ void k_vseeds(const int32_t *seeds, int k, int32_t *out, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) out[i] = i < k ? seeds[i] : -1;
}

__global__ void k_vclear(int *flag) { *flag = 0; }

__global__ void k_vcheck(const int32_t *seeds, int k, int64_t n, int *bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k && (seeds[i] < 0 || seeds[i] >= n)) *bad = 1;
}

// ---------------------------------------------------------------- host --

struct VWork {
  int64_t cols_cap = 0;  // columns the row arrays hold
  float4 *x = nullptr, *c0 = nullptr, *c1 = nullptr;
  double *hpart = nullptr;
  unsigned long long *wg_part = nullptr;
  VState *st = nullptr;
  VState *host_st = nullptr;
  IoPtrs *io = nullptr;  // where the sweep kernels find x
  void *io_last = nullptr;
  int32_t *seeds = nullptr;
  int seeds_cap = 0;
  int *flag = nullptr;
};

// The batched workspace of a graph hangs off the graph (calls on one graph
// never overlap, so no lock is needed).
VWork *vwork_for(pr_graph *g) {
  if (!g->vwork) g->vwork = new VWork();
  return static_cast<VWork *>(g->vwork);
}

int ensure_vwork(pr_graph *g, VWork &w, int T) {
  int rc;
  if (w.cols_cap < T) {
    const size_t n = (size_t)g->n;
    const DevPlan &P = g->fwd;
    const size_t rows = n * (size_t)(T / 4);
    if ((rc = fpr_dev_alloc(g, (void **)&w.x, sizeof(float4) * rows))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.c0, sizeof(float4) * rows))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.c1, sizeof(float4) * rows))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.hpart, sizeof(double) * (size_t)T * (size_t)std::max(1, P.n_chunks))))
      return rc;
    // partials for the largest grid a shape can ask for (two workgroups per CU)
    if ((rc = fpr_dev_alloc(g, (void **)&w.wg_part,
                            sizeof(unsigned long long) * 2 * (size_t)T * (size_t)(2 * std::max(1, g->n_cu)))))
      return rc;
    w.cols_cap = T;
  }
  if (!w.st && (rc = fpr_dev_alloc(g, (void **)&w.st, sizeof(VState)))) return rc;
  if (!w.io && (rc = fpr_dev_alloc(g, (void **)&w.io, sizeof(IoPtrs)))) return rc;
  if (!w.host_st && hipHostMalloc((void **)&w.host_st, sizeof(VState)) != hipSuccess)
    return pr_fail(PR_ENOMEM, "pinned allocation failed");
  if (!w.flag && (rc = fpr_dev_alloc(g, (void **)&w.flag, sizeof(int)))) return rc;
  return PR_OK;
}

int ensure_seeds(pr_graph *g, VWork &w, int total) {
  if (w.seeds_cap >= total) return PR_OK;
  int rc = fpr_dev_alloc(g, (void **)&w.seeds, sizeof(int32_t) * total);
  if (rc) return rc;
  w.seeds_cap = total;
  return PR_OK;
}

__global__ void k_vset_io(IoPtrs *io, void *x) { io->x = x; }

// Points the sweep kernels at x (queued on the work stream); skipped when
// the block already holds it.
int set_vio(pr_graph *g, VWork &w, void *x) {
  if (w.io_last == x) return PR_OK;
  hipLaunchKernelGGL(k_vset_io, dim3(1), dim3(1), 0, g->work, w.io, x);
  PR_HIP(hipGetLastError());
  w.io_last = x;
  return PR_OK;
}

bool shape_ok(const pr_batch_shape &s) {
  return s.tile >= 4 && s.tile <= kVMaxT && s.tile % 4 == 0 && s.items_per_grab >= 1 && s.items_per_grab <= 16 &&
         s.wg_per_cu >= 1 && s.wg_per_cu <= 2;
}

// Launch arguments of T columns from col0; x goes through w.io (left null here).
VArgs make_vargs(pr_graph *g, VWork &w, double d, int T, int col0, const pr_batch_shape &sh) {
  const DevPlan &P = g->fwd;
  VArgs a;
  memset(&a, 0, sizeof(a));
  a.rows = P.rows;
  a.rowpos = P.rowpos;
  a.rptr = P.rptr;
  a.idx = P.idx;
  a.items = P.bitems;
  a.vrun = P.vrun;
  a.hsplit = P.hsplit;
  a.gpos = P.gpos;
  a.inv_w = g->inv_w;
  a.seeds = w.seeds + col0;
  a.x = nullptr;
  a.io = w.io;
  a.c0 = w.c0;
  a.c1 = w.c1;
  a.hpart = w.hpart;
  a.wg_part = w.wg_part;
  a.st = w.st;
  a.d = d;
  a.inv_n = 1.0 / (double)g->n;
  a.n = g->n;
  a.n_items = P.n_bitems;
  a.n_split = P.n_split;
  a.n_wg = std::max(1, g->n_cu) * sh.wg_per_cu;
  a.ipg = sh.items_per_grab;
  a.chunk = P.chunk;
  a.T = T;
  a.Q = T / 4;
  a.par = 0;
  return a;
}

// The sweep kernel for a launch's row width: lanes per row = Q rounded up to
// a power of two, so a row of T columns is read by T / 4 lanes.
void launch_vsweep(const VArgs &a, hipStream_t s) {
  const dim3 grid(a.n_wg), block(kVBlock);
  if (a.Q <= 1) hipLaunchKernelGGL(k_vsweep<1>, grid, block, 0, s, a);
  else if (a.Q <= 2) hipLaunchKernelGGL(k_vsweep<2>, grid, block, 0, s, a);
  else if (a.Q <= 4) hipLaunchKernelGGL(k_vsweep<4>, grid, block, 0, s, a);
  else if (a.Q <= 8) hipLaunchKernelGGL(k_vsweep<8>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_vsweep<16>, grid, block, 0, s, a);
}

void launch_vsweeps(pr_graph *g, VArgs a, int par0, int cnt) {
  for (int s = 0; s < cnt; ++s) {
    a.par = (par0 + s) & 1;
    launch_vsweep(a, g->work);
    hipLaunchKernelGGL(k_vfinal, dim3(a.T), dim3(kVFin), 0, g->work, a);
  }
}

// `cnt` sweeps from a hipGraph cached with the graph's sweep graphs, keyed by
// the launch arguments (which hold no caller pointer), the first sweep's
// parity and the count.  Launches after every column froze exit at once.
int run_vsweeps(pr_graph *g, const VArgs &a, int par0, int cnt, bool use_graph) {
  if (!use_graph) {
    launch_vsweeps(g, a, par0, cnt);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  std::vector<unsigned char> key(1 + sizeof(a) + 2 * sizeof(int));
  key[0] = 'B';
  memcpy(key.data() + 1, &a, sizeof(a));
  const int extra[2] = {par0 & 1, cnt};
  memcpy(key.data() + 1 + sizeof(a), extra, sizeof(extra));
  for (auto &e : g->graph_cache)
    if (e.key == key) {
      PR_HIP(hipGraphLaunch(e.exec, g->work));
      return PR_OK;
    }
  if (g->graph_cache.size() >= 32) {
    for (auto &e : g->graph_cache) (void)hipGraphExecDestroy(e.exec);
    g->graph_cache.clear();
  }
  hipGraph_t graph;
  PR_HIP(hipStreamBeginCapture(g->work, hipStreamCaptureModeThreadLocal));
  launch_vsweeps(g, a, par0, cnt);
  hipError_t le = hipGetLastError();
  hipError_t ce = hipStreamEndCapture(g->work, &graph);
  if (le != hipSuccess) return pr_fail(PR_EDEVICE, "batched launch during capture: %s", hipGetErrorString(le));
  if (ce != hipSuccess) return pr_fail(PR_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ce));
  hipGraphExec_t exec;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return pr_fail(PR_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  g->graph_cache.push_back(GraphEntry{key, exec});
  g->graph_captures++;
  PR_HIP(hipGraphLaunch(exec, g->work));
  return PR_OK;
}

// Runs the T columns starting at col0 of the padded seed list to convergence
// (or exactly fixed_sweeps sweeps when > 0); writes their columns of X.
int run_columns(pr_graph *g, VWork &w, double d, double tol, int max_iter, int T, int col0, float *X, int k,
                int *iters, double *resid, bool write_out, int fixed_sweeps, const pr_batch_shape &sh) {
  if (T < 4 || T > kVMaxT || (T % 4) != 0 || T > w.cols_cap)
    return pr_fail(PR_EDEVICE, "batched: %d columns per launch", T);
  VArgs a = make_vargs(g, w, d, T, col0, sh);
  // one launch holding all k columns keeps its ranks in the caller's X (same
  // row-major layout), with no copy at the end
  const bool direct = write_out && T == k && ((uintptr_t)X % sizeof(float4)) == 0;
  float4 *xp = direct ? reinterpret_cast<float4 *>(X) : w.x;
  VArgs ax = a;  // the kernels launched outside graphs take x directly
  ax.x = xp;
  const int64_t rows = g->n * (int64_t)(T / 4);
  const int zgrid = (int)std::min<int64_t>(4096, (rows + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_vzero, dim3(zgrid), dim3(kBlock), 0, g->work, xp, a.c0, rows);
  hipLaunchKernelGGL(k_vseed, dim3(1), dim3(kVMaxT), 0, g->work, ax, fixed_sweeps > 0 ? -1.0 : tol,
                     fixed_sweeps > 0 ? fixed_sweeps : max_iter);
  PR_HIP(hipGetLastError());
  int rc;
  if ((rc = set_vio(g, w, xp))) return rc;
  const int G = 8;
  int done_sweeps = 0;
  const int limit = fixed_sweeps > 0 ? fixed_sweeps : max_iter;
  for (;;) {
    const int cnt = std::min(G, limit - done_sweeps);
    if ((rc = run_vsweeps(g, a, done_sweeps, cnt, fixed_sweeps == 0))) return rc;
    PR_HIP(hipMemcpyAsync(w.host_st, w.st, sizeof(VState), hipMemcpyDeviceToHost, g->work));
    PR_HIP(hipStreamSynchronize(g->work));
    done_sweeps += cnt;
    bool all = true;
    for (int c = 0; c < T; ++c) all &= w.host_st->done[c] != 0;
    if (all || done_sweeps >= limit) break;
  }
  if (write_out && !direct) {
    const int ogrid = (int)std::min<int64_t>(4096, (g->n * T + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_vout, dim3(ogrid), dim3(kBlock), 0, g->work, ax, X, k, col0);
    PR_HIP(hipGetLastError());
  }
  if (iters && resid) {
    for (int c = 0; c < T; ++c) {
      const int col = col0 + c;
      if (col < k) {
        iters[col] = w.host_st->iters[c];
        resid[col] = w.host_st->resid[c];
      }
    }
  }
  return PR_OK;
}

std::string tune_key(pr_graph *g, int k) {
  hipDeviceProp_t prop;
  char dev[256] = "unknown";
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) snprintf(dev, sizeof(dev), "%s", prop.gcnArchName);
  char buf[512];
  snprintf(buf, sizeof(buf), "n=%lld,m=%lld,sig=%016llx,k=%d,dev=%s", (long long)g->n, (long long)g->m,
           (unsigned long long)g->signature, k, dev);
  return buf;
}

// The launch shape recorded for `key` in the JSON-lines cache file, if any.
bool tune_lookup(const char *path, const std::string &key, pr_batch_shape *out) {
  if (!path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof(line), f)) {
    if (!strstr(line, pat.c_str())) continue;
    const char *t = strstr(line, "\"tile\": ");
    const char *i = strstr(line, "\"items_per_grab\": ");
    const char *w = strstr(line, "\"wg_per_cu\": ");
    if (!t || !i || !w) continue;
    pr_batch_shape s{atoi(t + 8), atoi(i + 18), atoi(w + 13)};
    if (shape_ok(s)) {
      *out = s;
      found = true;
    }
  }
  fclose(f);
  return found;
}

// The tuning cache file is shared by every graph of the process.
std::mutex g_tune_file;

}  // namespace

void fpr_batched_release(pr_graph *g) {
  VWork *w = static_cast<VWork *>(g->vwork);
  if (w) {
    if (w->host_st) (void)hipHostFree(w->host_st);
    delete w;
    g->vwork = nullptr;
  }
  g->tune_memo.clear();
}

extern "C" void pr_batch_shape_default(pr_batch_shape *s) {
  if (!s) return;
  s->tile = kVMaxT;
  s->items_per_grab = 1;
  s->wg_per_cu = 2;
}

extern "C" int pr_autotune_batched(pr_graph *g, int k, const char *cache_path, pr_batch_shape *shape, void *stream) {
  pr_clear_error();
  if (!g || !shape) return pr_fail(PR_EINVAL, "pr_autotune_batched: NULL argument");
  if (k < 1 || k > 1024) return pr_fail(PR_EINVAL, "k=%d outside [1, 1024]", k);
  if (g->weighted) return pr_fail(PR_EINVAL, "pr_autotune_batched: the graph has edge weights (unweighted graphs only)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  const std::string key = tune_key(g, k);
  for (auto &m : g->tune_memo)
    if (m.k == k) {
      *shape = pr_batch_shape{m.tile, m.ipw, m.wg};
      return PR_OK;
    }
  pr_batch_shape cached;
  bool hit;
  {
    std::lock_guard<std::mutex> lock(g_tune_file);
    hit = tune_lookup(cache_path, key, &cached);
  }
  if (hit) {
    *shape = cached;
    g->tune_memo.push_back(pr_graph::TuneMemo{k, cached.tile, cached.items_per_grab, cached.wg_per_cu});
    return PR_OK;
  }
  hipStream_t user = (hipStream_t)stream;
  (void)hipEventRecord(g->ev_in, user);
  (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  VWork &w = *vwork_for(g);
  const int kpad = (k + 3) / 4 * 4;
  int rc;
  if ((rc = ensure_seeds(g, w, kpad))) return rc;
  // tuning seeds: vertices 0.. (the timing does not depend on which)
  std::vector<int32_t> hs(kpad);
  for (int i = 0; i < kpad; ++i) hs[i] = i < k ? (int32_t)(i % g->n) : -1;
  PR_HIP(hipMemcpyAsync(w.seeds, hs.data(), sizeof(int32_t) * kpad, hipMemcpyHostToDevice, g->work));
  hipEvent_t e0, e1;
  PR_HIP(hipEventCreate(&e0));
  PR_HIP(hipEventCreate(&e1));
  double best_t = INFINITY;
  pr_batch_shape best{4, 1, 2};
  const int sweeps = 4;
  // tile widths 8..64 (4 when k is that small), items per grab 1/2/4,
  // one or two sweep workgroups per compute unit: the results are the same
  // bits for every shape, only the time differs
  for (int t = std::min(8, std::max(4, kpad)); t <= std::max(4, std::min(kVMaxT, kpad)); t *= 2) {
    if ((rc = ensure_vwork(g, w, t))) return rc;
    for (int ipg : {1, 2, 4})
      for (int wg : {1, 2}) {
        const pr_batch_shape sh{t, ipg, wg};
        // one warm-up, one timed run of `sweeps` sweeps on t columns
        if ((rc = run_columns(g, w, 0.85, 1.0, sweeps, t, 0, nullptr, k, nullptr, nullptr, false, sweeps, sh)))
          return rc;
        PR_HIP(hipEventRecord(e0, g->work));
        if ((rc = run_columns(g, w, 0.85, 1.0, sweeps, t, 0, nullptr, k, nullptr, nullptr, false, sweeps, sh)))
          return rc;
        PR_HIP(hipEventRecord(e1, g->work));
        PR_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        PR_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double per_col = ms / (double)t;
        if (per_col < best_t) {
          best_t = per_col;
          best = sh;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventRecord(g->ev_out, g->work);
  (void)hipStreamWaitEvent(user, g->ev_out, 0);
  *shape = best;
  g->tune_memo.push_back(pr_graph::TuneMemo{k, best.tile, best.items_per_grab, best.wg_per_cu});
  if (cache_path) {
    std::lock_guard<std::mutex> lock(g_tune_file);
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{\"key\": \"%s\", \"tile\": %d, \"items_per_grab\": %d, \"wg_per_cu\": %d, "
                 "\"ms_per_column_sweep\": %.6f}\n",
              key.c_str(), best.tile, best.items_per_grab, best.wg_per_cu, best_t / sweeps);
      fclose(f);
    }
  }
  return PR_OK;
}

extern "C" int pr_solve_batched(pr_graph *g, double d, double tol, int max_iter, int k,
                                const int32_t *seeds, const pr_batch_shape *shape, float *X, int *iters,
                                double *resid, void *stream) {
  pr_clear_error();
  if (!g) return pr_fail(PR_EINVAL, "graph is NULL");
  if (!(d > 0.0 && d < 1.0)) return pr_fail(PR_EINVAL, "d=%g is not in (0, 1)", d);
  if (!(tol > 0.0)) return pr_fail(PR_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return pr_fail(PR_EINVAL, "max_iter=%d must be >= 1", max_iter);
  if (k < 1 || k > 1024) return pr_fail(PR_EINVAL, "k=%d outside [1, 1024]", k);
  if (!seeds || !X || !iters || !resid) return pr_fail(PR_EINVAL, "NULL argument");
  if (g->weighted) return pr_fail(PR_EINVAL, "pr_solve_batched: the graph has edge weights (unweighted graphs only)");
  if (shape && !shape_ok(*shape))
    return pr_fail(PR_EINVAL,
                   "shape {tile %d, items_per_grab %d, wg_per_cu %d}: need a tile that is a multiple of 4 up to "
                   "%d, 1..16 items per grab, 1 or 2 workgroups per compute unit",
                   shape->tile, shape->items_per_grab, shape->wg_per_cu, kVMaxT);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  int rc;
  pr_batch_shape sh;
  if (shape) {
    sh = *shape;
  } else if ((rc = pr_autotune_batched(g, k, getenv("FUSEDPR_TUNE_CACHE"), &sh, stream))) {
    return rc;
  }
  hipStream_t user = (hipStream_t)stream;
  (void)hipEventRecord(g->ev_in, user);
  (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  VWork &w = *vwork_for(g);
  const int kpad = (k + 3) / 4 * 4;
  const int per_launch = std::min(kpad, sh.tile);
  if ((rc = ensure_seeds(g, w, kpad))) return rc;
  if ((rc = ensure_vwork(g, w, per_launch))) return rc;
  hipLaunchKernelGGL(k_vseeds, dim3((kpad + 255) / 256), dim3(256), 0, g->work, seeds, k, w.seeds, kpad);
  hipLaunchKernelGGL(k_vclear, dim3(1), dim3(1), 0, g->work, w.flag);
  hipLaunchKernelGGL(k_vcheck, dim3((k + 255) / 256), dim3(256), 0, g->work, seeds, k, (int64_t)g->n, w.flag);
  int bad = 0;
  PR_HIP(hipMemcpyAsync(&bad, w.flag, sizeof(int), hipMemcpyDeviceToHost, g->work));
  PR_HIP(hipStreamSynchronize(g->work));
  if (bad) return pr_fail(PR_EINVAL, "a seed vertex is outside [0, %lld)", (long long)g->n);
  for (int c0 = 0; c0 < kpad; c0 += per_launch) {
    const int T = std::min(per_launch, kpad - c0);
    if ((rc = run_columns(g, w, d, tol, max_iter, T, c0, X, k, iters, resid, true, 0, sh))) return rc;
  }
  PR_HIP(hipStreamSynchronize(g->work));
  (void)hipEventRecord(g->ev_out, g->work);
  (void)hipStreamWaitEvent(user, g->ev_out, 0);
  for (int j = 0; j < k; ++j)
    if (!(resid[j] < tol)) return PR_NOT_CONVERGED;
  return PR_OK;
}
