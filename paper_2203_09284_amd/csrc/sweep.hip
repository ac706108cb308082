// The PageRank sweep on gfx950: one persistent kernel per sweep that pulls,
// updates, and reduces, in the two forms of the paper.
//
//  * Jacobi (Section 3, Algorithm 1): contributions are double-buffered; sweep
//    k reads c_k and writes c_{k+1}, so every vertex sees the previous sweep.
//  * Fused (Section 4, Algorithm 2; Eq. 9): Gauss-Seidel over blocks of
//    vertices.  The plan cuts the vertices into blocks (hubs and high
//    out-degree first) whose gather slots are contiguous; the sweep launches
//    the kernel once per block, and a gather of a slot that belongs to an
//    earlier block reads the contribution written in this sweep, every other
//    gather the previous sweep's.  Kernel boundaries are the only points where
//    all of a launch's writes are visible to every XCD, so the blocks, not
//    individual vertices, are the Gauss-Seidel units; within a block the sweep
//    is Jacobi, which keeps it deterministic.
//
// Per vertex u the update is Eq. 1 with the dangling mass D spread uniformly,
//     x_u <- (1-d) p_u s + d (sum_{v->u} w c_v + D/n),   c_u <- x_u / W_u,
// where s = 1, except in the fused mass-scaled mode where s is the previous
// sweep's total mass (see the mode flag kFlagScaled).  The per-vertex change,
// the new dangling mass and the new total mass are reduced in FP64 per
// workgroup; a one-workgroup finalize kernel after each sweep sums the
// workgroup partials in a fixed order (deterministic) and sets the residual,
// the iteration count and the stop flag, so the next sweep needs no host
// work.  The hot kernel has no fences
// and no atomics.
//
// Work layout: a few workgroups per CU; each keeps the hottest slots of the
// gathered array in LDS and its wavefronts take work items round-robin; an
// item is a tile of short rows, a long row (a wavefront), a hub (all
// wavefronts of a workgroup), or a run of vertices without in-edges.
//
// FP32 storage (ranks and contributions) sums with Neumaier compensation per
// lane and TwoSum when lanes combine; the rank update and every reduction are
// FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "internal.h"

using namespace fpr;
using namespace fpr::dev;

namespace {

// Streaming accesses (graph arrays read once per sweep, per-vertex operands)
// can be issued non-temporal so they do not displace the gathered
// contributions from the caches: FPR_NT=1 for the reads and the rank store,
// FPR_NT=2 also for the contribution store.
#ifndef FPR_NT
#define FPR_NT 0
#endif
template <typename V>
__device__ __forceinline__ V sld(const V *p) {
  if constexpr (FPR_NT >= 1) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename V>
__device__ __forceinline__ void sst_x(V *p, V v) {
  if constexpr (FPR_NT >= 1) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <typename V>
__device__ __forceinline__ void sst_c(V *p, V v) {
  if constexpr (FPR_NT >= 2) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Weighted edge value: the product rounded on its own (never fused into the
// following add), so every form that sums it gets the same bits.
template <typename T>
__device__ __forceinline__ T wmul(T v, double w) {
#pragma clang fp contract(off)
  return (T)((double)v * w);
}

// ------------------------------------------------------------ arguments --

// How a sweep reads the value of an in-edge: gathered from the contribution
// array (plain, or times the edge weight), or read from the edge-ordered
// contributionList that a scatter kernel filled (weights already applied).
enum SweepMode : int { kModePlain = 0, kModeWeighted = 1, kModeList = 2 };

template <typename T>
constexpr int kHotSlots = kHotBytes / (int)sizeof(T);

template <typename T>
struct SweepArgs {
  const uint32_t *rows;
  const uint32_t *rowpos;
  const uint32_t *rptr;
  const int32_t *idx;
  const double *w;
  const int4 *items;
  const int4 *tiles;
  const int4 *msplit;  // hubs split into chunk items: {row index, first slot, chunks, 0}
  double *hpart;       // chunk sums
  const int32_t *tidx;
  const double *tw;
  const uint8_t *tmask;
  double *wave_part;
  SweepState *st;
  const double *inv_w;
  const IoPtrs *io;  // the caller's x and p, read when the kernel starts
  T *c0;
  T *c1;
  const T *cl;
  uint32_t cl_rows;
  double *trace;
  double d;
  double inv_n;
  int64_t nv;  // vertices
  int n_items;
  int n_msplit;
  int chunk;
  int n_waves;
  int hot;  // gather slots staged in LDS (<= kHotSlots<T>)
  int flags;
  // launch-specific: the blocks [blk_lo, blk_hi) of this launch, where its
  // workgroup partials go, and what the finalize kernel sums
  const int *block_pos;  // first list position of each block
  const int *wave_cnt;   // [block][wavefront] list lengths
  int blk_lo, blk_hi;
  int part_base;    // first partial slot written by this launch
  int part_stride;  // SoA stride of the three partial rows
  int n_part;       // partial slots the finalize kernel sums
  int fresh_lo, fresh_hi;  // slots rewritten by earlier blocks of this sweep (fused form)
  const int32_t *ip_range;  // in-place form: first block of each wavefront, [W+1]
};

template <typename T>
struct Ctx {
  const uint32_t *rows;
  const uint32_t *rowpos;
  const uint32_t *rptr;
  const int32_t *idx;
  const double *w;
  const double *inv_w;
  const double *p;
  T *x;
  const T *cl;        // contributionList (list mode), in the plan's edge positions
  uint32_t cl_rows;   // position of the first list edge (after the tiles)
  const T *cin;  // contributions of the previous sweep
  T *cout;       // contributions of this sweep
  double tele;   // (1-d) * mass scale
  double d;
  double dterm;  // D / n, 0 in leak mode
  double inv_n;
  int hot;
  int fresh_lo;  // gather slots [fresh_lo, fresh_lo + fresh_n) are read from cout
  int fresh_n;   // (earlier Gauss-Seidel blocks of this sweep)
  int flags;
};

// The iterate's state as of the start of the sweep (written by the previous
// finalize kernel) and the buffers it selects.
template <typename T, bool FUSED>
__device__ __forceinline__ Ctx<T> make_ctx(const SweepArgs<T> &a, const SweepState *st) {
  const int it = st->iter;
  const double S = st->S, D = st->D;
  Ctx<T> C;
  C.rows = a.rows;
  C.rowpos = a.rowpos;
  C.rptr = a.rptr;
  C.idx = a.idx;
  C.w = a.w;
  C.inv_w = a.inv_w;
  C.p = a.io->p;
  C.x = static_cast<T *>(a.io->x);
  C.cl = a.cl;
  C.cl_rows = a.cl_rows;
  C.cin = (it & 1) ? a.c1 : a.c0;
  C.cout = (it & 1) ? a.c0 : a.c1;
  C.fresh_lo = a.fresh_lo;
  C.fresh_n = FUSED ? a.fresh_hi - a.fresh_lo : 0;
  C.d = a.d;
  C.inv_n = a.inv_n;
  C.hot = a.hot;
  C.flags = a.flags;
  if (a.flags & kFlagAdjoint) {
    C.tele = 1.0;              // lam' = g + ...
    C.dterm = S * a.inv_n;     // added for dangling vertices only
  } else {
    C.tele = (1.0 - a.d) * ((a.flags & kFlagScaled) ? S : 1.0);
    C.dterm = (a.flags & kFlagLeak) ? 0.0 : D * a.inv_n;
  }
  return C;
}

// Row-table entry i: vertex u = rows[i], its gather slot rowpos[i].
template <typename T, bool FUSED>
__device__ __forceinline__ void update_loaded(const Ctx<T> &C, T *hot, uint32_t u, uint32_t slot,
                                              double xo, double iw, double pu, double s, Red &red);

template <typename T, bool FUSED>
__device__ __forceinline__ void update_vertex(const Ctx<T> &C, T *hot, int i, double s, Red &red) {
  const uint32_t u = sld(C.rows + i);
  const double pu = (C.flags & kFlagUniformP) ? C.inv_n : sld(C.p + u);
  update_loaded<T, FUSED>(C, hot, u, sld(C.rowpos + i), (double)sld(C.x + u), sld(C.inv_w + u), pu, s, red);
}

// The update of vertex u from its pulled sum s, with its operands loaded:
// old value xo, 1/W_u (iw), teleport (or adjoint right-hand side) pu, and the
// slot of u in the gather layout.
//   forward: x' = (1-d) p_u s + d (sum + D/n),  gathered value x' / W_u
//   adjoint: x' = g_u + d (sum / W_u + [W_u = 0] S/n),  gathered value x'
template <typename T, bool FUSED>
__device__ __forceinline__ void update_loaded(const Ctx<T> &C, T *hot, uint32_t u, uint32_t slot,
                                              double xo, double iw, double pu, double s, Red &red) {
  const bool adj = (C.flags & kFlagAdjoint) != 0;
  const double xn = adj ? pu + C.d * (iw * s + (iw == 0.0 ? C.dterm : 0.0))
                        : C.tele * pu + C.d * (s + C.dterm);
  const T xs = (T)xn;
  sst_x(C.x + u, xs);
  const double xd = (double)xs;
  if ((adj || iw != 0.0) && !(C.flags & kFlagList)) {
    sst_c(C.cout + slot, adj ? xs : (T)(xd * iw));
  }
  if (iw == 0.0) red.dang += xd;
  const double dl = fabs(xd - xo);
  red.chg = (C.flags & kFlagLinf) ? fmax(red.chg, dl) : red.chg + dl;
  red.tot += xd;
}

// The array slot s is read from: this sweep's contributions for slots of
// earlier Gauss-Seidel blocks (fused form), the previous sweep's otherwise.
template <typename T, bool FUSED>
__device__ __forceinline__ const T *src_of(const Ctx<T> &C, int32_t s) {
  return FUSED && (uint32_t)(s - C.fresh_lo) < (uint32_t)C.fresh_n ? C.cout : C.cin;
}

// Gather of slot s (always a valid slot).  Both the LDS copy and the global
// array are read unconditionally, at slot 0 of the side that is not used, and
// the value is selected: this keeps the gathers of a batch independent (no
// branch, no address-space select that would turn them into flat loads).
//
// The global side is read through an address-space-1 (global) pointer: a
// generic pointer would let the compiler fold the two loads into one flat
// load of a selected address, which serialises on both wait counters.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

template <typename T, bool FUSED>
__device__ __forceinline__ T gather(const Ctx<T> &C, const T *hot, int32_t s) {
  const bool h = s < C.hot;
  const T vh = hot[h ? s : 0];
  // global load only on the lanes whose slot is not in LDS
  T vg = vh;
  if (!h) vg = ((gptr<T>)src_of<T, FUSED>(C, s))[s];
  return vg;
}

// ---------------------------------------------------- work item kinds --

// A wavefront works on 64/lpr consecutive rows at a time, lpr lanes per row;
// each lane issues up to kBatch index loads, then kBatch gathers, per batch.
// The lpr partial sums of a row combine by a butterfly inside the lane group.
// The list bounds of up to kPrefetch rounds are loaded before the first round,
// and each round issues its rank-update loads before its gathers, so a round
// costs about two dependent memory latencies.
template <typename T, bool FUSED, int MODE>
__device__ __forceinline__ void row_group(const Ctx<T> &C, T *hot, int i0, int i1, int lpr,
                                          Red &red) {
  constexpr bool WEIGHTED = MODE == kModeWeighted, CL = MODE == kModeList;
  const int lane = threadIdx.x & 63;
  const int q = lane & (lpr - 1);
  const int g = lane / lpr;
  const int per = 64 / lpr;
  for (int rb = i0; rb < i1; rb += per * kPrefetch) {
    uint32_t eb[kPrefetch];
    int len[kPrefetch];
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const int r = rb + k * per + g;
      eb[k] = 0;
      len[k] = 0;
      if (r < i1) {
        eb[k] = sld(C.rptr + (r));
        len[k] = (int)(sld(C.rptr + (r + 1)) - eb[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const int r = rb + k * per + g;
      if (rb + k * per >= i1) break;
      const bool active = r < i1;
      const bool owner = active && q == 0;
      // rank-update operands, loaded ahead of the gathers
      uint32_t u = 0, slot = 0;
      double xo = 0.0, iw = 0.0, pu = C.inv_n;
      if (owner) {
        u = sld(C.rows + (r));
        slot = sld(C.rowpos + (r));
        xo = (double)sld(C.x + (u));
        iw = sld(C.inv_w + (u));
        if (!(C.flags & kFlagUniformP)) pu = sld(C.p + (u));
      }
      const uint32_t e0 = eb[k];
      const int L = len[k];
      LaneSum<T> acc;
      for (int j0 = q; j0 < L; j0 += kBatch * lpr) {
        int32_t s[kBatch];
        double wt[kBatch];
        T v[kBatch];
        if constexpr (CL) {
#pragma unroll
          for (int b = 0; b < kBatch; ++b) {
            const int j = j0 + b * lpr;
            v[b] = j < L ? sld(C.cl + (C.cl_rows + e0 + j)) : (T)0;
          }
        } else {
#pragma unroll
          for (int b = 0; b < kBatch; ++b) {
            const int j = j0 + b * lpr;
            s[b] = j < L ? sld(C.idx + (e0 + j)) : 0;
            if constexpr (WEIGHTED) wt[b] = j < L ? sld(C.w + (e0 + j)) : 0.0;
          }
#pragma unroll
          for (int b = 0; b < kBatch; ++b) v[b] = gather<T, FUSED>(C, hot, s[b]);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          T x = j0 + b * lpr < L ? v[b] : (T)0;
          if constexpr (WEIGHTED) x = wmul(x, wt[b]);
          acc.add(x);
        }
      }
      acc.group_reduce(lpr);
      if (owner) update_loaded<T, FUSED>(C, hot, u, slot, xo, iw, pu, acc.value(), red);
    }
  }
}

// A tile of consecutive rows r0.. (nr <= kTileRows rows, ne <= kTileEdges
// edges, all given by the work item).  Lane
// l loads edges 8l..8l+7 (lane-transposed storage: each load instruction reads
// 256 contiguous bytes), gathers them, and sums runs between row starts.  A
// row that starts in lane a and ends in lane b > a is completed by a
// segmented inclusive scan over the lanes: lane values are the sum after the
// lane's last row start (or the whole lane when it has none), segments reset
// at lanes that hold a row start.  Completed row sums go to the wavefront's
// LDS slice; then lane r updates rows r and r + 64 with operands it loaded
// before the gathers.
template <typename T, bool FUSED, int MODE>
__device__ __forceinline__ void tile_rows(const Ctx<T> &C, const SweepArgs<T> &a, T *hot,
                                          double *rowsum, int t, int r0, int nr, int ne, Red &red) {
  constexpr bool WEIGHTED = MODE == kModeWeighted, CL = MODE == kModeList;
  const int lane = threadIdx.x & 63;
  // rank-update operands of rows r0 + lane and r0 + 64 + lane
  uint32_t u[2] = {0, 0}, slot[2] = {0, 0};
  double xo[2] = {0.0, 0.0}, iw[2] = {0.0, 0.0}, pu[2] = {C.inv_n, C.inv_n};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = lane + 64 * k;
    if (r < nr) {
      u[k] = sld(C.rows + (r0 + r));
      slot[k] = sld(C.rowpos + (r0 + r));
      xo[k] = (double)sld(C.x + u[k]);
      iw[k] = sld(C.inv_w + u[k]);
      if (!(C.flags & kFlagUniformP)) pu[k] = sld(C.p + u[k]);
    }
  }
  const size_t base = (size_t)t * kTileEdges;
  const uint32_t fl = sld(a.tmask + ((size_t)t * 64 + lane));
  T v[kBatch];
  if constexpr (CL) {
#pragma unroll
    for (int k = 0; k < kBatch; ++k) v[k] = sld(C.cl + (base + k * 64 + lane));
  } else {
    int32_t s[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) s[k] = sld(a.tidx + (base + k * 64 + lane));
#pragma unroll
    for (int k = 0; k < kBatch; ++k) v[k] = gather<T, FUSED>(C, hot, s[k]);
  }
#pragma unroll
  for (int k = 0; k < kBatch; ++k) {
    if constexpr (WEIGHTED) v[k] = wmul(v[k], sld(a.tw + (base + k * 64 + lane)));  // padding weight 0
    else v[k] = lane * kBatch + k < ne ? v[k] : (T)0;
  }
  // row index (within the tile) of this lane's first row start
  const int pc = __popc(fl);
  const int rowbase = wave_incl_scan(pc) - pc;
  // lane-local runs: head = before the first start, complete rows, tail = after the last start
  LaneSum<T> cur, head;
  bool seen = false;
  int j = 0;
#pragma unroll
  for (int k = 0; k < kBatch; ++k) {
    const bool st = (fl >> k) & 1u;
    if (st && seen) rowsum[rowbase + j - 1] = cur.value();
    head = (st && !seen) ? cur : head;
    j += st ? 1 : 0;
    seen = seen || st;
    cur = st ? LaneSum<T>() : cur;
    cur.add(v[k]);
  }
  if (!seen) head = cur;
  // segmented inclusive scan over lanes of (flag, value), then each lane's
  // predecessor (lane 0 reads zero)
  LaneSum<T> sc = cur;
  seg_scan<T>(sc, seen);
  LaneSum<T> carry = sc.template dpp<kDppWaveShr1>();
  if (seen && lane > 0) {
    carry.combine_with(head);
    rowsum[rowbase - 1] = carry.value();
  }
  if (lane == ((ne - 1) >> 3)) rowsum[nr - 1] = sc.value();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = lane + 64 * k;
    if (r < nr) update_loaded<T, FUSED>(C, hot, u[k], slot[k], xo[k], iw[k], pu[k], rowsum[r], red);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Vertices without in-edges: lane per vertex, the update only.
template <typename T, bool FUSED>
__device__ __forceinline__ void zero_rows(const Ctx<T> &C, T *hot, int i0, int i1, Red &red) {
  const int lane = threadIdx.x & 63;
  for (int r = i0 + lane; r < i1; r += 64) update_vertex<T, FUSED>(C, hot, r, 0.0, red);
}

// One `chunk`-edge piece of a very long hub list per wavefront; the piece sum
// goes to its slot and the finalize kernel adds the pieces in order.
template <typename T, bool FUSED, int MODE>
__device__ __forceinline__ void hub_chunk(const Ctx<T> &C, const T *hot, double *hpart, int chunk, int i, int c,
                                          int slot) {
  constexpr bool WEIGHTED = MODE == kModeWeighted, CL = MODE == kModeList;
  const int lane = threadIdx.x & 63;
  const uint32_t rb = sld(C.rptr + (i));
  const int L = (int)(sld(C.rptr + (i + 1)) - rb);
  const uint32_t eb = rb + (uint32_t)c * (uint32_t)chunk;
  const int ne = min(chunk, L - c * chunk);
  LaneSum<T> acc;
  for (int j0 = lane; j0 < ne; j0 += kBatch * 64) {
    int32_t s[kBatch];
    double wt[kBatch];
    T v[kBatch];
    if constexpr (CL) {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int j = j0 + 64 * k;
        v[k] = j < ne ? sld(C.cl + (C.cl_rows + eb + j)) : (T)0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int j = j0 + 64 * k;
        s[k] = j < ne ? sld(C.idx + (eb + j)) : 0;
        if constexpr (WEIGHTED) wt[k] = j < ne ? sld(C.w + (eb + j)) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) v[k] = gather<T, FUSED>(C, hot, s[k]);
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      T x = j0 + 64 * k < ne ? v[k] : (T)0;
      if constexpr (WEIGHTED) x = wmul(x, wt[k]);
      acc.add(x);
    }
  }
  acc.group_reduce(64);
  if (lane == 0) hpart[slot + c] = acc.value();
}

// A hub (list longer than the plan's chunk, at most 8 chunks) is an item of a
// whole workgroup:
// the plan gives it to all 8 wavefronts of one workgroup in the same round.
// Wavefront k sums the 512-edge pieces k, k+8, k+16, ... of the list; the 8
// sums meet in LDS and wavefront 0 adds them in wavefront order and updates
// the row.  `par` alternates the LDS buffer between consecutive hub items.
template <typename T, bool FUSED, int MODE>
__device__ __forceinline__ void hub_wg(const Ctx<T> &C, const T *hot, double (*s_hub)[kSweepWaves], int &par,
                                       int i, Red &red) {
  constexpr bool WEIGHTED = MODE == kModeWeighted, CL = MODE == kModeList;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t rb = sld(C.rptr + (i));
  const int L = (int)(sld(C.rptr + (i + 1)) - rb);
  uint32_t u = 0, slot = 0;
  double xo = 0.0, iw = 0.0, pu = C.inv_n;
  if (wave == 0 && lane == 0) {
    u = sld(C.rows + (i));
    slot = sld(C.rowpos + (i));
    xo = (double)sld(C.x + (u));
    iw = sld(C.inv_w + (u));
    if (!(C.flags & kFlagUniformP)) pu = sld(C.p + (u));
  }
  LaneSum<T> acc;
  for (int j0 = wave * (kBatch * 64) + lane; j0 < L; j0 += kSweepWaves * kBatch * 64) {
    int32_t sl[kBatch];
    double wt[kBatch];
    T v[kBatch];
    if constexpr (CL) {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int j = j0 + 64 * k;
        v[k] = j < L ? sld(C.cl + (C.cl_rows + rb + j)) : (T)0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int j = j0 + 64 * k;
        sl[k] = j < L ? sld(C.idx + (rb + j)) : 0;
        if constexpr (WEIGHTED) wt[k] = j < L ? sld(C.w + (rb + j)) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) v[k] = gather<T, FUSED>(C, hot, sl[k]);
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      T x = j0 + 64 * k < L ? v[k] : (T)0;
      if constexpr (WEIGHTED) x = wmul(x, wt[k]);
      acc.add(x);
    }
  }
  acc.group_reduce(64);
  if (lane == 0) s_hub[par][wave] = acc.value();
  __syncthreads();
  if (wave == 0 && lane == 0) {
    double tot = 0.0;
    for (int k = 0; k < kSweepWaves; ++k) tot += s_hub[par][k];
    update_loaded<T, FUSED>(C, nullptr, u, slot, xo, iw, pu, tot, red);
  }
  par ^= 1;
}

// A few workgroups per CU.  The workgroup first copies the hottest gather
// slots (the first `hot` of the gather layout) into LDS, then each wavefront
// works through its own list of items in each block of the launch (the plan
// deals the items to wavefronts, longest first, to balance them).
// Every wavefront accumulates its rows' change / dangling / total mass; the
// workgroup writes one partial of each; a fixed item-to-wavefront map keeps
// the sums reproducible.
#ifndef FPR_WAVES_PER_EU
#define FPR_WAVES_PER_EU 4
#endif

// Copy of the hot slots [0, C.hot) into LDS with 16-byte loads, all issued
// before the first LDS write (one memory latency per launch, not one per
// slot).  A 16-byte group that straddles the fresh range falls back to one
// load per slot.
template <typename T, bool FUSED>
__device__ __forceinline__ void load_hot(const Ctx<T> &C, T *hot) {
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int kPer = (kHotSlots<T> / V + kSweepBlock - 1) / kSweepBlock;
  const int nvec = C.hot / V;
  uint4 buf[kPer];
  bool mixed[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int q = (int)threadIdx.x + k * kSweepBlock;
    mixed[k] = false;
    buf[k] = make_uint4(0, 0, 0, 0);
    if (q < nvec) {
      const int s0 = q * V;
      const T *src = src_of<T, FUSED>(C, s0);
      mixed[k] = FUSED && src_of<T, FUSED>(C, s0 + V - 1) != src;
      buf[k] = *reinterpret_cast<const uint4 *>(src + s0);
    }
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int q = (int)threadIdx.x + k * kSweepBlock;
    if (q < nvec) {
      *reinterpret_cast<uint4 *>(hot + q * V) = buf[k];
      if (mixed[k])
        for (int j = 0; j < V; ++j) hot[q * V + j] = src_of<T, FUSED>(C, q * V + j)[q * V + j];
    }
  }
  for (int s = nvec * V + (int)threadIdx.x; s < C.hot; s += kSweepBlock) hot[s] = src_of<T, FUSED>(C, s)[s];
}

template <typename T, bool FUSED, int MODE>
__global__ __launch_bounds__(kSweepBlock) __attribute__((amdgpu_waves_per_eu(FPR_WAVES_PER_EU)))
void k_sweep(SweepArgs<T> a) {
  constexpr bool WEIGHTED = MODE == kModeWeighted, CL = MODE == kModeList;
  __shared__ __align__(16) T hot[kHotSlots<T>];
  __shared__ double rowsum_all[kSweepWaves][kTileRows];
  __shared__ double s_part[3][kSweepWaves];
  __shared__ double s_hub[2][kSweepWaves];
  const SweepState *st = a.st;
  if (st->done) return;
  const Ctx<T> C = make_ctx<T, FUSED>(a, st);
  const int wave = threadIdx.x >> 6;
  const int gw = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kSweepWaves + wave));
  // the first block's list length and first item record are loaded while the
  // hot set is staged
  int base = a.block_pos[a.blk_lo];
  int cnt = a.wave_cnt[(size_t)a.blk_lo * a.n_waves + gw];
  int4 next = cnt > 0 ? a.items[base + gw] : make_int4(kZero, 0, 0, 0);
  if constexpr (!CL) load_hot<T, FUSED>(C, hot);
  __syncthreads();
  Red red;
  int par = 0;
  double *rowsum = rowsum_all[wave];
  for (int b = a.blk_lo; b < a.blk_hi; ++b) {
    if (b != a.blk_lo) {
      base = a.block_pos[b];
      cnt = a.wave_cnt[(size_t)b * a.n_waves + gw];
      next = cnt > 0 ? a.items[base + gw] : make_int4(kZero, 0, 0, 0);
    }
    // the next item's record is loaded while the current one runs
    for (int k = 0; k < cnt; ++k) {
      const int4 wi = next;
      if (k + 1 < cnt) next = a.items[base + (k + 1) * a.n_waves + gw];
      if (wi.x == kTile) tile_rows<T, FUSED, MODE>(C, a, hot, rowsum, wi.y, wi.z, wi.w >> 16, wi.w & 0xffff, red);
      else if (wi.x == kRows) row_group<T, FUSED, MODE>(C, hot, wi.y, wi.z, wi.w, red);
      else if (wi.x == kHubWG) hub_wg<T, FUSED, MODE>(C, hot, s_hub, par, wi.y, red);
      else if (wi.x == kHeavy) hub_chunk<T, FUSED, MODE>(C, hot, a.hpart, a.chunk, wi.y, wi.z, wi.w);
      else zero_rows<T, FUSED>(C, hot, wi.y, wi.z, red);
    }
  }
  // one partial per workgroup: wavefront sums, then the waves in order
  const bool linf = (a.flags & kFlagLinf) != 0;
  const double chg = linf ? wave_max(red.chg) : wave_sum(red.chg);
  const double dang = wave_sum(red.dang);
  const double tot = wave_sum(red.tot);
  if ((threadIdx.x & 63) == 0) {
    s_part[0][wave] = chg;
    s_part[1][wave] = dang;
    s_part[2][wave] = tot;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int r = threadIdx.x;
    double v = s_part[r][0];
    for (int k = 1; k < kSweepWaves; ++k) v = (r == 0 && linf) ? fmax(v, s_part[r][k]) : v + s_part[r][k];
    a.wave_part[(size_t)r * a.part_stride + a.part_base + blockIdx.x] = v;
  }
}

// The in-place form (Algorithm 2 / Eq. 9 swept in place, Section 4.3's
// asynchronous blocks).  The contributions live in one array c, read and
// written during the sweep.  Wavefront w takes a contiguous range of the
// blocks of kIpVpb consecutive vertices, in ascending order (on a grid in
// row-major order this reads more values of the same sweep than blocks dealt
// round robin: 42 sweeps to 1e-8 instead of 60); for each block it copies the block's
// contributions into its own LDS slice, then updates the block in kIpRun
// steps: in step k lane l updates vertex l * kIpRun + k of the block, so each
// lane walks its own run of consecutive vertices in order.  The plan stores
// the block interleaved (that vertex at position 64 k + l, in c and in every
// per-position array), so the 64 lanes of a step read and write consecutive
// positions; only p is read by vertex.  There is no rank array: a vertex's
// slot of c holds x / W, or x itself for a dangling vertex (never gathered),
// and the ranks are read back from c after the last sweep.
// A source inside the block is read from LDS, where it already holds this
// sweep's value once its lane has passed it (the earlier vertices of every
// run); a source outside the block is read from c as it stands, this sweep's
// value if it has reached this wavefront's caches, the previous one if not
// (the asynchrony that Section 4.3 allows; a write from another XCD may not
// be seen before the launch ends).
// Within a step the rows use the values from before the step: lanes sum the
// rows of up to kIpShort in-edges themselves (kBatch loads in flight), then
// the wavefront sums the longer rows of the step one by one, its 64 lanes
// striding the list.
// The update is Eq. 1 with the lagged dangling mass and, with kFlagScaled,
// the mass-scaled teleport of the fused form; the new contribution goes to
// LDS and to c, and the change |x' - x| is read off c.  Reductions as in
// k_sweep (one partial per workgroup).
constexpr int kIpShort = 32;  // longest row a single lane sums

// Edge e's value for the in-place form (ok: e is an edge of the row; a lane
// past the row's end reads nothing from memory): from the block's LDS copy
// when the source s lies in the block, else from the shared array (the global
// load runs only on the lanes that need it, so a batch stays branch-free).
template <typename T, bool WEIGHTED>
__device__ __forceinline__ T ip_value(const SweepArgs<T> &a, const T *blk, const T *c, int64_t b0, int nb,
                                      int32_t s, uint32_t e, bool ok) {
  const uint32_t ls = (uint32_t)((int64_t)s - b0);
  const bool in = ls < (uint32_t)nb;
  const T vh = blk[in ? ls : 0];
  T v = vh;
  if (ok && !in) v = ((gptr<T>)c)[s];
  if constexpr (WEIGHTED) v = ok ? wmul(v, sld(a.w + e)) : (T)0;
  return v;
}

template <typename T, bool WEIGHTED>
__global__ __launch_bounds__(kSweepBlock) __attribute__((amdgpu_waves_per_eu(FPR_WAVES_PER_EU)))
void k_inplace(SweepArgs<T> a) {
  constexpr int VPB = kIpVpb;
  constexpr int PER = kIpRun;
  __shared__ __align__(16) T blk_all[kSweepWaves][VPB];
  __shared__ double s_part[3][kSweepWaves];
  const SweepState *st = a.st;
  if (st->done) return;
  const Ctx<T> C = make_ctx<T, true>(a, st);
  T *c = C.cout;  // == C.cin: one array, in place
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T *blk = blk_all[wave];
  const int64_t W = (int64_t)gridDim.x * kSweepWaves;
  const int64_t nblocks = (a.nv + VPB - 1) / VPB;
  // each wavefront takes its contiguous range of blocks (the plan cuts them
  // at equal cost), in ascending order
  const int64_t gw = (int64_t)blockIdx.x * kSweepWaves + wave;
  const int64_t bend = gw < W ? min(nblocks, (int64_t)a.ip_range[gw + 1]) : 0;
  Red red;
  for (int64_t b = gw < W ? a.ip_range[gw] : 0; b < bend; ++b) {
    const int64_t b0 = b * VPB;
    const int nb = (int)min((int64_t)VPB, a.nv - b0);
    {
      // the block's contributions into LDS: every load issued before the
      // first LDS write (one memory round trip per block)
      T v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) v[k] = lane + 64 * k < nb ? c[b0 + lane + 64 * k] : (T)0;
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (lane + 64 * k < nb) blk[lane + 64 * k] = v[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // step k: lane l takes position b0 + 64 k + l, which holds vertex
    // b0 + l * PER + k of a full block (the k-th of the lane's run), vertex
    // b0 + 64 k + l of the last, partial block
    const bool full = nb == VPB;
    for (int k = 0; k < PER; ++k) {
      const int i = k * 64 + lane;
      const bool act = i < nb;
      const int64_t u = full ? b0 + lane * PER + k : b0 + i;
      // update operands, independent of the sums
      const uint32_t e0 = act ? sld(a.rptr + (b0 + i)) : 0u;
      const uint32_t e1 = act ? sld(a.rptr + (b0 + i + 1)) : 0u;
      double iw = 0.0, pu = C.inv_n;
      if (act) {
        iw = sld(C.inv_w + (b0 + i));
        if (!(C.flags & kFlagUniformP)) pu = sld(C.p + u);
      }
      const uint32_t L = act ? e1 - e0 : 0u;
      const bool lng = L > (uint32_t)kIpShort;
      LaneSum<T> acc;
      if (!lng) {
        // rows of up to kIpShort edges: kBatch neighbour ids, then kBatch
        // values, in flight per lane
        for (uint32_t j0 = 0; j0 < L; j0 += kBatch) {
          int32_t sv[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) sv[j] = j0 + j < L ? sld(a.idx + (e0 + j0 + j)) : (int32_t)b0;
          T v[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j)
            v[j] = ip_value<T, WEIGHTED>(a, blk, c, b0, nb, sv[j], e0 + j0 + j, j0 + j < L);
#pragma unroll
          for (int j = 0; j < kBatch; ++j)
            if (j0 + j < L) acc.add(v[j]);
        }
      }
      double sum = acc.value();
      // the step's long rows, one at a time, by the whole wavefront (a lane's
      // edges are f0 + lane, + 64, ...; kBatch loads in flight)
      uint64_t lm = __ballot(lng);
      while (lm) {
        const int r = __builtin_ctzll(lm);
        lm &= lm - 1;
        const uint32_t f0 = __builtin_amdgcn_readlane(e0, r), f1 = __builtin_amdgcn_readlane(e1, r);
        LaneSum<T> part;
        for (uint32_t e = f0 + lane; e < f1; e += 64 * kBatch) {
          int32_t sv[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) sv[j] = e + 64 * j < f1 ? sld(a.idx + (e + 64 * j)) : (int32_t)b0;
          T v[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j)
            v[j] = ip_value<T, WEIGHTED>(a, blk, c, b0, nb, sv[j], e + 64 * j, e + 64 * j < f1);
#pragma unroll
          for (int j = 0; j < kBatch; ++j)
            if (e + 64 * j < f1) part.add(v[j]);
        }
        part.group_reduce(64);
        if (lane == r) sum = part.value();
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (act) {
        // no rank array: the slot of c holds x / W, or x itself for a
        // dangling vertex (never gathered), and the change is read off c
        // (the previous value is the block's LDS copy): |x' - x| =
        // |c' - c| / (1/W), exactly 0 once c stops changing
        const double xn = C.tele * pu + C.d * (sum + C.dterm);
        const T xs = (T)xn;
        const double xd = (double)xs;
        const double co = (double)blk[i];
        if (iw != 0.0) {
          const T cv = (T)(xd * iw);
          blk[i] = cv;
          c[b0 + i] = cv;
          red.chg += fabs((double)cv - co) / iw;
        } else {
          c[b0 + i] = xs;
          red.dang += xd;
          red.chg += fabs(xd - co);
        }
        red.tot += xd;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  const double chg = wave_sum(red.chg);
  const double dang = wave_sum(red.dang);
  const double tot = wave_sum(red.tot);
  if (lane == 0) {
    s_part[0][wave] = chg;
    s_part[1][wave] = dang;
    s_part[2][wave] = tot;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int r = threadIdx.x;
    double v = s_part[r][0];
    for (int k = 1; k < kSweepWaves; ++k) v += s_part[r][k];
    a.wave_part[(size_t)r * a.part_stride + a.part_base + blockIdx.x] = v;
  }
}

// Phase 1 of the edge-centric form (Algorithm 1): every out-edge v -> u gets
// v's contribution x_v / W_v (times the edge weight) in its contributionList
// position, the position of that edge in the sweep's edge layout.  The value
// is computed exactly as the pull computes the gathered one, so both forms
// sum the same numbers in the same order.
template <typename T>
struct ScatterArgs {
  const int32_t *src;  // [m] source of each out-edge
  const int32_t *pos;  // [m] its list position
  const double *w;     // [m] its weight (weighted graphs)
  const double *inv_w;
  const IoPtrs *io;  // x: the ranks of the previous sweep
  T *cl;
  int64_t m;
  const SweepState *st;
};
constexpr int kScatterGrid = 2048;

template <typename T, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_scatter(ScatterArgs<T> a) {
  if (a.st->done) return;
  const T *x = static_cast<const T *>(a.io->x);
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < a.m; e += (int64_t)gridDim.x * kBlock) {
    const int32_t v = sld(a.src + e);
    const double xd = (double)x[v];
    T c = (T)(xd * a.inv_w[v]);
    if constexpr (WEIGHTED) c = wmul(c, sld(a.w + e));
    a.cl[sld(a.pos + e)] = c;
  }
}

// The hubs split into chunk items: each adds its chunk sums in chunk order and
// is updated (one thread per hub, chunk loads batched; `first` is the record
// of the thread's first hub, loaded ahead).
template <typename T, bool FUSED>
__device__ __forceinline__ void finish_split_hubs(const Ctx<T> &C, const SweepArgs<T> &a, int4 first, Red &red) {
  for (int h = threadIdx.x; h < a.n_msplit; h += kFinBlock) {
    const int4 hs = h == (int)threadIdx.x ? first : a.msplit[h];
    const uint32_t u = C.rows[hs.x];
    const uint32_t slot = C.rowpos[hs.x];
    const double xo = (double)C.x[u];
    const double iw = C.inv_w[u];
    const double pu = (C.flags & kFlagUniformP) ? C.inv_n : C.p[u];
    double tot = 0.0;
    for (int k0 = 0; k0 < hs.z; k0 += 8) {
      double part[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) part[k] = k0 + k < hs.z ? a.hpart[hs.y + k0 + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) tot += part[k];
    }
    update_loaded<T, FUSED>(C, nullptr, u, slot, xo, iw, pu, tot, red);
  }
}

// Completes the sweep in one workgroup: updates the split hubs, sums the
// workgroup partials in a fixed order and publishes residual, dangling mass, total mass, iteration
// count and the stop flag.
template <typename T, bool FUSED>
__global__ __launch_bounds__(kFinBlock) void k_finalize(SweepArgs<T> a) {
  __shared__ double s_red[3][kFinBlock / 64];
  SweepState *st = a.st;
  const bool linf = (a.flags & kFlagLinf) != 0;
  const int n = a.n_part;
  const size_t ps = (size_t)a.part_stride;
  // the first batch of partials and the first split hub's record are loaded
  // together with the state: none depends on the others
  double c[8], dg[8], tt[8];
  auto load = [&](int i0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * kFinBlock;
      const bool ok = i < n;
      c[k] = ok ? a.wave_part[i] : 0.0;
      dg[k] = ok ? a.wave_part[ps + i] : 0.0;
      tt[k] = ok ? a.wave_part[2 * ps + i] : 0.0;
    }
  };
  load(threadIdx.x);
  const int4 hub0 = (int)threadIdx.x < a.n_msplit ? a.msplit[threadIdx.x] : make_int4(0, 0, 0, 0);
  if (st->done) return;
  const Ctx<T> C = make_ctx<T, FUSED>(a, st);
  const double S_old = st->S;
  Red red;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * kFinBlock) {
    if (i0 != (int)threadIdx.x) load(i0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      red.chg = linf ? fmax(red.chg, c[k]) : red.chg + c[k];
      red.dang += dg[k];
      red.tot += tt[k];
    }
  }
  finish_split_hubs<T, FUSED>(C, a, hub0, red);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double chg = linf ? wave_max(red.chg) : wave_sum(red.chg);
  double dang = wave_sum(red.dang);
  double tot = wave_sum(red.tot);
  if (lane == 0) {
    s_red[0][wave] = chg;
    s_red[1][wave] = dang;
    s_red[2][wave] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double raw = s_red[0][0], Dn = s_red[1][0], Sn = s_red[2][0];
    for (int k = 1; k < kFinBlock / 64; ++k) {
      raw = linf ? fmax(raw, s_red[0][k]) : raw + s_red[0][k];
      Dn += s_red[1][k];
      Sn += s_red[2][k];
    }
    double resid = raw;
    if (a.flags & kFlagScaled) resid = (raw + fabs(Sn - S_old)) / S_old;
    st->raw = raw;
    st->resid = resid;
    st->D = Dn;
    st->S = Sn;
    const int it = st->iter + 1;
    st->iter = it;
    if (a.trace) a.trace[it - 1] = resid;
    if (!(resid >= st->tol) || it >= st->max_iter) st->done = 1;
  }
}

// ------------------------------------------------------- init / finish --

template <typename T>
struct InitArgs {
  const uint32_t *gpos;
  const double *inv_w;
  const double *p;
  const double *x_in;  // warm start (FP64), or null: start from p
  T *x;
  T *c;
  double *part;  // [2][gridDim.x]
  int64_t n;
  double inv_n;
  int uniform_p;
  int raw;         // adjoint: gathered value = x for every vertex
  int x_at_slot;   // x stored by gpos too (the in-place form's interleaved layout)
  int dangling_x;  // in-place form: a dangling vertex's slot of c holds its rank
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(InitArgs<T> a) {
  __shared__ double s_red[2][kWaves];
  double dang = 0.0, tot = 0.0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < a.n;
       u += (int64_t)gridDim.x * kBlock) {
    double xv = a.x_in ? a.x_in[u] : (a.uniform_p ? a.inv_n : a.p[u]);
    T xs = (T)xv;
    const size_t slot = a.gpos ? (size_t)a.gpos[u] : (size_t)u;  // null: vertex order
    a.x[a.x_at_slot ? slot : (size_t)u] = xs;
    const double xd = (double)xs;
    const double iw = a.inv_w[u];
    if (a.raw) a.c[slot] = xs;
    else if (iw != 0.0) a.c[slot] = (T)(xd * iw);
    else if (a.dangling_x) a.c[slot] = xs;
    if (iw == 0.0) dang += xd;
    tot += xd;
  }
  dang = wave_sum(dang);
  tot = wave_sum(tot);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_red[0][wave] = dang;
    s_red[1][wave] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < kWaves; ++k) {
      a0 += s_red[0][k];
      a1 += s_red[1][k];
    }
    a.part[blockIdx.x] = a0;
    a.part[gridDim.x + blockIdx.x] = a1;
  }
}

__global__ __launch_bounds__(kFinBlock) void k_init_final(const double *part, int nparts,
                                                          SweepState *st, double tol, int max_iter) {
  __shared__ double s_red[2][kFinBlock / 64];
  double D = 0.0, S = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kFinBlock) {
    D += part[i];
    S += part[nparts + i];
  }
  D = wave_sum(D);
  S = wave_sum(S);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_red[0][wave] = D;
    s_red[1][wave] = S;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  D = 0.0;
  S = 0.0;
  for (int k = 0; k < kFinBlock / 64; ++k) {
    D += s_red[0][k];
    S += s_red[1][k];
  }
  st->iter = 0;
  st->done = 0;
  st->max_iter = max_iter;
  st->tol = tol;
  st->D = D;
  st->S = S;
  st->resid = INFINITY;
  st->raw = INFINITY;
}

// x64[u] = x[u] * scale (FP32 or FP64 source; scale = 1/S for mass-scaled
// iterates), x read at map[u] when a map is given.  With iw (the in-place FP64
// form, whose source is its contribution array): the rank is the contribution
// divided by 1/W, or the slot itself for a dangling vertex (iw = 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to64(const T *x, double *out, int64_t n,
                                                 const SweepState *st, int scaled,
                                                 const uint32_t *map = nullptr, const double *iw = nullptr) {
  const double scale = scaled ? 1.0 / st->S : 1.0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kBlock) {
    const size_t at = map ? (size_t)map[u] : (size_t)u;
    double v = (double)x[at];
    if (iw && iw[at] != 0.0) v /= iw[at];
    out[u] = v * scale;
  }
}

constexpr int kInitGrid = 1024;

// ------------------------------------------------------------ host side --

template <typename T>
T *contrib(pr_graph *g, int which);
template <>
double *contrib<double>(pr_graph *g, int which) {
  return g->c64[which];
}
template <>
float *contrib<float>(pr_graph *g, int which) {
  return g->c32[which];
}

template <typename T>
int ensure_contrib(pr_graph *g) {
  for (int k = 0; k < 2; ++k) {
    void **slot = std::is_same<T, double>::value ? (void **)&g->c64[k] : (void **)&g->c32[k];
    if (!*slot) {
      int rc = fpr_dev_alloc(g, slot, sizeof(T) * (size_t)g->n);
      if (rc) return rc;
    }
  }
  return PR_OK;
}

template <typename T>
T *cl_buf(pr_graph *g) {
  if constexpr (sizeof(T) == 8) return g->cl64;
  else return g->cl32;
}

// The contributionList of the edge-centric form, zeroed once (tile padding
// positions are never written and must read zero).
template <typename T>
int ensure_cl(pr_graph *g) {
  T **slot;
  if constexpr (sizeof(T) == 8) slot = &g->cl64;
  else slot = &g->cl32;
  if (*slot) return PR_OK;
  const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(1, g->fwd.cl_size);
  int rc = fpr_dev_alloc(g, (void **)slot, bytes);
  if (rc) return rc;
  PR_HIP(hipMemsetAsync(*slot, 0, bytes, g->work));
  return PR_OK;
}

int ensure_trace(pr_graph *g, int max_iter) {
  if (g->trace_cap >= max_iter) return PR_OK;
  int rc = fpr_dev_alloc(g, (void **)&g->trace_dev, sizeof(double) * (size_t)max_iter);
  if (rc) return rc;
  g->trace_cap = max_iter;
  return PR_OK;
}

// Initial ranks and contributions (in the plan's gather layout, or in vertex
// order for the in-place form).
template <typename T>
int launch_init(pr_graph *g, DevPlan &P, const double *p, const double *x_in, T *x, double tol,
                int max_iter, T *c0 = nullptr, int raw = 0, bool vertex_order = false) {
  InitArgs<T> a;
  a.gpos = vertex_order ? P.ip_pos : P.gpos;
  a.x_at_slot = vertex_order ? 1 : 0;
  a.dangling_x = vertex_order ? 1 : 0;
  a.inv_w = g->inv_w;
  a.p = p;
  a.x_in = x_in;
  a.x = x;
  a.c = c0 ? c0 : contrib<T>(g, 0);
  a.raw = raw;
  a.part = g->red_tmp;
  a.n = g->n;
  a.inv_n = 1.0 / (double)g->n;
  a.uniform_p = p == nullptr;
  const int grid = (int)std::min<int64_t>(kInitGrid, (g->n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_init<T>, dim3(grid), dim3(kBlock), 0, g->work, a);
  hipLaunchKernelGGL(k_init_final, dim3(1), dim3(kFinBlock), 0, g->work, (const double *)g->red_tmp,
                     grid, P.st, tol, max_iter);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

__global__ void k_set_io(IoPtrs *io, void *x, const double *p) {
  io->x = x;
  io->p = p;
}

// Points the plan's IoPtrs block at x and p (queued on the work stream, so it
// takes effect for the launches queued after it).  Skipped when the block
// already holds them.
int set_io(pr_graph *g, DevPlan &P, void *x, const double *p) {
  if (P.io_valid && P.io_last.x == x && P.io_last.p == p) return PR_OK;
  hipLaunchKernelGGL(k_set_io, dim3(1), dim3(1), 0, g->work, P.io, x, p);
  PR_HIP(hipGetLastError());
  P.io_last = IoPtrs{x, p};
  P.io_valid = true;
  return PR_OK;
}

// The launch arguments of the sweeps of plan P; x and p go through P's IoPtrs
// block (set_io), only whether p is given is part of the arguments.
template <typename T>
SweepArgs<T> make_args(pr_graph *g, DevPlan &P, const double *p, double d, int flags,
                       double *trace, T *c0 = nullptr, T *c1 = nullptr, int form = PR_JACOBI) {
  SweepArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.rows = P.rows;
  a.rowpos = P.rowpos;
  a.rptr = P.rptr;
  a.idx = P.idx;
  a.w = P.w;
  a.items = P.items;
  a.tiles = P.tiles;
  a.msplit = P.msplit;
  a.hpart = P.hpart;
  a.n_msplit = P.n_msplit;
  a.chunk = P.chunk;
  a.tidx = P.tidx;
  a.tw = P.tw;
  a.tmask = P.tmask;
  a.wave_part = P.wave_part;
  a.st = P.st;
  a.inv_w = g->inv_w;
  a.io = P.io;
  a.c0 = c0 ? c0 : contrib<T>(g, 0);
  a.c1 = c1 ? c1 : contrib<T>(g, 1);
  a.cl = cl_buf<T>(g);
  a.cl_rows = P.cl_rows;
  a.trace = trace;
  a.d = d;
  a.inv_n = 1.0 / (double)g->n;
  a.n_items = P.n_items;
  a.n_waves = P.n_waves;
  {
    int64_t hot = g->popts.hot_slots < 0 ? kHotSlots<T> : std::min<int64_t>(g->popts.hot_slots, kHotSlots<T>);
    a.hot = (int)std::min<int64_t>(hot, g->n);
  }
  a.flags = flags | (p ? 0 : kFlagUniformP);
  a.block_pos = P.block_pos;
  a.wave_cnt = P.wave_cnt;
  a.blk_lo = 0;
  a.blk_hi = P.n_blocks;
  a.part_base = 0;
  a.part_stride = P.part_stride;
  a.n_part = P.n_waves / kSweepWaves;
  a.fresh_lo = 0;
  a.fresh_hi = 0;
  a.nv = g->n;
  if (form == PR_INPLACE) {
    // vertex-order in-lists and one contribution array, updated in place
    a.rptr = P.ip_ptr;
    a.idx = P.ip_src;
    a.w = P.ip_w;
    a.inv_w = P.ip_iw;
    a.ip_range = P.ip_range;
    a.c1 = a.c0;
    a.n_msplit = 0;
    a.hot = 0;
  }
  return a;
}

// One sweep: the sweep kernel, then the finalize kernel.  The fused form with
// several Gauss-Seidel blocks launches the sweep kernel once per block, so
// each block reads what the blocks before it wrote in this sweep.  `mark`,
// when given, is recorded right before the finalize kernel.
template <typename T, bool FUSED, int MODE>
void launch_one(const DevPlan &P, const SweepArgs<T> &a0, hipStream_t s, hipEvent_t mark) {
  const dim3 grid(a0.n_waves / kSweepWaves), block(kSweepBlock);
  if (!FUSED || P.n_blocks <= 1) {
    hipLaunchKernelGGL((k_sweep<T, FUSED, MODE>), grid, block, 0, s, a0);
    if (mark) (void)hipEventRecord(mark, s);
    hipLaunchKernelGGL((k_finalize<T, FUSED>), dim3(1), dim3(kFinBlock), 0, s, a0);
    return;
  }
  const int B = P.n_blocks;
  SweepArgs<T> a = a0;
  a.fresh_lo = P.block_slots[0];
  for (int b = 0; b < B; ++b) {
    a.blk_lo = b;
    a.blk_hi = b + 1;
    a.part_base = b * (P.n_waves / kSweepWaves);
    a.fresh_hi = P.block_slots[b];
    hipLaunchKernelGGL((k_sweep<T, FUSED, MODE>), grid, block, 0, s, a);
  }
  if (mark) (void)hipEventRecord(mark, s);
  a.n_part = B * (P.n_waves / kSweepWaves);
  hipLaunchKernelGGL((k_finalize<T, FUSED>), dim3(1), dim3(kFinBlock), 0, s, a);
}

// Phase 1 of the list forms over scatter entries [lo, hi) (Algorithm 1's
// scatter, or Algorithm 2's fused scatter of one launch's vertices).
template <typename T>
void scatter_range(pr_graph *g, const SweepArgs<T> &a, bool weighted, int64_t lo, int64_t hi, hipStream_t s) {
  if (hi <= lo) return;
  const DevPlan &P = g->fwd;
  ScatterArgs<T> sa;
  sa.src = P.cl_src + lo;
  sa.pos = P.cl_pos + lo;
  sa.w = P.cl_w ? P.cl_w + lo : nullptr;
  sa.inv_w = g->inv_w;
  sa.io = a.io;
  sa.cl = const_cast<T *>(a.cl);
  sa.m = hi - lo;
  sa.st = a.st;
  const int grid = (int)std::min<int64_t>(kScatterGrid, (hi - lo + kBlock - 1) / kBlock);
  if (weighted) hipLaunchKernelGGL((k_scatter<T, true>), dim3(grid), dim3(kBlock), 0, s, sa);
  else hipLaunchKernelGGL((k_scatter<T, false>), dim3(grid), dim3(kBlock), 0, s, sa);
}

// The loop-fused list form (Algorithm 2 with the paper's contributionList):
// per Gauss-Seidel block, the launch that sums its rows' list slices and
// updates them, then the scatter of those vertices' new contributions into
// the list; the split hubs, updated by the finalize kernel, scatter after it.
// A block reads, through the list, this sweep's contributions of the blocks
// before it and the previous sweep's of the others: the values the block
// Gauss-Seidel pull gathers, summed in the same order.
template <typename T>
void launch_fused_list(pr_graph *g, const SweepArgs<T> &a0, bool weighted, hipStream_t s, hipEvent_t mark) {
  const DevPlan &P = g->fwd;
  const int B = P.n_blocks, G = a0.n_waves / kSweepWaves;
  SweepArgs<T> a = a0;
  for (int b = 0; b < B; ++b) {
    a.blk_lo = b;
    a.blk_hi = b + 1;
    a.part_base = b * G;
    hipLaunchKernelGGL((k_sweep<T, false, kModeList>), dim3(G), dim3(kSweepBlock), 0, s, a);
    scatter_range<T>(g, a, weighted, P.cl_group[b], P.cl_group[b + 1], s);
  }
  if (mark) (void)hipEventRecord(mark, s);
  a.n_part = B * G;
  hipLaunchKernelGGL((k_finalize<T, false>), dim3(1), dim3(kFinBlock), 0, s, a);
  scatter_range<T>(g, a, weighted, P.cl_group[B], P.cl_group[B + 1], s);
}

template <typename T>
void launch_marked(pr_graph *g, const SweepArgs<T> &a, int form, bool weighted, hipStream_t s,
                   hipEvent_t mark) {
  const DevPlan &P = g->fwd;  // the fused and list forms run on the forward plan only
  if (form == PR_EDGE_LIST) {
    // Algorithm 1 as the paper lays it out: scatter the contributions into the
    // edge-ordered list, then sum each row's contiguous slice
    ScatterArgs<T> sa;
    sa.src = P.cl_src;
    sa.pos = P.cl_pos;
    sa.w = P.cl_w;
    sa.inv_w = g->inv_w;
    sa.io = a.io;
    sa.cl = const_cast<T *>(a.cl);
    sa.m = P.m;
    sa.st = a.st;
    if (weighted) hipLaunchKernelGGL((k_scatter<T, true>), dim3(kScatterGrid), dim3(kBlock), 0, s, sa);
    else hipLaunchKernelGGL((k_scatter<T, false>), dim3(kScatterGrid), dim3(kBlock), 0, s, sa);
    launch_one<T, false, kModeList>(P, a, s, mark);
  } else if (form == PR_FUSED_EDGE_LIST) {
    launch_fused_list<T>(g, a, weighted, s, mark);
  } else if (form == PR_INPLACE) {
    const dim3 grid(a.n_waves / kSweepWaves), block(kSweepBlock);
    if (weighted) hipLaunchKernelGGL((k_inplace<T, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_inplace<T, false>), grid, block, 0, s, a);
    if (mark) (void)hipEventRecord(mark, s);
    hipLaunchKernelGGL((k_finalize<T, true>), dim3(1), dim3(kFinBlock), 0, s, a);
  } else if (form == PR_FUSED) {
    if (weighted) launch_one<T, true, kModeWeighted>(P, a, s, mark);
    else launch_one<T, true, kModePlain>(P, a, s, mark);
  } else {
    if (weighted) launch_one<T, false, kModeWeighted>(P, a, s, mark);
    else launch_one<T, false, kModePlain>(P, a, s, mark);
  }
}

template <typename T>
void launch_sweeps(pr_graph *g, const SweepArgs<T> &a, int form, bool weighted, int count,
                   hipStream_t s) {
  for (int k = 0; k < count; ++k) launch_marked<T>(g, a, form, weighted, s, nullptr);
}

// The queued sweeps run from a hipGraph cached per graph, keyed by the bytes
// of their launch arguments (which hold no caller pointer: x and p go through
// the plan's IoPtrs block), the form and the sweep count.
template <typename T>
int run_sweeps(pr_graph *g, const SweepArgs<T> &a, int form, bool use_graph, int count) {
  if (!use_graph) {
    launch_sweeps(g, a, form, g->weighted, count, g->work);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  std::vector<unsigned char> key(sizeof(a) + 3 * sizeof(int));
  memcpy(key.data(), &a, sizeof(a));
  int extra[3] = {form, count, (int)sizeof(T)};
  memcpy(key.data() + sizeof(a), extra, sizeof(extra));
  for (auto &e : g->graph_cache) {
    if (e.key == key) {
      PR_HIP(hipGraphLaunch(e.exec, g->work));
      return PR_OK;
    }
  }
  if (g->graph_cache.size() >= 32) {
    for (auto &e : g->graph_cache) (void)hipGraphExecDestroy(e.exec);
    g->graph_cache.clear();
  }
  hipGraph_t graph;
  PR_HIP(hipStreamBeginCapture(g->work, hipStreamCaptureModeThreadLocal));
  launch_sweeps(g, a, form, g->weighted, count, g->work);
  hipError_t le = hipGetLastError();
  hipError_t ce = hipStreamEndCapture(g->work, &graph);
  if (le != hipSuccess) return pr_fail(PR_EDEVICE, "sweep launch during capture: %s", hipGetErrorString(le));
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

int poll_state(pr_graph *g, DevPlan &P) {
  PR_HIP(hipMemcpyAsync(g->host_st, P.st, sizeof(SweepState), hipMemcpyDeviceToHost, g->work));
  PR_HIP(hipStreamSynchronize(g->work));
  return PR_OK;
}

bool is_list_form(int form) { return form == PR_EDGE_LIST || form == PR_FUSED_EDGE_LIST; }

// The loop-fused list form keeps its list up to date sweep by sweep: it is
// filled once from the start vector (Algorithm 2 primes it before its loop).
template <typename T>
void prime_list(pr_graph *g, const SweepArgs<T> &a, int form) {
  if (form == PR_FUSED_EDGE_LIST) scatter_range<T>(g, a, g->weighted, 0, g->fwd.m, g->work);
}

// The device buffers of a solve: the contribution arrays of each precision
// (previous and current sweep) and the FP32 copy of the ranks.  Null members
// mean the graph's own buffers, allocated on first use.
struct SolveBufs {
  double *c64[2] = {nullptr, nullptr};
  float *c32[2] = {nullptr, nullptr};
  float *x32 = nullptr;
};

template <typename T>
void bufs_of(const SolveBufs &b, T *&c0, T *&c1);

// The in-place form updates one contribution array and keeps no rank array
// (the kernel reads a rank back from its contribution); the precision's
// second contribution buffer (the caller's, or the library's once
// allocated) only receives the start vector, in the plan's interleaved
// order.
template <typename T>
int inplace_x(pr_graph *g, const SolveBufs &b, T *&xs) {
  T *c0 = nullptr, *c1 = nullptr;
  bufs_of<T>(b, c0, c1);
  if (!c0) {
    int rc = ensure_contrib<T>(g);
    if (rc) return rc;
    c1 = contrib<T>(g, 1);
  }
  xs = c1;
  return PR_OK;
}

// Where the in-place form's final ranks are read from: its contribution
// array (the caller's, or the library's), divided back by 1/W.
template <typename T>
const T *inplace_c(pr_graph *g, const SolveBufs &b) {
  T *c0 = nullptr, *c1 = nullptr;
  bufs_of<T>(b, c0, c1);
  return c0 ? c0 : contrib<T>(g, 0);
}

template <typename T>
void bufs_of(const SolveBufs &b, T *&c0, T *&c1) {
  if constexpr (sizeof(T) == 8) {
    c0 = b.c64[0];
    c1 = b.c64[1];
  } else {
    c0 = b.c32[0];
    c1 = b.c32[1];
  }
}

// One stage: init from (p | x_in) then sweeps until the state says done.
// stall: stop polling once the residual fails to halve between polls (FP32 floor).
template <typename T>
int solve_stage(pr_graph *g, double d, double tol, int max_iter, const pr_opts &o, const double *p,
                const double *x_in, T *x, int flags, int form, double *trace, bool stall,
                int *iters, double *resid, const SolveBufs &bufs) {
  int rc;
  T *c0 = nullptr, *c1 = nullptr;
  bufs_of<T>(bufs, c0, c1);
  if (!c0 && (rc = ensure_contrib<T>(g))) return rc;
  if (is_list_form(form) && (rc = ensure_cl<T>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<T>(g, P, p, x_in, x, tol, max_iter, c0, 0, form == PR_INPLACE))) return rc;
  if ((rc = set_io(g, P, x, p))) return rc;
  SweepArgs<T> a = make_args<T>(g, P, p, d, flags, trace, c0, c1, form);
  prime_list<T>(g, a, form);
  // Sweeps are queued in batches between host polls: G, then G/2, then as
  // many as the residual's decay over the last batch predicts are still
  // needed (at most G), so that few sweeps queue past convergence.  A batch
  // runs as hipGraphs of power-of-two sweep counts, so at most four graphs
  // per form are captured.  The FP32 stage keeps batches of G: it stops when
  // the residual fails to halve between polls (its floor).
  const int G = std::max(1, o.sweeps_per_poll);
  double prev = INFINITY;
  int done_sweeps = 0;
  int cnt = std::min(G, max_iter);
  for (;;) {
    for (int left = cnt; left > 0;) {
      int piece = 1;
      while (piece * 2 <= left) piece *= 2;
      if ((rc = run_sweeps<T>(g, a, form, o.use_hip_graph != 0, piece))) return rc;
      left -= piece;
    }
    if ((rc = poll_state(g, P))) return rc;
    const int before = done_sweeps;
    done_sweeps = g->host_st->iter;
    if (g->host_st->done || done_sweeps >= max_iter) break;
    if (done_sweeps != before + cnt)
      return pr_fail(PR_EDEVICE, "internal: %d sweeps completed after %d + %d launched", done_sweeps, before, cnt);
    const double r = g->host_st->resid;
    if (!(r == r)) return pr_fail(PR_EDEVICE, "residual is NaN after sweep %d", done_sweeps);
    if (stall && r >= 0.5 * prev) break;
    int next = G;
    if (!stall && prev == INFINITY) {
      next = std::max(1, G / 2);
    } else if (!stall && r > 0.0 && r < prev && tol > 0.0) {
      const double rate = std::pow(r / prev, 1.0 / cnt);
      const double need = std::log(tol / r) / std::log(rate);
      if (need == need) next = (int)std::min<double>(G, std::max(1.0, std::ceil(need + 0.25)));
    }
    prev = r;
    cnt = std::min(next, max_iter - done_sweeps);
  }
  *iters = g->host_st->iter;
  *resid = g->host_st->resid;
  return PR_OK;
}

int validate_common(pr_graph *g, double d, const pr_opts &o) {
  if (!g) return pr_fail(PR_EINVAL, "graph is NULL");
  if (!(d > 0.0 && d < 1.0)) return pr_fail(PR_EINVAL, "d=%g is not in (0, 1)", d);
  if (o.mode != PR_JACOBI && o.mode != PR_FUSED && o.mode != PR_EDGE_LIST && o.mode != PR_INPLACE &&
      o.mode != PR_FUSED_EDGE_LIST)
    return pr_fail(PR_EINVAL, "bad mode %d", o.mode);
  if (o.mode == PR_INPLACE && !g->fwd.ip_ptr)
    return pr_fail(PR_EINVAL, "the in-place form needs a graph planned with with_inplace = 1");
  if ((o.mode == PR_EDGE_LIST || o.mode == PR_FUSED_EDGE_LIST) && !g->fwd.cl_pos)
    return pr_fail(PR_EINVAL, "the edge-list forms need a graph planned with with_cl = 1");
  if (o.precision != PR_FP64 && o.precision != PR_FP32)
    return pr_fail(PR_EINVAL, "bad precision %d", o.precision);
  if (o.dangling != PR_DANGLING_UNIFORM && o.dangling != PR_DANGLING_LEAK)
    return pr_fail(PR_EINVAL, "bad dangling mode %d", o.dangling);
  if (o.norm != PR_NORM_L1 && o.norm != PR_NORM_LINF) return pr_fail(PR_EINVAL, "bad norm %d", o.norm);
  const bool gs = o.mode == PR_FUSED || o.mode == PR_INPLACE || o.mode == PR_FUSED_EDGE_LIST;
  if (gs && o.fused_scaled && (o.dangling != PR_DANGLING_UNIFORM || o.norm != PR_NORM_L1))
    return pr_fail(PR_EINVAL, "the mass-scaled fused form needs uniform dangling and the L1 norm");
  if (gs && o.norm == PR_NORM_LINF)
    return pr_fail(PR_EINVAL, "the max-norm residual is supported by the Jacobi form only");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  return PR_OK;
}

int flags_of(const pr_opts &o) {
  int f = 0;
  if (o.dangling == PR_DANGLING_LEAK) f |= kFlagLeak;
  if (o.norm == PR_NORM_LINF) f |= kFlagLinf;
  if ((o.mode == PR_FUSED || o.mode == PR_INPLACE || o.mode == PR_FUSED_EDGE_LIST) && o.fused_scaled)
    f |= kFlagScaled;
  if (o.mode == PR_EDGE_LIST || o.mode == PR_FUSED_EDGE_LIST) f |= kFlagList;
  return f;
}

struct StreamJoin {
  pr_graph *g;
  hipStream_t user;
  StreamJoin(pr_graph *g_, void *s) : g(g_), user((hipStream_t)s) {
    (void)hipEventRecord(g->ev_in, user);
    (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  }
  ~StreamJoin() {
    (void)hipEventRecord(g->ev_out, g->work);
    (void)hipStreamWaitEvent(user, g->ev_out, 0);
  }
};

}  // namespace

// ------------------------------------------------------------------ ABI --

void fpr_sweep_release(pr_graph *g) {
  for (auto &e : g->graph_cache) (void)hipGraphExecDestroy(e.exec);
  g->graph_cache.clear();
}

int fpr_grid_for(pr_graph *g) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep<double, false, kModePlain>, kSweepBlock, 0) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  return std::max(1, g->n_cu) * nb;  // workgroups resident at once
}

extern "C" void pr_opts_default(pr_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->mode = PR_JACOBI;
  o->precision = PR_FP64;
  o->dangling = PR_DANGLING_UNIFORM;
  o->norm = PR_NORM_L1;
  o->warm_start = 0;
  o->fused_scaled = 1;
  o->sweeps_per_poll = 8;
  o->use_hip_graph = 1;
  o->refine_tol = -1.0;  // negative: use the solve's tol
  o->fp32_tol = 0.0;     // 0: max(tol, 1e-7)
  o->trace = nullptr;
}

namespace {

int validate_solve(pr_graph *g, double d, double tol, int max_iter, const pr_opts &o, const double *x,
                   const int *iters, const double *resid) {
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!(tol > 0.0)) return pr_fail(PR_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return pr_fail(PR_EINVAL, "max_iter=%d must be >= 1", max_iter);
  if (!x) return pr_fail(PR_EINVAL, "x is NULL");
  if (!iters || !resid) return pr_fail(PR_EINVAL, "iters/resid are NULL");
  return PR_OK;
}

// The body of pr_solve; `bufs` names the device buffers to work in (members
// left null are the graph's own).
int solve_impl(pr_graph *g, double d, double tol, int max_iter, const pr_opts &o, const double *p, double *x,
               int *iters, double *resid, void *stream, const SolveBufs &bufs) {
  int rc;
  StreamJoin join(g, stream);
  double *trace = nullptr;
  if (o.trace) {
    if ((rc = ensure_trace(g, max_iter))) return rc;
    trace = g->trace_dev;
  }
  const int flags = flags_of(o);
  const int form = o.mode;
  const bool scaled = (flags & kFlagScaled) != 0;
  int it = 0;
  double r = INFINITY;
  double target = tol;
  const bool ip = form == PR_INPLACE;
  const uint32_t *map = ip ? g->fwd.ip_pos : nullptr;  // the in-place form's ranks are interleaved
  if (o.precision == PR_FP64) {
    double *xs = x;
    if (ip && (rc = inplace_x<double>(g, bufs, xs))) return rc;
    if ((rc = solve_stage<double>(g, d, tol, max_iter, o, p, o.warm_start ? x : nullptr, xs, flags,
                                  form, trace, false, &it, &r, bufs)))
      return rc;
    if (scaled || ip) {
      hipLaunchKernelGGL(k_to64<double>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                         ip ? inplace_c<double>(g, bufs) : (const double *)xs, x, g->n, (const SweepState *)g->fwd.st,
                         scaled ? 1 : 0, map, ip ? (const double *)g->fwd.ip_iw : nullptr);
    }
  } else {
    float *x32 = bufs.x32;
    if (ip) {
      if ((rc = inplace_x<float>(g, bufs, x32))) return rc;
    } else if (!x32) {
      if (!g->x32 && (rc = fpr_dev_alloc(g, (void **)&g->x32, sizeof(float) * (size_t)g->n))) return rc;
      x32 = g->x32;
    }
    const double tol32 = o.fp32_tol > 0.0 ? o.fp32_tol : std::max(tol, 1e-7);
    const double rtol = o.refine_tol < 0.0 ? tol : o.refine_tol;
    if ((rc = solve_stage<float>(g, d, tol32, max_iter, o, p, o.warm_start ? x : nullptr, x32,
                                 flags, form, trace, rtol > 0.0, &it, &r, bufs)))
      return rc;
    target = rtol > 0.0 ? rtol : tol32;
    hipLaunchKernelGGL(k_to64<float>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                       ip ? inplace_c<float>(g, bufs) : (const float *)x32, x, g->n, (const SweepState *)g->fwd.st,
                       scaled ? 1 : 0, map, ip ? (const double *)g->fwd.ip_iw : nullptr);
    if (rtol > 0.0 && it < max_iter) {
      int it2 = 0;
      double r2 = INFINITY;
      double *xs = x;
      if (ip && (rc = inplace_x<double>(g, bufs, xs))) return rc;
      if ((rc = solve_stage<double>(g, d, rtol, max_iter - it, o, p, x, xs, flags, form,
                                    trace ? trace + it : nullptr, false, &it2, &r2, bufs)))
        return rc;
      if (scaled || ip)
        hipLaunchKernelGGL(k_to64<double>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                           ip ? inplace_c<double>(g, bufs) : (const double *)xs, x, g->n,
                           (const SweepState *)g->fwd.st, scaled ? 1 : 0, map,
                           ip ? (const double *)g->fwd.ip_iw : nullptr);
      it += it2;
      r = r2;
    }
  }
  PR_HIP(hipGetLastError());
  if (o.trace && it > 0)
    PR_HIP(hipMemcpyAsync(o.trace, trace, sizeof(double) * (size_t)std::min(it, max_iter),
                          hipMemcpyDeviceToHost, g->work));
  PR_HIP(hipStreamSynchronize(g->work));
  *iters = it;
  *resid = r;
  return (r < target) ? PR_OK : PR_NOT_CONVERGED;
}

}  // namespace

extern "C" int pr_solve(pr_graph *g, double d, double tol, int max_iter, const pr_opts *opts,
                        const double *p, double *x, int *iters, double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_solve(g, d, tol, max_iter, o, x, iters, resid);
  if (rc) return rc;
  return solve_impl(g, d, tol, max_iter, o, p, x, iters, resid, stream, SolveBufs());
}

// ------------------------------------------------------- caller workspace --

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The workspace a solve with options o takes: two contribution arrays of each
// precision it sweeps in (FP64 also for the refinement of an FP32 solve) and
// the FP32 copy of the ranks, each rounded up to 256 bytes.  With `base`, the
// buffers are carved from it in that order.
size_t ws_layout(const pr_graph *g, const pr_opts &o, double tol, unsigned char *base, SolveBufs *b) {
  const size_t n = (size_t)g->n;
  const double rtol = o.refine_tol < 0.0 ? tol : o.refine_tol;
  const bool fp64 = o.precision == PR_FP64 || rtol > 0.0;
  const bool fp32 = o.precision == PR_FP32;
  const size_t b64 = align256(sizeof(double) * n), b32 = align256(sizeof(float) * n);
  size_t off = 0;
  if (fp64) {
    if (base) {
      b->c64[0] = reinterpret_cast<double *>(base + off);
      b->c64[1] = reinterpret_cast<double *>(base + off + b64);
    }
    off += 2 * b64;
  }
  if (fp32) {
    if (base) {
      b->c32[0] = reinterpret_cast<float *>(base + off);
      b->c32[1] = reinterpret_cast<float *>(base + off + b32);
      b->x32 = reinterpret_cast<float *>(base + off + 2 * b32);
    }
    off += 3 * b32;
  }
  return off;
}

// What a solve in a caller's (or the static) workspace cannot take: the
// forms and options whose buffers it would have to allocate or clear.
int ws_refuse(const char *who, const pr_opts &o) {
  if (is_list_form(o.mode))
    return pr_fail(PR_EINVAL, "%s: the edge-list forms need their contributionList (m values)", who);
  if (o.trace) return pr_fail(PR_EINVAL, "%s: a residual trace needs a device buffer", who);
  return PR_OK;
}

}  // namespace

extern "C" int pr_workspace_bytes(const pr_graph *g, double tol, const pr_opts *opts, size_t *bytes) {
  pr_clear_error();
  if (!g || !bytes) return pr_fail(PR_EINVAL, "pr_workspace_bytes: NULL argument");
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = ws_refuse("pr_workspace_bytes", o);
  if (rc) return rc;
  *bytes = ws_layout(g, o, tol, nullptr, nullptr);
  return PR_OK;
}

extern "C" int pr_solve_ws(pr_graph *g, double d, double tol, int max_iter, const pr_opts *opts, const double *p,
                           double *x, void *ws, size_t ws_bytes, int *iters, double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_solve(g, d, tol, max_iter, o, x, iters, resid);
  if (rc) return rc;
  if ((rc = ws_refuse("pr_solve_ws", o))) return rc;
  if (!ws || ((uintptr_t)ws & 255) != 0)
    return pr_fail(PR_EINVAL, "pr_solve_ws: ws must be a 256-byte aligned device pointer");
  const size_t need = ws_layout(g, o, tol, nullptr, nullptr);
  if (ws_bytes < need)
    return pr_fail(PR_EINVAL, "pr_solve_ws: the workspace holds %zu bytes, the solve needs %zu", ws_bytes, need);
  SolveBufs b;
  ws_layout(g, o, tol, static_cast<unsigned char *>(ws), &b);
  return solve_impl(g, d, tol, max_iter, o, p, x, iters, resid, stream, b);
}

// ----------------------------------------------------- no-allocation solve --
//
// pr_solve_noalloc works in a fixed device array instead of buffers it would
// otherwise allocate on first use: one array per device, in the library's
// image, whose address each device gets once (hipGetSymbolAddress, with that
// device current) and keeps.  Host code uses only that address: the array's
// name is a host-side stand-in.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kScratchDevices] = {};

// The address of `scratch` on device `dev` (the current device), looked up on
// the first call for that device.
int scratch_on(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kScratchDevices)
    return pr_fail(PR_EINVAL, "pr_solve_noalloc: device %d outside the %d the scratch table holds", dev,
                   kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return pr_fail(PR_EDEVICE, "pr_solve_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PR_OK;
}

}  // namespace

extern "C" size_t pr_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int pr_solve_noalloc(pr_graph *g, double d, double tol, int max_iter, const pr_opts *opts,
                                const double *p, double *x, int *iters, double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_solve(g, d, tol, max_iter, o, x, iters, resid);
  if (rc) return rc;
  if ((rc = ws_refuse("pr_solve_noalloc", o))) return rc;
  o.use_hip_graph = 0;  // instantiating a hipGraph may allocate
  const size_t need = ws_layout(g, o, tol, nullptr, nullptr);
  if (need > kScratchBytes)
    return pr_fail(PR_EINVAL, "pr_solve_noalloc: n = %lld needs %zu bytes of scratch, more than the %zu it holds",
                   (long long)g->n, need, kScratchBytes);
  unsigned char *base = nullptr;
  if ((rc = scratch_on(g->device, &base))) return rc;
  SolveBufs b;
  ws_layout(g, o, tol, base, &b);
  return solve_impl(g, d, tol, max_iter, o, p, x, iters, resid, stream, b);
}

namespace {

// `sweeps` sweeps of precision T from the FP64 vector x (read, cast, written back).
template <typename T>
int iterate_impl(pr_graph *g, double d, const pr_opts &o, const double *p, double *x, int sweeps,
                 double *resid, double *elapsed_ms) {
  int rc;
  T *xs = nullptr;
  const bool vo = o.mode == PR_INPLACE;
  if ((rc = ensure_contrib<T>(g))) return rc;
  if (vo) {
    xs = contrib<T>(g, 1);  // the in-place form's interleaved ranks
  } else if constexpr (sizeof(T) == 8) {
    xs = x;
  } else {
    if (!g->x32 && (rc = fpr_dev_alloc(g, (void **)&g->x32, sizeof(float) * (size_t)g->n))) return rc;
    xs = g->x32;
  }
  if (is_list_form(o.mode) && (rc = ensure_cl<T>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<T>(g, P, p, x, xs, -1.0, std::max(1, sweeps), nullptr, 0, vo))) return rc;
  const int flags = flags_of(o);
  if ((rc = set_io(g, P, xs, p))) return rc;
  SweepArgs<T> a = make_args<T>(g, P, p, d, flags, nullptr, nullptr, nullptr, o.mode);
  prime_list<T>(g, a, o.mode);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (elapsed_ms) {
    PR_HIP(hipEventCreate(&e0));
    PR_HIP(hipEventCreate(&e1));
    PR_HIP(hipEventRecord(e0, g->work));
  }
  if (sweeps > 0 && (rc = run_sweeps<T>(g, a, o.mode, o.use_hip_graph != 0, sweeps))) return rc;
  if (elapsed_ms) PR_HIP(hipEventRecord(e1, g->work));
  if (sizeof(T) != 8 || (flags & kFlagScaled) || vo) {
    // the in-place form reads its ranks back from its contributions
    const bool from_c = vo;
    hipLaunchKernelGGL(k_to64<T>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                       from_c ? (const T *)contrib<T>(g, 0) : (const T *)xs, x, g->n, (const SweepState *)P.st,
                       (flags & kFlagScaled) ? 1 : 0, vo ? P.ip_pos : nullptr,
                       from_c ? (const double *)P.ip_iw : nullptr);
  }
  PR_HIP(hipGetLastError());
  if ((rc = poll_state(g, P))) return rc;
  if (resid) *resid = sweeps > 0 ? g->host_st->resid : INFINITY;
  if (elapsed_ms) {
    float ms = 0.0f;
    PR_HIP(hipEventElapsedTime(&ms, e0, e1));
    *elapsed_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return PR_OK;
}

}  // namespace

extern "C" int pr_iterate(pr_graph *g, double d, const pr_opts *opts, const double *p, double *x,
                          int sweeps, double *resid, double *elapsed_ms, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!x) return pr_fail(PR_EINVAL, "x is NULL");
  if (sweeps < 0) return pr_fail(PR_EINVAL, "sweeps=%d must be >= 0", sweeps);
  StreamJoin join(g, stream);
  if (o.precision == PR_FP32) return iterate_impl<float>(g, d, o, p, x, sweeps, resid, elapsed_ms);
  return iterate_impl<double>(g, d, o, p, x, sweeps, resid, elapsed_ms);
}

namespace {

template <typename T>
int profile_impl(pr_graph *g, double d, const pr_opts &o, double *x, int sweeps, double *sweep_ms,
                 double *finalize_ms) {
  int rc;
  T *xs = nullptr;
  const bool vo = o.mode == PR_INPLACE;
  if ((rc = ensure_contrib<T>(g))) return rc;
  if (vo) {
    xs = contrib<T>(g, 1);  // the in-place form's interleaved ranks
  } else if constexpr (sizeof(T) == 8) {
    xs = x;
  } else {
    if (!g->x32 && (rc = fpr_dev_alloc(g, (void **)&g->x32, sizeof(float) * (size_t)g->n))) return rc;
    xs = g->x32;
  }
  if (is_list_form(o.mode) && (rc = ensure_cl<T>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<T>(g, P, nullptr, x, xs, -1.0, sweeps, nullptr, 0, vo))) return rc;
  if ((rc = set_io(g, P, xs, nullptr))) return rc;
  SweepArgs<T> a = make_args<T>(g, P, nullptr, d, flags_of(o), nullptr, nullptr, nullptr, o.mode);
  prime_list<T>(g, a, o.mode);
  std::vector<hipEvent_t> ev(3 * (size_t)sweeps, nullptr);
  for (auto &e : ev) PR_HIP(hipEventCreate(&e));
  for (int k = 0; k < sweeps; ++k) {
    PR_HIP(hipEventRecord(ev[3 * k], g->work));
    launch_marked<T>(g, a, o.mode, g->weighted, g->work, ev[3 * k + 1]);
    PR_HIP(hipEventRecord(ev[3 * k + 2], g->work));
  }
  PR_HIP(hipGetLastError());
  if (sizeof(T) != 8 || (a.flags & kFlagScaled) || vo) {
    const bool from_c = vo;
    hipLaunchKernelGGL(k_to64<T>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                       from_c ? (const T *)contrib<T>(g, 0) : (const T *)xs, x, g->n, (const SweepState *)P.st,
                       (a.flags & kFlagScaled) ? 1 : 0, vo ? P.ip_pos : nullptr,
                       from_c ? (const double *)P.ip_iw : nullptr);
  }
  PR_HIP(hipStreamSynchronize(g->work));
  double ts = 0.0, tf = 0.0;
  for (int k = 0; k < sweeps; ++k) {
    float a0 = 0.0f, a1 = 0.0f;
    PR_HIP(hipEventElapsedTime(&a0, ev[3 * k], ev[3 * k + 1]));
    PR_HIP(hipEventElapsedTime(&a1, ev[3 * k + 1], ev[3 * k + 2]));
    ts += a0;
    tf += a1;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  *sweep_ms = ts / sweeps;
  *finalize_ms = tf / sweeps;
  return PR_OK;
}

}  // namespace

extern "C" int pr_profile_sweeps(pr_graph *g, double d, const pr_opts *opts, double *x, int sweeps,
                                 double *sweep_ms, double *finalize_ms, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!x || !sweep_ms || !finalize_ms) return pr_fail(PR_EINVAL, "x/sweep_ms/finalize_ms are NULL");
  if (sweeps < 1 || sweeps > 4096) return pr_fail(PR_EINVAL, "sweeps=%d outside [1, 4096]", sweeps);
  StreamJoin join(g, stream);
  if (o.precision == PR_FP32) return profile_impl<float>(g, d, o, x, sweeps, sweep_ms, finalize_ms);
  return profile_impl<double>(g, d, o, x, sweeps, sweep_ms, finalize_ms);
}

extern "C" int pr_certificate(pr_graph *g, double d, const double *p, const double *x,
                              double *result, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!x || !result) return pr_fail(PR_EINVAL, "x/result are NULL");
  StreamJoin join(g, stream);
  if (!g->xtmp && (rc = fpr_dev_alloc(g, (void **)&g->xtmp, sizeof(double) * (size_t)g->n))) return rc;
  if ((rc = ensure_contrib<double>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<double>(g, P, p, x, g->xtmp, -1.0, 1))) return rc;
  if ((rc = set_io(g, P, g->xtmp, p))) return rc;
  SweepArgs<double> a = make_args<double>(g, P, p, d, 0, nullptr);
  launch_sweeps(g, a, false, g->weighted, 1, g->work);
  PR_HIP(hipGetLastError());
  if ((rc = poll_state(g, P))) return rc;
  *result = g->host_st->raw;
  return PR_OK;
}

extern "C" int pr_adjoint(pr_graph *g, double d, const double *x, const double *dLdx, double tol,
                          int max_iter, double *lam, double *dLdp, double *dLdw, int *iters,
                          double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!g->has_adj) return pr_fail(PR_EINVAL, "pr_adjoint: the graph was created without with_adjoint");
  if (!x || !dLdx || !lam || !iters || !resid) return pr_fail(PR_EINVAL, "pr_adjoint: NULL argument");
  if (!(tol > 0.0)) return pr_fail(PR_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return pr_fail(PR_EINVAL, "max_iter=%d must be >= 1", max_iter);
  StreamJoin join(g, stream);
  for (int k = 0; k < 2; ++k)
    if (!g->ca64[k] && (rc = fpr_dev_alloc(g, (void **)&g->ca64[k], sizeof(double) * (size_t)g->n))) return rc;
  DevPlan &P = g->adj;
  // lam^0 = g; gathered value = lam (no 1/W scaling), all vertices
  if ((rc = launch_init<double>(g, P, dLdx, dLdx, lam, tol, max_iter, g->ca64[0], 1))) return rc;
  const int flags = kFlagAdjoint | kFlagLinf;
  if ((rc = set_io(g, P, lam, dLdx))) return rc;
  SweepArgs<double> a = make_args<double>(g, P, dLdx, d, flags, nullptr, g->ca64[0], g->ca64[1]);
  const int G = 8;
  int done_sweeps = 0;
  for (;;) {
    const int cnt = std::min(G, max_iter - done_sweeps);
    launch_sweeps(g, a, false, g->weighted, cnt, g->work);
    PR_HIP(hipGetLastError());
    if ((rc = poll_state(g, P))) return rc;
    const int before = done_sweeps;
    done_sweeps = g->host_st->iter;
    if (g->host_st->done || done_sweeps >= max_iter) break;
    if (done_sweeps != before + cnt)
      return pr_fail(PR_EDEVICE, "internal: %d sweeps completed after %d + %d launched", done_sweeps, before, cnt);
    if (!(g->host_st->resid == g->host_st->resid)) return pr_fail(PR_EDEVICE, "adjoint residual is NaN");
  }
  if ((rc = fpr_adjoint_gradients(g, d, x, lam, dLdp, dLdw, g->work))) return rc;
  PR_HIP(hipStreamSynchronize(g->work));
  *iters = g->host_st->iter;
  *resid = g->host_st->resid;
  return (*resid < tol) ? PR_OK : PR_NOT_CONVERGED;
}
