// Batched personalized PageRank: k teleport vectors, one-hot on seeds[j],
//     X[:, j] = (1-d) e_{seed_j} + d (P X[:, j])      (Eq. 1 with a personalised teleport),
// solved as one multi-column Jacobi pull per sweep.
//
// Columns are grouped four to a "pass" (a float4 per vertex), so one random
// 16-byte gather serves four columns; a launch runs `tile`/4 passes side by
// side (grid.y = pass), which is the autotuned tile width.  The work items are
// the forward plan's (row tiles with a segmented scan across lanes, one
// wavefront per long row, chunked hubs completed by the finalize kernel, rows
// without in-edges), applied to four columns at once.
//
// Each workgroup copies the first `hot` gather slots (the most gathered
// vertices) of its pass into LDS before the sweep; a gather below that slot
// reads the copy.  The copy holds the values the sweep would load, so the
// results do not depend on its size.
//
// Ranks and contributions are FP32 (sums with Neumaier compensation per
// column, TwoSum when lanes combine); per-column residuals and dangling mass
// are FP64.  A column whose L1 residual drops below tol is frozen: its values
// stop changing and its sweep count is recorded; a pass ends when its four
// columns are frozen, and the launch when every pass has ended.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "device_common.h"
#include "internal.h"

using namespace fpr;
using namespace fpr::dev;

namespace {

constexpr int kBC = 4;           // columns per pass
constexpr int kBBlock = 512;     // threads per workgroup
constexpr int kBWaves = kBBlock / 64;
constexpr int kBFin = 256;       // threads of the finalize kernel
#ifndef FPR_BATCHED_HOT
#define FPR_BATCHED_HOT 3072
#endif
constexpr int kBHot = FPR_BATCHED_HOT;  // float4 gather slots staged in LDS (16 bytes each)
static_assert(kBHot % kBBlock == 0, "the LDS copy is loaded in whole rounds of the workgroup");

struct BState {
  double D[kBC];      // dangling mass per column of the current iterate
  double resid[kBC];  // last L1 change per column
  int done[kBC];      // column frozen
  int iters[kBC];     // sweeps until the column froze (or so far)
  int iter;           // sweeps run in this pass
  int all_done;       // every column frozen, or max_iter reached
  int max_iter;
  int pad;
  double tol;
};

struct BArgs {
  const uint32_t *rows;
  const uint32_t *rowpos;
  const uint32_t *rptr;
  const int32_t *idx;
  const int4 *items;
  const int4 *tiles;
  const int32_t *tidx;
  const uint8_t *tmask;
  const int4 *hsplit;
  const uint32_t *gpos;
  const double *inv_w;
  const int32_t *seeds;  // [passes * 4], -1 for padding columns
  float4 *x;             // [passes][n] vertex order
  float4 *c0;            // [passes][n] gather-layout order
  float4 *c1;
  double *hpart;         // [passes][n_chunks][4]
  double *wave_part;     // [passes][2][4][n_waves]: change, dangling per column
  BState *st;            // [passes]
  double d;
  double inv_n;
  int64_t n;
  int n_items;
  int n_split;
  int n_chunks;
  int n_waves;
  int chunk;
  int hot;  // gather slots staged in LDS (<= kBHot)
};

struct Col4 {
  LaneSum<float> v[kBC];
  __device__ __forceinline__ void add(const float4 &a) {
    v[0].add(a.x);
    v[1].add(a.y);
    v[2].add(a.z);
    v[3].add(a.w);
  }
  __device__ __forceinline__ Col4 shfl_up(int off) const {
    Col4 r;
#pragma unroll
    for (int c = 0; c < kBC; ++c) r.v[c] = v[c].shfl_up(off);
    return r;
  }
  __device__ __forceinline__ void add_before(const Col4 &e) {
#pragma unroll
    for (int c = 0; c < kBC; ++c) v[c].add_before(e.v[c]);
  }
  __device__ __forceinline__ void combine_with(const Col4 &l) {
#pragma unroll
    for (int c = 0; c < kBC; ++c) v[c].combine_with(l.v[c]);
  }
  __device__ __forceinline__ void group_reduce(int lanes) {
#pragma unroll
    for (int c = 0; c < kBC; ++c) v[c].group_reduce(lanes);
  }
};

struct BRed {
  double chg[kBC] = {0.0, 0.0, 0.0, 0.0};
  double dang[kBC] = {0.0, 0.0, 0.0, 0.0};
};

// Pass-local view: the pass index selects the columns and buffers.
struct BCtx {
  const BArgs *a;
  const float4 *cin;
  float4 *cout;
  float4 *x;
  double dterm[kBC];
  int seed[kBC];
  int done[kBC];
};

__device__ __forceinline__ BCtx make_bctx(const BArgs &a, int pass) {
  BCtx C;
  C.a = &a;
  const BState *st = a.st + pass;
  const int it = st->iter;
  const size_t off = (size_t)pass * a.n;
  C.cin = ((it & 1) ? a.c1 : a.c0) + off;
  C.cout = ((it & 1) ? a.c0 : a.c1) + off;
  C.x = a.x + off;
#pragma unroll
  for (int c = 0; c < kBC; ++c) {
    C.dterm[c] = st->D[c] * a.inv_n;
    C.seed[c] = a.seeds[pass * kBC + c];
    C.done[c] = st->done[c];
  }
  return C;
}

// The global load goes through an explicit global address-space pointer so
// that it is not merged with the LDS read into one flat load.
typedef float f4v __attribute__((ext_vector_type(4)));
using gptr4 = const __attribute__((address_space(1))) f4v *;

__device__ __forceinline__ float4 bgather(const BCtx &C, const float4 *hot, int32_t s) {
  const bool h = s < C.a->hot;
  const float4 vh = hot[h ? s : 0];
  float4 vg = vh;
  if (!h) {
    const f4v t = ((gptr4)C.cin)[s];
    vg = make_float4(t.x, t.y, t.z, t.w);
  }
  return vg;
}

// Copy of the pass's gather slots [0, hot) into LDS, all loads issued before
// the first LDS write.
__device__ __forceinline__ void bload_hot(const BCtx &C, float4 *hot) {
  constexpr int kPer = kBHot / kBBlock;
  const int H = C.a->hot;
  float4 buf[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int q = (int)threadIdx.x + k * kBBlock;
    buf[k] = q < H ? C.cin[q] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int q = (int)threadIdx.x + k * kBBlock;
    if (q < H) hot[q] = buf[k];
  }
}

__device__ __forceinline__ float comp(const float4 &v, int c) {
  return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

// Update of row-table entry i with column sums s[4]; frozen columns keep x.
__device__ __forceinline__ void bupdate(const BCtx &C, int i, const double *s, BRed &red) {
  const BArgs &a = *C.a;
  const uint32_t u = a.rows[i];
  const float4 xo = C.x[u];
  const double iw = a.inv_w[u];
  float xn[kBC];
#pragma unroll
  for (int c = 0; c < kBC; ++c) {
    const float old = comp(xo, c);
    if (C.done[c] || C.seed[c] < 0) {
      xn[c] = old;
    } else {
      const double tele = ((int)u == C.seed[c]) ? (1.0 - a.d) : 0.0;
      xn[c] = (float)(tele + a.d * (s[c] + C.dterm[c]));
      red.chg[c] += fabs((double)xn[c] - (double)old);
    }
  }
  C.x[u] = make_float4(xn[0], xn[1], xn[2], xn[3]);
  if (iw != 0.0) {
    C.cout[a.rowpos[i]] = make_float4((float)((double)xn[0] * iw), (float)((double)xn[1] * iw),
                                      (float)((double)xn[2] * iw), (float)((double)xn[3] * iw));
  } else {
#pragma unroll
    for (int c = 0; c < kBC; ++c) red.dang[c] += (double)xn[c];
  }
}

// Tile of short rows (see the single-vector sweep): lane l takes edges
// 8l..8l+7, a segmented scan across lanes completes rows; four columns at once.
__device__ __forceinline__ void btile(const BCtx &C, const float4 *hot, double (*rowsum)[kBC], int t,
                                      BRed &red) {
  const BArgs &a = *C.a;
  const int lane = threadIdx.x & 63;
  const int4 d = a.tiles[t];
  const int r0 = d.x, nr = d.y, ne = d.z;
  const size_t base = (size_t)t * kTileEdges;
  int32_t s[kBatch];
#pragma unroll
  for (int k = 0; k < kBatch; ++k) s[k] = a.tidx[base + k * 64 + lane];
  const uint32_t fl = a.tmask[(size_t)t * 64 + lane];
  float4 v[kBatch];
#pragma unroll
  for (int k = 0; k < kBatch; ++k) {
    v[k] = bgather(C, hot, s[k]);
    if (lane * kBatch + k >= ne) v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int pc = __popc(fl);
  int incl = pc;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  const int rowbase = incl - pc;
  Col4 cur, head;
  bool seen = false;
  int j = 0;
#pragma unroll
  for (int k = 0; k < kBatch; ++k) {
    const bool st = (fl >> k) & 1u;
    if (st && seen) {
#pragma unroll
      for (int c = 0; c < kBC; ++c) rowsum[rowbase + j - 1][c] = cur.v[c].value();
    }
    if (st && !seen) head = cur;
    j += st ? 1 : 0;
    seen = seen || st;
    if (st) cur = Col4();
    cur.add(v[k]);
  }
  if (!seen) head = cur;
  Col4 sc = cur;
  bool f = seen;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Col4 prev = sc.shfl_up(off);
    const bool pf = __shfl_up((int)f, off, 64) != 0;
    if (lane >= off) {
      if (!f) sc.add_before(prev);
      f = f || pf;
    }
  }
  Col4 carry = sc.shfl_up(1);
  if (lane == 0) carry = Col4();
  if (seen && lane > 0) {
    carry.combine_with(head);
#pragma unroll
    for (int c = 0; c < kBC; ++c) rowsum[rowbase - 1][c] = carry.v[c].value();
  }
  if (lane == ((ne - 1) >> 3)) {
#pragma unroll
    for (int c = 0; c < kBC; ++c) rowsum[nr - 1][c] = sc.v[c].value();
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int r = lane; r < nr; r += 64) bupdate(C, r0 + r, rowsum[r], red);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Edges [e0, e0 + L) summed by the whole wavefront (lanes stride the list).
__device__ __forceinline__ void bstride(const BCtx &C, const float4 *hot, uint32_t e0, int L, double *out) {
  const BArgs &a = *C.a;
  const int lane = threadIdx.x & 63;
  Col4 acc;
  for (int j0 = lane; j0 < L; j0 += kBatch * 64) {
    int32_t s[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) s[b] = j0 + 64 * b < L ? a.idx[e0 + j0 + 64 * b] : 0;
    float4 v[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) v[b] = bgather(C, hot, s[b]);
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
      if (j0 + 64 * b < L) acc.add(v[b]);
  }
  acc.group_reduce(64);
#pragma unroll
  for (int c = 0; c < kBC; ++c) out[c] = acc.v[c].value();
}

__global__ __launch_bounds__(kBBlock) void k_bsweep(BArgs a) {
  __shared__ __align__(16) float4 hot[kBHot];
  __shared__ double rowsum_all[kBWaves][kTileRows][kBC];
  const int pass = blockIdx.y;
  if (a.st[pass].all_done) return;
  const BCtx C = make_bctx(a, pass);
  bload_hot(C, hot);
  __syncthreads();
  const int gw = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kBWaves + (threadIdx.x >> 6)));
  const int lane = threadIdx.x & 63;
  double(*rowsum)[kBC] = rowsum_all[threadIdx.x >> 6];
  BRed red;
  for (int item = gw; item < a.n_items; item += a.n_waves) {
    const int4 wi = a.items[item];
    if (wi.x == kTile) {
      btile(C, hot, rowsum, wi.y, red);
    } else if (wi.x == kRows) {
      for (int r = wi.y; r < wi.z; ++r) {
        double s[kBC];
        const uint32_t e0 = a.rptr[r];
        bstride(C, hot, e0, (int)(a.rptr[r + 1] - e0), s);
        if (lane == 0) bupdate(C, r, s, red);
      }
    } else if (wi.x == kHeavy) {
      double s[kBC];
      const uint32_t rb = a.rptr[wi.y];
      const int L = (int)(a.rptr[wi.y + 1] - rb);
      const int ne = min(a.chunk, L - wi.z * a.chunk);
      bstride(C, hot, rb + (uint32_t)wi.z * (uint32_t)a.chunk, ne, s);
      if (lane == 0) {
        double *hp = a.hpart + ((size_t)pass * a.n_chunks + wi.w + wi.z) * kBC;
#pragma unroll
        for (int c = 0; c < kBC; ++c) hp[c] = s[c];
      }
    } else {
      const double zero[kBC] = {0.0, 0.0, 0.0, 0.0};
      for (int r = wi.y + lane; r < wi.z; r += 64) bupdate(C, r, zero, red);
    }
  }
  double *wp = a.wave_part + (size_t)pass * 2 * kBC * a.n_waves;
#pragma unroll
  for (int c = 0; c < kBC; ++c) {
    const double ch = wave_sum(red.chg[c]);
    const double dg = wave_sum(red.dang[c]);
    if (lane == 0) {
      wp[(size_t)c * a.n_waves + gw] = ch;
      wp[(size_t)(kBC + c) * a.n_waves + gw] = dg;
    }
  }
}

__global__ __launch_bounds__(kBFin) void k_bfinal(BArgs a) {
  __shared__ double s_red[2 * kBC][kBFin / 64];
  const int pass = blockIdx.x;
  BState *st = a.st + pass;
  if (st->all_done) return;
  const BCtx C = make_bctx(a, pass);
  BRed red;
  for (int h = threadIdx.x; h < a.n_split; h += kBFin) {
    const int4 hs = a.hsplit[h];
    double s[kBC] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < hs.z; ++k) {
      const double *hp = a.hpart + ((size_t)pass * a.n_chunks + hs.y + k) * kBC;
#pragma unroll
      for (int c = 0; c < kBC; ++c) s[c] += hp[c];
    }
    bupdate(C, hs.x, s, red);
  }
  const double *wp = a.wave_part + (size_t)pass * 2 * kBC * a.n_waves;
  for (int i = threadIdx.x; i < a.n_waves; i += kBFin) {
#pragma unroll
    for (int c = 0; c < kBC; ++c) {
      red.chg[c] += wp[(size_t)c * a.n_waves + i];
      red.dang[c] += wp[(size_t)(kBC + c) * a.n_waves + i];
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < kBC; ++c) {
    const double ch = wave_sum(red.chg[c]);
    const double dg = wave_sum(red.dang[c]);
    if (lane == 0) {
      s_red[c][wave] = ch;
      s_red[kBC + c][wave] = dg;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int it = st->iter + 1;
    st->iter = it;
    int all = 1;
    for (int c = 0; c < kBC; ++c) {
      double ch = 0.0, dg = 0.0;
      for (int w = 0; w < kBFin / 64; ++w) {
        ch += s_red[c][w];
        dg += s_red[kBC + c][w];
      }
      st->D[c] = dg;
      if (!st->done[c]) {
        st->resid[c] = ch;
        st->iters[c] = it;
        if (!(ch >= st->tol)) st->done[c] = 1;
      }
      all &= st->done[c];
    }
    if (all || it >= st->max_iter) st->all_done = 1;
  }
}

// x = one-hot seeds, c = x / W in gather order, partial dangling mass per column.
__global__ __launch_bounds__(kBlock) void k_binit(BArgs a, double *part, int nparts) {
  __shared__ double s_red[kBC][kWaves];
  const int pass = blockIdx.y;
  const size_t off = (size_t)pass * a.n;
  int seed[kBC];
#pragma unroll
  for (int c = 0; c < kBC; ++c) seed[c] = a.seeds[pass * kBC + c];
  double dang[kBC] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < a.n; u += (int64_t)gridDim.x * kBlock) {
    float xv[kBC];
#pragma unroll
    for (int c = 0; c < kBC; ++c) xv[c] = ((int)u == seed[c]) ? 1.0f : 0.0f;
    a.x[off + u] = make_float4(xv[0], xv[1], xv[2], xv[3]);
    const double iw = a.inv_w[u];
    if (iw != 0.0) {
      a.c0[off + a.gpos[u]] = make_float4((float)(xv[0] * iw), (float)(xv[1] * iw), (float)(xv[2] * iw),
                                          (float)(xv[3] * iw));
    } else {
#pragma unroll
      for (int c = 0; c < kBC; ++c) dang[c] += xv[c];
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < kBC; ++c) {
    const double v = wave_sum(dang[c]);
    if (lane == 0) s_red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < kBC; ++c) {
      double v = 0.0;
      for (int w = 0; w < kWaves; ++w) v += s_red[c][w];
      part[((size_t)pass * kBC + c) * nparts + blockIdx.x] = v;
    }
  }
}

__global__ void k_binit_final(BArgs a, const double *part, int nparts, double tol, int max_iter) {
  if (threadIdx.x != 0) return;
  const int pass = blockIdx.x;
  BState *st = a.st + pass;
  for (int c = 0; c < kBC; ++c) {
    double D = 0.0;
    for (int i = 0; i < nparts; ++i) D += part[((size_t)pass * kBC + c) * nparts + i];
    st->D[c] = D;
    st->resid[c] = INFINITY;
    const int active = a.seeds[pass * kBC + c] >= 0;
    st->done[c] = active ? 0 : 1;
    st->iters[c] = 0;
  }
  st->iter = 0;
  st->all_done = 0;
  st->max_iter = max_iter;
  st->tol = tol;
}

// Scatter the pass's columns into the caller's row-major X[n][k].
__global__ __launch_bounds__(kBlock) void k_bout(BArgs a, float *X, int k, int pass0) {
  const int pass = blockIdx.y;
  const size_t off = (size_t)pass * a.n;
  const int col0 = (pass0 + pass) * kBC;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < a.n; u += (int64_t)gridDim.x * kBlock) {
    const float4 v = a.x[off + u];
    float *row = X + (size_t)u * k + col0;
    if (col0 + 0 < k) row[0] = v.x;
    if (col0 + 1 < k) row[1] = v.y;
    if (col0 + 2 < k) row[2] = v.z;
    if (col0 + 3 < k) row[3] = v.w;
  }
}

__global__ void k_bseeds(const int32_t *seeds, int k, int32_t *out, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) out[i] = i < k ? seeds[i] : -1;
}

__global__ void k_bcheck(const int32_t *seeds, int k, int64_t n, int *bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k && (seeds[i] < 0 || seeds[i] >= n)) *bad = 1;
}

// ---------------------------------------------------------------- host --

struct BWork {
  int passes_cap = 0;
  float4 *x = nullptr, *c0 = nullptr, *c1 = nullptr;
  double *hpart = nullptr, *wave_part = nullptr, *part = nullptr;
  BState *st = nullptr;
  BState *host_st = nullptr;
  int32_t *seeds = nullptr;
  int seeds_cap = 0;
  int *flag = nullptr;
};

std::vector<std::pair<const pr_graph *, BWork>> g_bwork;

BWork *bwork_for(pr_graph *g) {
  for (auto &e : g_bwork)
    if (e.first == g) return &e.second;
  g_bwork.emplace_back(g, BWork());
  return &g_bwork.back().second;
}

int ensure_bwork(pr_graph *g, BWork &w, int passes) {
  int rc;
  if (w.passes_cap < passes) {
    const size_t n = (size_t)g->n;
    const DevPlan &P = g->fwd;
    if ((rc = fpr_dev_alloc(g, (void **)&w.x, sizeof(float4) * n * passes))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.c0, sizeof(float4) * n * passes))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.c1, sizeof(float4) * n * passes))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.hpart, sizeof(double) * kBC * (size_t)std::max(1, P.n_chunks) * passes)))
      return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.wave_part, sizeof(double) * 2 * kBC * (size_t)P.n_waves * passes)))
      return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.part, sizeof(double) * kBC * 1024 * passes))) return rc;
    if ((rc = fpr_dev_alloc(g, (void **)&w.st, sizeof(BState) * passes))) return rc;
    if (w.host_st) (void)hipHostFree(w.host_st);
    w.host_st = nullptr;
    if (hipHostMalloc((void **)&w.host_st, sizeof(BState) * passes) != hipSuccess)
      return pr_fail(PR_ENOMEM, "pinned allocation failed");
    w.passes_cap = passes;
  }
  if (!w.flag && (rc = fpr_dev_alloc(g, (void **)&w.flag, sizeof(int)))) return rc;
  return PR_OK;
}

int ensure_seeds(pr_graph *g, BWork &w, int total) {
  if (w.seeds_cap >= total) return PR_OK;
  int rc = fpr_dev_alloc(g, (void **)&w.seeds, sizeof(int32_t) * total);
  if (rc) return rc;
  w.seeds_cap = total;
  return PR_OK;
}

BArgs make_bargs(pr_graph *g, BWork &w, double d, int passes, int pass0) {
  const DevPlan &P = g->fwd;
  BArgs a;
  memset(&a, 0, sizeof(a));
  a.rows = P.rows;
  a.rowpos = P.rowpos;
  a.rptr = P.rptr;
  a.idx = P.idx;
  a.items = P.bitems;
  a.tiles = P.tiles;
  a.tidx = P.tidx;
  a.tmask = P.tmask;
  a.hsplit = P.hsplit;
  a.gpos = P.gpos;
  a.inv_w = g->inv_w;
  a.seeds = w.seeds + (size_t)pass0 * kBC;
  a.x = w.x;
  a.c0 = w.c0;
  a.c1 = w.c1;
  a.hpart = w.hpart;
  a.wave_part = w.wave_part;
  a.st = w.st;
  a.d = d;
  a.inv_n = 1.0 / (double)g->n;
  a.n = g->n;
  a.n_items = P.n_bitems;
  a.n_split = P.n_split;
  a.n_chunks = std::max(1, P.n_chunks);
  a.n_waves = P.n_waves;
  a.chunk = P.chunk;
  const int64_t hot = g->popts.hot_slots < 0 ? kBHot : std::min<int64_t>(g->popts.hot_slots, kBHot);
  a.hot = (int)std::min<int64_t>(hot, g->n);
  (void)passes;
  return a;
}

// Runs `passes` passes (starting at pass0 of the padded seed list) to
// convergence; writes their columns of X.  sweeps_out / resid_out: per column.
int run_passes(pr_graph *g, BWork &w, double d, double tol, int max_iter, int passes, int pass0,
               float *X, int k, int *iters, double *resid, bool write_out, int fixed_sweeps) {
  int rc;
  BArgs a = make_bargs(g, w, d, passes, pass0);
  const int igrid = (int)std::min<int64_t>(1024, (g->n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_binit, dim3(igrid, passes), dim3(kBlock), 0, g->work, a, w.part, igrid);
  hipLaunchKernelGGL(k_binit_final, dim3(passes), dim3(64), 0, g->work, a, (const double *)w.part, igrid,
                     fixed_sweeps > 0 ? -1.0 : tol, fixed_sweeps > 0 ? fixed_sweeps : max_iter);
  PR_HIP(hipGetLastError());
  const int grid = g->fwd.n_waves / kBWaves;
  if (grid * kBWaves != g->fwd.n_waves) return pr_fail(PR_EDEVICE, "batched: wave count mismatch");
  const int G = 8;
  int done_sweeps = 0;
  const int limit = fixed_sweeps > 0 ? fixed_sweeps : max_iter;
  for (;;) {
    const int cnt = std::min(G, limit - done_sweeps);
    for (int s = 0; s < cnt; ++s) {
      hipLaunchKernelGGL(k_bsweep, dim3(grid, passes), dim3(kBBlock), 0, g->work, a);
      hipLaunchKernelGGL(k_bfinal, dim3(passes), dim3(kBFin), 0, g->work, a);
    }
    PR_HIP(hipGetLastError());
    PR_HIP(hipMemcpyAsync(w.host_st, w.st, sizeof(BState) * passes, hipMemcpyDeviceToHost, g->work));
    PR_HIP(hipStreamSynchronize(g->work));
    done_sweeps += cnt;
    bool all = true;
    for (int p = 0; p < passes; ++p) all &= w.host_st[p].all_done != 0;
    if (all || done_sweeps >= limit) break;
  }
  if (write_out) {
    hipLaunchKernelGGL(k_bout, dim3(igrid, passes), dim3(kBlock), 0, g->work, a, X, k, pass0);
    PR_HIP(hipGetLastError());
  }
  if (iters && resid) {
    for (int p = 0; p < passes; ++p)
      for (int c = 0; c < kBC; ++c) {
        const int col = (pass0 + p) * kBC + c;
        if (col < k) {
          iters[col] = w.host_st[p].iters[c];
          resid[col] = w.host_st[p].resid[c];
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
  snprintf(buf, sizeof(buf), "n=%lld,m=%lld,k=%d,dev=%s", (long long)g->n, (long long)g->m, k, dev);
  return buf;
}

int tune_lookup(const char *path, const std::string &key) {
  if (!path) return 0;
  FILE *f = fopen(path, "r");
  if (!f) return 0;
  char line[1024];
  int best = 0;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof(line), f)) {
    if (strstr(line, pat.c_str())) {
      const char *t = strstr(line, "\"tile\": ");
      if (t) best = atoi(t + 8);
    }
  }
  fclose(f);
  return best;
}

struct TuneMemo {
  const pr_graph *g;
  int k;
  int tile;
};
std::vector<TuneMemo> g_tune_memo;

}  // namespace

void fpr_batched_release(pr_graph *g) {
  for (size_t i = 0; i < g_bwork.size();) {
    if (g_bwork[i].first == g) {
      if (g_bwork[i].second.host_st) (void)hipHostFree(g_bwork[i].second.host_st);
      g_bwork.erase(g_bwork.begin() + i);
    } else {
      ++i;
    }
  }
  for (size_t i = 0; i < g_tune_memo.size();) {
    if (g_tune_memo[i].g == g) g_tune_memo.erase(g_tune_memo.begin() + i);
    else ++i;
  }
}

extern "C" int pr_autotune_batched(pr_graph *g, int k, const char *cache_path, int *tile, void *stream) {
  pr_clear_error();
  if (!g || !tile) return pr_fail(PR_EINVAL, "pr_autotune_batched: NULL argument");
  if (k < 1 || k > 1024) return pr_fail(PR_EINVAL, "k=%d outside [1, 1024]", k);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  const std::string key = tune_key(g, k);
  for (auto &m : g_tune_memo)
    if (m.g == g && m.k == k) {
      *tile = m.tile;
      return PR_OK;
    }
  int cached = tune_lookup(cache_path, key);
  if (cached > 0) {
    *tile = cached;
    g_tune_memo.push_back(TuneMemo{g, k, cached});
    return PR_OK;
  }
  hipStream_t user = (hipStream_t)stream;
  (void)hipEventRecord(g->ev_in, user);
  (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  BWork &w = *bwork_for(g);
  const int kpad = (k + kBC - 1) / kBC * kBC;
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
  int best = kBC;
  const int sweeps = 4;
  for (int t = kBC; t <= std::max(kBC, std::min(64, kpad)); t *= 2) {
    const int passes = t / kBC;
    if ((rc = ensure_bwork(g, w, passes))) return rc;
    // one warm-up, one timed run of `sweeps` sweeps on `passes` passes
    if ((rc = run_passes(g, w, 0.85, 1.0, sweeps, passes, 0, nullptr, k, nullptr, nullptr, false, sweeps)))
      return rc;
    PR_HIP(hipEventRecord(e0, g->work));
    if ((rc = run_passes(g, w, 0.85, 1.0, sweeps, passes, 0, nullptr, k, nullptr, nullptr, false, sweeps)))
      return rc;
    PR_HIP(hipEventRecord(e1, g->work));
    PR_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    PR_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double per_col = ms / (double)t;
    if (per_col < best_t) {
      best_t = per_col;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventRecord(g->ev_out, g->work);
  (void)hipStreamWaitEvent(user, g->ev_out, 0);
  *tile = best;
  g_tune_memo.push_back(TuneMemo{g, k, best});
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{\"key\": \"%s\", \"tile\": %d, \"ms_per_column_sweep\": %.6f}\n", key.c_str(), best,
              best_t / sweeps);
      fclose(f);
    }
  }
  return PR_OK;
}

extern "C" int pr_solve_batched(pr_graph *g, double d, double tol, int max_iter, int k,
                                const int32_t *seeds, int tile, float *X, int *iters, double *resid,
                                void *stream) {
  pr_clear_error();
  if (!g) return pr_fail(PR_EINVAL, "graph is NULL");
  if (!(d > 0.0 && d < 1.0)) return pr_fail(PR_EINVAL, "d=%g is not in (0, 1)", d);
  if (!(tol > 0.0)) return pr_fail(PR_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return pr_fail(PR_EINVAL, "max_iter=%d must be >= 1", max_iter);
  if (k < 1 || k > 1024) return pr_fail(PR_EINVAL, "k=%d outside [1, 1024]", k);
  if (!seeds || !X || !iters || !resid) return pr_fail(PR_EINVAL, "NULL argument");
  if (tile < 0 || tile > 64 || (tile % kBC) != 0)
    return pr_fail(PR_EINVAL, "tile=%d must be 0 (autotune) or a multiple of %d up to 64", tile, kBC);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return pr_fail(PR_EINVAL, "the graph lives on device %d but device %d is current", g->device, cur);
  int rc;
  if (tile == 0) {
    if ((rc = pr_autotune_batched(g, k, getenv("FUSEDPR_TUNE_CACHE"), &tile, stream))) return rc;
  }
  hipStream_t user = (hipStream_t)stream;
  (void)hipEventRecord(g->ev_in, user);
  (void)hipStreamWaitEvent(g->work, g->ev_in, 0);
  BWork &w = *bwork_for(g);
  const int kpad = (k + kBC - 1) / kBC * kBC;
  const int npass = kpad / kBC;
  const int per_launch = std::min(npass, tile / kBC);
  if ((rc = ensure_seeds(g, w, kpad))) return rc;
  if ((rc = ensure_bwork(g, w, per_launch))) return rc;
  hipLaunchKernelGGL(k_bseeds, dim3((kpad + 255) / 256), dim3(256), 0, g->work, seeds, k, w.seeds, kpad);
  PR_HIP(hipMemsetAsync(w.flag, 0, sizeof(int), g->work));
  hipLaunchKernelGGL(k_bcheck, dim3((k + 255) / 256), dim3(256), 0, g->work, seeds, k, (int64_t)g->n, w.flag);
  int bad = 0;
  PR_HIP(hipMemcpyAsync(&bad, w.flag, sizeof(int), hipMemcpyDeviceToHost, g->work));
  PR_HIP(hipStreamSynchronize(g->work));
  if (bad) return pr_fail(PR_EINVAL, "a seed vertex is outside [0, %lld)", (long long)g->n);
  for (int p0 = 0; p0 < npass; p0 += per_launch) {
    const int passes = std::min(per_launch, npass - p0);
    if ((rc = run_passes(g, w, d, tol, max_iter, passes, p0, X, k, iters, resid, true, 0))) return rc;
  }
  PR_HIP(hipStreamSynchronize(g->work));
  (void)hipEventRecord(g->ev_out, g->work);
  (void)hipStreamWaitEvent(user, g->ev_out, 0);
  for (int j = 0; j < k; ++j)
    if (!(resid[j] < tol)) return PR_NOT_CONVERGED;
  return PR_OK;
}
