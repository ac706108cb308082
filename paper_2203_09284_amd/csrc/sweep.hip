// The PageRank sweep on gfx950: one persistent kernel per sweep that pulls,
// updates, and reduces, in the two forms of the paper.
//
//  * Jacobi (Section 3, Algorithm 1): contributions are double-buffered; sweep
//    k reads c_k and writes c_{k+1}, so every vertex sees the previous sweep.
//  * Fused (Section 4, Algorithm 2; Eq. 9): one contribution array, updated in
//    place right after each vertex's rank; work items are claimed in ticket
//    order, so items that start later read the contributions written by items
//    that finished earlier in the same sweep (the paper's parallel variant,
//    Section 6.3, an asynchronous Gauss-Seidel iteration).  Reads and writes
//    of the shared array are relaxed atomics: a reader gets either the old or
//    the new value, never a torn one.
//
// Per vertex u the update is Eq. 1 with the dangling mass D spread uniformly,
//     x_u <- (1-d) p_u s + d (sum_{v->u} w c_v + D/n),   c_u <- x_u / W_u,
// where s = 1, except in the fused mass-scaled mode where s is the previous
// sweep's total mass (see the mode flag kFlagScaled).  The per-vertex change,
// the new dangling mass and the new total mass are reduced in FP64 per work
// item; the last workgroup to finish sums the item partials in item order
// (deterministic), sets the residual, the iteration count and the stop flag,
// and resets the ticket, so the next launch needs no host work.
//
// FP32 storage (ranks and contributions) sums with Neumaier compensation per
// lane and TwoSum when lanes combine; the rank update and every reduction are
// FP64.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace fpr;

// Memory scope of the relaxed atomic loads/stores of the shared contribution
// array in the fused form.
#ifndef FPR_FUSED_SCOPE
#define FPR_FUSED_SCOPE __HIP_MEMORY_SCOPE_AGENT
#endif

namespace {

// ------------------------------------------------------------ arithmetic --

// Per-lane sum: plain FP64, or FP32 with Neumaier compensation.
template <typename T>
struct LaneSum;

template <>
struct LaneSum<double> {
  double s = 0.0;
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ double value() const { return s; }
  __device__ __forceinline__ void wave_reduce() {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
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
  // TwoSum of the leading parts, compensations added
  __device__ __forceinline__ void combine(float s2, float c2) {
#pragma clang fp contract(off)
    float t = s + s2;
    float bp = t - s;
    float err = (s - (t - bp)) + (s2 - bp);
    c = c + c2 + err;
    s = t;
  }
  __device__ __forceinline__ void wave_reduce() {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
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

template <bool FUSED, typename T>
__device__ __forceinline__ T ld_c(const T *p) {
  if constexpr (FUSED) return __hip_atomic_load(p, __ATOMIC_RELAXED, FPR_FUSED_SCOPE);
  else return *p;
}

template <bool FUSED, typename T>
__device__ __forceinline__ void st_c(T *p, T v) {
  if constexpr (FUSED) __hip_atomic_store(p, v, __ATOMIC_RELAXED, FPR_FUSED_SCOPE);
  else *p = v;
}

// ------------------------------------------------------------ arguments --

template <typename T>
struct SweepArgs {
  const uint32_t *rows;
  const uint32_t *rptr;
  const int32_t *idx;
  const double *w;
  const int4 *items;
  const uint32_t *hbase;
  double *hpart;
  unsigned *hcnt;
  double *item_part;
  SweepState *st;
  const double *inv_w;
  const double *p;
  T *x;
  T *c0;
  T *c1;
  double *trace;
  double d;
  double inv_n;
  int n_items;
  int split;
  int flags;
};

template <typename T>
struct Ctx {
  const uint32_t *rows;
  const uint32_t *rptr;
  const int32_t *idx;
  const double *w;
  const double *inv_w;
  const double *p;
  T *x;
  const T *cin;
  T *cout;
  double tele;   // (1-d) * mass scale
  double d;
  double dterm;  // D / n, 0 in leak mode
  double inv_n;
  int flags;
};

template <typename T, bool FUSED>
__device__ __forceinline__ void update_vertex(const Ctx<T> &C, uint32_t u, double s, Red &red) {
  const double xo = (double)C.x[u];
  const double pu = (C.flags & kFlagUniformP) ? C.inv_n : C.p[u];
  const double xn = C.tele * pu + C.d * (s + C.dterm);
  const T xs = (T)xn;
  C.x[u] = xs;
  const double xd = (double)xs;
  const double iw = C.inv_w[u];
  if (iw != 0.0) st_c<FUSED>(C.cout + u, (T)(xd * iw));
  else red.dang += xd;
  const double dl = fabs(xd - xo);
  red.chg = (C.flags & kFlagLinf) ? fmax(red.chg, dl) : red.chg + dl;
  red.tot += xd;
}

// ---------------------------------------------------- work item kinds --

// Thread per vertex: the block's edges (contiguous, <= kLightCap) are
// gathered edge-parallel into LDS, then each thread sums its vertex's slice.
template <typename T, bool FUSED, bool WEIGHTED>
__device__ __forceinline__ void light_block(const Ctx<T> &C, int i0, int i1, T *lds, Red &red) {
  const uint32_t eb = C.rptr[i0];
  const int ne = (int)(C.rptr[i1] - eb);
  constexpr int K = kLightCap / kBlock;
  int32_t src[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = threadIdx.x + k * kBlock;
    src[k] = j < ne ? C.idx[eb + j] : 0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = threadIdx.x + k * kBlock;
    if (j < ne) {
      T v = ld_c<FUSED>(C.cin + src[k]);
      if constexpr (WEIGHTED) v = (T)((double)v * C.w[eb + j]);
      lds[j] = v;
    }
  }
  __syncthreads();
  const int r = i0 + (int)threadIdx.x;
  if (r < i1) {
    const int a = (int)(C.rptr[r] - eb), b = (int)(C.rptr[r + 1] - eb);
    LaneSum<T> acc;
    for (int j = a; j < b; ++j) acc.add(lds[j]);
    update_vertex<T, FUSED>(C, C.rows[r], acc.value(), red);
  }
  __syncthreads();
}

// Wavefront per vertex: 64 lanes stride over the vertex's edges.
template <typename T, bool FUSED, bool WEIGHTED>
__device__ __forceinline__ void medium_group(const Ctx<T> &C, int i0, int i1, Red &red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = i0 + wave; r < i1; r += kWaves) {
    const uint32_t eb = C.rptr[r];
    const int L = (int)(C.rptr[r + 1] - eb);
    LaneSum<T> acc;
    for (int j0 = 0; j0 < L; j0 += 4 * 64) {
      int32_t s[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = j0 + lane + 64 * k;
        s[k] = j < L ? C.idx[eb + j] : 0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = j0 + lane + 64 * k;
        if (j < L) {
          T v = ld_c<FUSED>(C.cin + s[k]);
          if constexpr (WEIGHTED) v = (T)((double)v * C.w[eb + j]);
          acc.add(v);
        }
      }
    }
    acc.wave_reduce();
    if (lane == 0) update_vertex<T, FUSED>(C, C.rows[r], acc.value(), red);
  }
}

// Workgroup per chunk of a long row; chunk partials combined in order by the
// last chunk to arrive.
template <typename T, bool FUSED, bool WEIGHTED>
__device__ __forceinline__ void heavy_chunk(const Ctx<T> &C, const SweepArgs<T> &a, int i, int c,
                                            int h, Red &red) {
  __shared__ double s_part[kWaves];
  const uint32_t rb = C.rptr[i];
  const int L = (int)(C.rptr[i + 1] - rb);
  const int split = a.split;
  const uint32_t eb = rb + (uint32_t)c * (uint32_t)split;
  const int ne = min(split, L - c * split);
  LaneSum<T> acc;
  for (int j0 = 0; j0 < ne; j0 += 8 * kBlock) {
    int32_t s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = j0 + (int)threadIdx.x + kBlock * k;
      s[k] = j < ne ? C.idx[eb + j] : 0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = j0 + (int)threadIdx.x + kBlock * k;
      if (j < ne) {
        T v = ld_c<FUSED>(C.cin + s[k]);
        if constexpr (WEIGHTED) v = (T)((double)v * C.w[eb + j]);
        acc.add(v);
      }
    }
  }
  acc.wave_reduce();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) s_part[wave] = acc.value();
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) sum += s_part[k];
    const int nch = (L + split - 1) / split;
    if (nch == 1) {
      update_vertex<T, FUSED>(C, C.rows[i], sum, red);
    } else {
      const uint32_t base = a.hbase[h];
      a.hpart[base + c] = sum;
      __threadfence();
      const unsigned prev = atomicAdd(&a.hcnt[h], 1u);
      if (prev == (unsigned)(nch - 1)) {
        __threadfence();
        double tot = 0.0;
        for (int k = 0; k < nch; ++k) tot += __hip_atomic_load(&a.hpart[base + k], __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
        a.hcnt[h] = 0u;
        update_vertex<T, FUSED>(C, C.rows[i], tot, red);
      }
    }
  }
  __syncthreads();
}

// Block reduction of a thread's Red; thread 0 writes the item partial.
__device__ __forceinline__ void store_item_partial(Red &red, double *dst, bool linf) {
  __shared__ double s_red[3][kWaves];
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
    double a = s_red[0][0], b = s_red[1][0], c = s_red[2][0];
#pragma unroll
    for (int k = 1; k < kWaves; ++k) {
      a = linf ? fmax(a, s_red[0][k]) : a + s_red[0][k];
      b += s_red[1][k];
      c += s_red[2][k];
    }
    dst[0] = a;
    dst[1] = b;
    dst[2] = c;
  }
  __syncthreads();
}

// Sum the per-item partials in item order (fixed split over the threads, fixed
// tree), then publish the sweep result.  Runs in the last workgroup.
template <typename T>
__device__ void finalize_sweep(const SweepArgs<T> &a, double S_old, double *scratch) {
  double(*s_red)[kBlock] = reinterpret_cast<double(*)[kBlock]>(scratch);
  const bool linf = (a.flags & kFlagLinf) != 0;
  const int n = a.n_items;
  const int per = (n + kBlock - 1) / kBlock;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  double chg = 0.0, dang = 0.0, tot = 0.0;
  for (int i = lo; i < hi; ++i) {
    const double *q = a.item_part + 3 * (size_t)i;
    const double c0 = __hip_atomic_load(q + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    chg = linf ? fmax(chg, c0) : chg + c0;
    dang += __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tot += __hip_atomic_load(q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  s_red[0][threadIdx.x] = chg;
  s_red[1][threadIdx.x] = dang;
  s_red[2][threadIdx.x] = tot;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_red[0][threadIdx.x] = linf ? fmax(s_red[0][threadIdx.x], s_red[0][threadIdx.x + s])
                                   : s_red[0][threadIdx.x] + s_red[0][threadIdx.x + s];
      s_red[1][threadIdx.x] += s_red[1][threadIdx.x + s];
      s_red[2][threadIdx.x] += s_red[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    SweepState *st = a.st;
    const double raw = s_red[0][0];
    const double Sn = s_red[2][0];
    double resid = raw;
    if (a.flags & kFlagScaled) resid = (raw + fabs(Sn - S_old)) / S_old;
    st->raw = raw;
    st->resid = resid;
    st->D = s_red[1][0];
    st->S = Sn;
    const int it = st->iter + 1;
    st->iter = it;
    if (a.trace) a.trace[it - 1] = resid;
    if (!(resid >= st->tol) || it >= st->max_iter) st->done = 1;
    st->ticket = 0u;
    st->finished = 0u;
  }
}

static_assert(kLightCap * sizeof(float) >= 3 * kBlock * sizeof(double), "LDS reuse by the final reduction");

template <typename T, bool FUSED, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs<T> a) {
  __shared__ __attribute__((aligned(16))) T lds[kLightCap];
  __shared__ int s_item;
  __shared__ int s_last;
  SweepState *st = a.st;
  if (st->done) return;
  const int it = st->iter;
  const double S = st->S, D = st->D;
  Ctx<T> C;
  C.rows = a.rows;
  C.rptr = a.rptr;
  C.idx = a.idx;
  C.w = a.w;
  C.inv_w = a.inv_w;
  C.p = a.p;
  C.x = a.x;
  if (FUSED) {
    C.cin = a.c0;
    C.cout = a.c0;
  } else {
    C.cin = (it & 1) ? a.c1 : a.c0;
    C.cout = (it & 1) ? a.c0 : a.c1;
  }
  C.d = a.d;
  C.inv_n = a.inv_n;
  C.flags = a.flags;
  C.tele = (1.0 - a.d) * ((a.flags & kFlagScaled) ? S : 1.0);
  C.dterm = (a.flags & kFlagLeak) ? 0.0 : D * a.inv_n;
  const bool linf = (a.flags & kFlagLinf) != 0;

  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&st->ticket, 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= a.n_items) break;
    const int4 wi = a.items[item];
    Red red;
    if (wi.x == kLight) light_block<T, FUSED, WEIGHTED>(C, wi.y, wi.z, lds, red);
    else if (wi.x == kMedium) medium_group<T, FUSED, WEIGHTED>(C, wi.y, wi.z, red);
    else heavy_chunk<T, FUSED, WEIGHTED>(C, a, wi.y, wi.z, wi.w, red);
    store_item_partial(red, a.item_part + 3 * (size_t)item, linf);
  }

  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&st->finished, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  finalize_sweep<T>(a, S, reinterpret_cast<double *>(lds));
}

// ------------------------------------------------------- init / finish --

template <typename T>
struct InitArgs {
  const double *inv_w;
  const double *p;
  const double *x_in;  // warm start (FP64), or null: start from p
  T *x;
  T *c;
  double *part;  // [gridDim.x * 2]
  int64_t n;
  double inv_n;
  int uniform_p;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(InitArgs<T> a) {
  __shared__ double s_red[2][kWaves];
  double dang = 0.0, tot = 0.0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < a.n;
       u += (int64_t)gridDim.x * kBlock) {
    double xv = a.x_in ? a.x_in[u] : (a.uniform_p ? a.inv_n : a.p[u]);
    T xs = (T)xv;
    a.x[u] = xs;
    const double xd = (double)xs;
    const double iw = a.inv_w[u];
    if (iw != 0.0) a.c[u] = (T)(xd * iw);
    else dang += xd;
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
    a.part[2 * blockIdx.x] = a0;
    a.part[2 * blockIdx.x + 1] = a1;
  }
}

__global__ void k_init_final(const double *part, int nparts, SweepState *st, double tol,
                             int max_iter) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double D = 0.0, S = 0.0;
  for (int i = 0; i < nparts; ++i) {
    D += part[2 * i];
    S += part[2 * i + 1];
  }
  st->ticket = 0u;
  st->finished = 0u;
  st->iter = 0;
  st->done = 0;
  st->max_iter = max_iter;
  st->tol = tol;
  st->D = D;
  st->S = S;
  st->resid = INFINITY;
  st->raw = INFINITY;
}

// x64[u] = x[u] * scale (FP32 or FP64 source; scale = 1/S for mass-scaled iterates)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to64(const T *x, double *out, int64_t n,
                                                 const SweepState *st, int scaled) {
  const double scale = scaled ? 1.0 / st->S : 1.0;
  for (int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kBlock)
    out[u] = (double)x[u] * scale;
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

int ensure_trace(pr_graph *g, int max_iter) {
  if (g->trace_cap >= max_iter) return PR_OK;
  int rc = fpr_dev_alloc(g, (void **)&g->trace_dev, sizeof(double) * (size_t)max_iter);
  if (rc) return rc;
  g->trace_cap = max_iter;
  return PR_OK;
}

template <typename T>
int launch_init(pr_graph *g, DevPlan &P, const double *p, const double *x_in, T *x, double tol,
                int max_iter) {
  InitArgs<T> a;
  a.inv_w = g->inv_w;
  a.p = p;
  a.x_in = x_in;
  a.x = x;
  a.c = contrib<T>(g, 0);
  a.part = g->red_tmp;
  a.n = g->n;
  a.inv_n = 1.0 / (double)g->n;
  a.uniform_p = p == nullptr;
  const int grid = (int)std::min<int64_t>(kInitGrid, (g->n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_init<T>, dim3(grid), dim3(kBlock), 0, g->work, a);
  hipLaunchKernelGGL(k_init_final, dim3(1), dim3(64), 0, g->work, (const double *)g->red_tmp, grid,
                     P.st, tol, max_iter);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

template <typename T>
SweepArgs<T> make_args(pr_graph *g, DevPlan &P, const double *p, T *x, double d, int flags,
                       double *trace) {
  SweepArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.rows = P.rows;
  a.rptr = P.rptr;
  a.idx = P.idx;
  a.w = P.w;
  a.items = P.items;
  a.hbase = P.hbase;
  a.hpart = P.hpart;
  a.hcnt = P.hcnt;
  a.item_part = P.item_part;
  a.st = P.st;
  a.inv_w = g->inv_w;
  a.p = p;
  a.x = x;
  a.c0 = contrib<T>(g, 0);
  a.c1 = contrib<T>(g, 1);
  a.trace = trace;
  a.d = d;
  a.inv_n = 1.0 / (double)g->n;
  a.n_items = P.n_items;
  a.split = P.split;
  a.flags = flags | (p ? 0 : kFlagUniformP);
  return a;
}

template <typename T>
void launch_sweeps(pr_graph *g, const SweepArgs<T> &a, bool fused, bool weighted, int count,
                   hipStream_t s) {
  for (int k = 0; k < count; ++k) {
    if (fused) {
      if (weighted) hipLaunchKernelGGL((k_sweep<T, true, true>), dim3(g->grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((k_sweep<T, true, false>), dim3(g->grid), dim3(kBlock), 0, s, a);
    } else {
      if (weighted) hipLaunchKernelGGL((k_sweep<T, false, true>), dim3(g->grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((k_sweep<T, false, false>), dim3(g->grid), dim3(kBlock), 0, s, a);
    }
  }
}

// Cached hipGraph executables of `count` sweeps for one exact argument set.
struct GraphEntry {
  const void *key_graph;
  std::vector<unsigned char> key;
  hipGraphExec_t exec;
};
static std::vector<GraphEntry> g_graph_cache;

template <typename T>
int run_sweeps(pr_graph *g, const SweepArgs<T> &a, bool fused, bool use_graph, int count) {
  if (!use_graph) {
    launch_sweeps(g, a, fused, g->weighted, count, g->work);
    PR_HIP(hipGetLastError());
    return PR_OK;
  }
  std::vector<unsigned char> key(sizeof(a) + 3 * sizeof(int));
  memcpy(key.data(), &a, sizeof(a));
  int extra[3] = {fused ? 1 : 0, count, (int)sizeof(T)};
  memcpy(key.data() + sizeof(a), extra, sizeof(extra));
  for (auto &e : g_graph_cache) {
    if (e.key_graph == g && e.key == key) {
      PR_HIP(hipGraphLaunch(e.exec, g->work));
      return PR_OK;
    }
  }
  if (g_graph_cache.size() >= 32) {
    for (auto &e : g_graph_cache) (void)hipGraphExecDestroy(e.exec);
    g_graph_cache.clear();
  }
  hipGraph_t graph;
  PR_HIP(hipStreamBeginCapture(g->work, hipStreamCaptureModeThreadLocal));
  launch_sweeps(g, a, fused, g->weighted, count, g->work);
  hipError_t le = hipGetLastError();
  hipError_t ce = hipStreamEndCapture(g->work, &graph);
  if (le != hipSuccess) return pr_fail(PR_EDEVICE, "sweep launch during capture: %s", hipGetErrorString(le));
  if (ce != hipSuccess) return pr_fail(PR_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ce));
  hipGraphExec_t exec;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return pr_fail(PR_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  g_graph_cache.push_back(GraphEntry{g, key, exec});
  PR_HIP(hipGraphLaunch(exec, g->work));
  return PR_OK;
}

int poll_state(pr_graph *g, DevPlan &P) {
  PR_HIP(hipMemcpyAsync(g->host_st, P.st, sizeof(SweepState), hipMemcpyDeviceToHost, g->work));
  PR_HIP(hipStreamSynchronize(g->work));
  return PR_OK;
}

// One stage: init from (p | x_in) then sweeps until the state says done.
// stall: stop polling once the residual fails to halve between polls (FP32 floor).
template <typename T>
int solve_stage(pr_graph *g, double d, double tol, int max_iter, const pr_opts &o, const double *p,
                const double *x_in, T *x, int flags, bool fused, double *trace, bool stall,
                int *iters, double *resid) {
  int rc;
  if ((rc = ensure_contrib<T>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<T>(g, P, p, x_in, x, tol, max_iter))) return rc;
  SweepArgs<T> a = make_args<T>(g, P, p, x, d, flags, trace);
  const int G = std::max(1, o.sweeps_per_poll);
  double prev = INFINITY;
  int done_sweeps = 0;
  for (;;) {
    const int cnt = std::min(G, max_iter - done_sweeps);
    if ((rc = run_sweeps<T>(g, a, fused, o.use_hip_graph != 0, cnt))) return rc;
    if ((rc = poll_state(g, P))) return rc;
    done_sweeps = g->host_st->iter;
    if (g->host_st->done || done_sweeps >= max_iter) break;
    const double r = g->host_st->resid;
    if (!(r == r)) return pr_fail(PR_EDEVICE, "residual is NaN after sweep %d", done_sweeps);
    if (stall && r >= 0.5 * prev) break;
    prev = r;
  }
  *iters = g->host_st->iter;
  *resid = g->host_st->resid;
  return PR_OK;
}

int validate_common(pr_graph *g, double d, const pr_opts &o) {
  if (!g) return pr_fail(PR_EINVAL, "graph is NULL");
  if (!(d > 0.0 && d < 1.0)) return pr_fail(PR_EINVAL, "d=%g is not in (0, 1)", d);
  if (o.mode != PR_JACOBI && o.mode != PR_FUSED) return pr_fail(PR_EINVAL, "bad mode %d", o.mode);
  if (o.precision != PR_FP64 && o.precision != PR_FP32)
    return pr_fail(PR_EINVAL, "bad precision %d", o.precision);
  if (o.dangling != PR_DANGLING_UNIFORM && o.dangling != PR_DANGLING_LEAK)
    return pr_fail(PR_EINVAL, "bad dangling mode %d", o.dangling);
  if (o.norm != PR_NORM_L1 && o.norm != PR_NORM_LINF) return pr_fail(PR_EINVAL, "bad norm %d", o.norm);
  if (o.mode == PR_FUSED && o.fused_scaled && (o.dangling != PR_DANGLING_UNIFORM || o.norm != PR_NORM_L1))
    return pr_fail(PR_EINVAL, "the mass-scaled fused form needs uniform dangling and the L1 norm");
  if (o.mode == PR_FUSED && o.norm == PR_NORM_LINF)
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
  if (o.mode == PR_FUSED && o.fused_scaled) f |= kFlagScaled;
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

int fpr_grid_for(pr_graph *g) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep<double, false, false>, kBlock, 0) !=
          hipSuccess ||
      nb < 1)
    nb = 4;
  nb = std::min(nb, 8);
  return std::max(1, g->n_cu) * nb;
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

extern "C" int pr_solve(pr_graph *g, double d, double tol, int max_iter, const pr_opts *opts,
                        const double *p, double *x, int *iters, double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!(tol > 0.0)) return pr_fail(PR_EINVAL, "tol=%g must be > 0", tol);
  if (max_iter < 1) return pr_fail(PR_EINVAL, "max_iter=%d must be >= 1", max_iter);
  if (!x) return pr_fail(PR_EINVAL, "x is NULL");
  if (!iters || !resid) return pr_fail(PR_EINVAL, "iters/resid are NULL");
  StreamJoin join(g, stream);
  double *trace = nullptr;
  if (o.trace) {
    if ((rc = ensure_trace(g, max_iter))) return rc;
    trace = g->trace_dev;
  }
  const int flags = flags_of(o);
  const bool fused = o.mode == PR_FUSED;
  const bool scaled = (flags & kFlagScaled) != 0;
  int it = 0;
  double r = INFINITY;
  double target = tol;
  if (o.precision == PR_FP64) {
    if ((rc = solve_stage<double>(g, d, tol, max_iter, o, p, o.warm_start ? x : nullptr, x, flags,
                                  fused, trace, false, &it, &r)))
      return rc;
    if (scaled) {
      hipLaunchKernelGGL(k_to64<double>, dim3(kInitGrid), dim3(kBlock), 0, g->work, (const double *)x,
                         x, g->n, (const SweepState *)g->fwd.st, 1);
    }
  } else {
    if (!g->x32 && (rc = fpr_dev_alloc(g, (void **)&g->x32, sizeof(float) * (size_t)g->n))) return rc;
    const double tol32 = o.fp32_tol > 0.0 ? o.fp32_tol : std::max(tol, 1e-7);
    const double rtol = o.refine_tol < 0.0 ? tol : o.refine_tol;
    if ((rc = solve_stage<float>(g, d, tol32, max_iter, o, p, o.warm_start ? x : nullptr, g->x32,
                                 flags, fused, trace, rtol > 0.0, &it, &r)))
      return rc;
    target = rtol > 0.0 ? rtol : tol32;
    hipLaunchKernelGGL(k_to64<float>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                       (const float *)g->x32, x, g->n, (const SweepState *)g->fwd.st, scaled ? 1 : 0);
    if (rtol > 0.0 && it < max_iter) {
      int it2 = 0;
      double r2 = INFINITY;
      if ((rc = solve_stage<double>(g, d, rtol, max_iter - it, o, p, x, x, flags, fused,
                                    trace ? trace + it : nullptr, false, &it2, &r2)))
        return rc;
      if (scaled)
        hipLaunchKernelGGL(k_to64<double>, dim3(kInitGrid), dim3(kBlock), 0, g->work,
                           (const double *)x, x, g->n, (const SweepState *)g->fwd.st, 1);
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

extern "C" int pr_iterate(pr_graph *g, double d, const pr_opts *opts, const double *p, double *x,
                          int sweeps, double *resid, void *stream) {
  pr_clear_error();
  pr_opts o;
  pr_opts_default(&o);
  if (opts) o = *opts;
  o.precision = PR_FP64;
  int rc = validate_common(g, d, o);
  if (rc) return rc;
  if (!x) return pr_fail(PR_EINVAL, "x is NULL");
  if (sweeps < 0) return pr_fail(PR_EINVAL, "sweeps=%d must be >= 0", sweeps);
  StreamJoin join(g, stream);
  if ((rc = ensure_contrib<double>(g))) return rc;
  DevPlan &P = g->fwd;
  if ((rc = launch_init<double>(g, P, p, x, x, -1.0, std::max(1, sweeps)))) return rc;
  const int flags = flags_of(o);
  SweepArgs<double> a = make_args<double>(g, P, p, x, d, flags, nullptr);
  if (sweeps > 0) launch_sweeps(g, a, o.mode == PR_FUSED, g->weighted, sweeps, g->work);
  if (flags & kFlagScaled)
    hipLaunchKernelGGL(k_to64<double>, dim3(kInitGrid), dim3(kBlock), 0, g->work, (const double *)x, x,
                       g->n, (const SweepState *)P.st, 1);
  PR_HIP(hipGetLastError());
  if ((rc = poll_state(g, P))) return rc;
  if (resid) *resid = sweeps > 0 ? g->host_st->resid : INFINITY;
  return PR_OK;
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
  SweepArgs<double> a = make_args<double>(g, P, p, g->xtmp, d, 0, nullptr);
  launch_sweeps(g, a, false, g->weighted, 1, g->work);
  PR_HIP(hipGetLastError());
  if ((rc = poll_state(g, P))) return rc;
  *result = g->host_st->raw;
  return PR_OK;
}
