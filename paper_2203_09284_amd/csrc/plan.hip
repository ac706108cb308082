// Device graph and execution plan (pr_graph_create).
//
// The plan bins vertices by the length of the list they pull over (in-degree
// for the forward pull, out-degree for the transposed pull of the adjoint):
//   light  (<= light_max):  thread per vertex; up to 256 consecutive light
//                           vertices form one block whose edges (<= block_edges)
//                           are gathered edge-parallel into LDS first
//   medium (<= medium_max): wavefront per vertex; groups of rows per workgroup
//   heavy  (>  medium_max): workgroup per chunk of `split` edges; the last
//                           chunk to finish combines the partial sums in order
// The neighbour lists are copied in bin order (heavy, medium, light; vertex
// ids ascending inside a bin) so every work item reads one contiguous range.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace fpr;

extern "C" void pr_plan_opts_default(pr_plan_opts *o) {
  if (!o) return;
  o->light_max = 32;
  o->medium_max = 2048;
  o->split = 8192;
  o->block_edges = kLightCap;
  o->with_adjoint = 0;
}

int fpr_dev_alloc(pr_graph *g, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return pr_fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EDEVICE, "hipMalloc(%zu): %s", bytes,
                   hipGetErrorString(e));
  }
  g->owned.push_back(*p);
  g->device_bytes += (int64_t)bytes;
  return PR_OK;
}

template <typename T>
static int upload(pr_graph *g, T **dst, const T *src, size_t count) {
  int rc = fpr_dev_alloc(g, (void **)dst, sizeof(T) * count);
  if (rc) return rc;
  if (count) PR_HIP(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return PR_OK;
}

// Build one binned pull plan from a CSR (ptr[n+1], nbr[m], w[m] nullable).
static int build_plan(pr_graph *g, DevPlan &P, int64_t n, const int64_t *ptr, const int32_t *nbr,
                      const double *w, const pr_plan_opts &o) {
  P.n = n;
  P.m = ptr[n];
  P.split = o.split;
  std::vector<uint32_t> heavy, medium, light;
  for (int64_t v = 0; v < n; ++v) {
    int64_t L = ptr[v + 1] - ptr[v];
    if (L <= o.light_max) light.push_back((uint32_t)v);
    else if (L <= o.medium_max) medium.push_back((uint32_t)v);
    else heavy.push_back((uint32_t)v);
  }
  std::vector<uint32_t> rows;
  rows.reserve(n);
  rows.insert(rows.end(), heavy.begin(), heavy.end());
  rows.insert(rows.end(), medium.begin(), medium.end());
  rows.insert(rows.end(), light.begin(), light.end());
  std::vector<uint32_t> rptr(n + 1);
  rptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t v = rows[i];
    rptr[i + 1] = rptr[i] + (uint32_t)(ptr[v + 1] - ptr[v]);
  }
  const int64_t m = P.m;
  std::vector<int32_t> idx(m);
  std::vector<double> wv(w ? m : 0);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t v = rows[i];
    int64_t L = ptr[v + 1] - ptr[v];
    memcpy(&idx[rptr[i]], nbr + ptr[v], sizeof(int32_t) * L);
    if (w) memcpy(&wv[rptr[i]], w + ptr[v], sizeof(double) * L);
  }

  // work items, in ticket order: heavy chunks, medium groups, light blocks
  std::vector<int4> items;
  std::vector<uint32_t> hbase;
  int64_t i = 0, chunks = 0;
  for (size_t h = 0; h < heavy.size(); ++h, ++i) {
    int64_t L = rptr[i + 1] - rptr[i];
    int64_t nch = (L + o.split - 1) / o.split;
    hbase.push_back((uint32_t)chunks);
    for (int64_t c = 0; c < nch; ++c) items.push_back(make_int4(kHeavy, (int)i, (int)c, (int)h));
    chunks += nch;
    P.e_heavy += L;
  }
  const int64_t med_end = i + (int64_t)medium.size();
  while (i < med_end) {
    int64_t i0 = i, edges = 0;
    while (i < med_end && i - i0 < 64 && edges < 8192) {
      edges += rptr[i + 1] - rptr[i];
      ++i;
    }
    items.push_back(make_int4(kMedium, (int)i0, (int)i, 0));
    P.e_medium += edges;
  }
  while (i < n) {
    int64_t i0 = i, edges = 0;
    while (i < n && i - i0 < kBlock) {
      int64_t L = rptr[i + 1] - rptr[i];
      if (edges + L > o.block_edges) break;
      edges += L;
      ++i;
    }
    items.push_back(make_int4(kLight, (int)i0, (int)i, 0));
    P.e_light += edges;
  }
  P.n_light = (int64_t)light.size();
  P.n_medium = (int64_t)medium.size();
  P.n_heavy_rows = (int64_t)heavy.size();
  P.n_items = (int)items.size();
  P.n_heavy = (int)heavy.size();
  P.n_chunks = (int)chunks;

  int64_t before = g->device_bytes;
  int rc;
  if ((rc = upload(g, &P.rows, rows.data(), rows.size()))) return rc;
  if ((rc = upload(g, &P.rptr, rptr.data(), rptr.size()))) return rc;
  if ((rc = upload(g, &P.idx, idx.data(), idx.size()))) return rc;
  if (w && (rc = upload(g, &P.w, wv.data(), wv.size()))) return rc;
  if ((rc = upload(g, &P.items, items.data(), items.size()))) return rc;
  if ((rc = upload(g, &P.hbase, hbase.data(), hbase.size()))) return rc;
  if ((rc = fpr_dev_alloc(g, (void **)&P.hpart, sizeof(double) * (chunks > 0 ? chunks : 1)))) return rc;
  if ((rc = fpr_dev_alloc(g, (void **)&P.hcnt, sizeof(unsigned) * (P.n_heavy > 0 ? P.n_heavy : 1))))
    return rc;
  PR_HIP(hipMemset(P.hcnt, 0, sizeof(unsigned) * (P.n_heavy > 0 ? P.n_heavy : 1)));
  if ((rc = fpr_dev_alloc(g, (void **)&P.item_part, sizeof(double) * 3 * (P.n_items > 0 ? P.n_items : 1))))
    return rc;
  if ((rc = fpr_dev_alloc(g, (void **)&P.st, sizeof(SweepState)))) return rc;
  PR_HIP(hipMemset(P.st, 0, sizeof(SweepState)));
  P.bytes = g->device_bytes - before;
  return PR_OK;
}

static void destroy(pr_graph *g) {
  if (!g) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  if (g->work) (void)hipStreamSynchronize(g->work);
  for (void *p : g->owned) (void)hipFree(p);
  g->owned.clear();
  if (g->host_st) (void)hipHostFree(g->host_st);
  if (g->bhost) (void)hipHostFree(g->bhost);
  if (g->ev_in) (void)hipEventDestroy(g->ev_in);
  if (g->ev_out) (void)hipEventDestroy(g->ev_out);
  if (g->work) (void)hipStreamDestroy(g->work);
  (void)hipSetDevice(cur);
  delete g;
}

extern "C" void pr_graph_destroy(pr_graph *g) { destroy(g); }

extern "C" int pr_graph_create(const pr_csr *csr, const pr_plan_opts *opts, pr_graph **out) {
  pr_clear_error();
  if (!out) return pr_fail(PR_EINVAL, "pr_graph_create: out is NULL");
  *out = nullptr;
  if (!csr || !csr->in_ptr || !csr->out_ptr || !csr->out_deg || csr->n < 1)
    return pr_fail(PR_EINVAL, "pr_graph_create: csr is not a pr_build_csr result");
  if (csr->m > (int64_t)UINT32_MAX - 2)
    return pr_fail(PR_EINVAL, "pr_graph_create: %lld edges exceed the per-graph limit",
                   (long long)csr->m);
  pr_plan_opts o;
  pr_plan_opts_default(&o);
  if (opts) o = *opts;
  if (o.block_edges < 1 || o.block_edges > kLightCap || o.light_max < 0 ||
      o.light_max > o.block_edges || o.medium_max <= o.light_max || o.split < kBlock)
    return pr_fail(PR_EINVAL,
                   "pr_graph_create: need 0 <= light_max <= block_edges <= %d, medium_max > "
                   "light_max, split >= %d",
                   kLightCap, kBlock);
  int dev_count = 0;
  hipError_t he = hipGetDeviceCount(&dev_count);
  if (he != hipSuccess || dev_count < 1)
    return pr_fail(PR_EDEVICE, "pr_graph_create: no HIP device (%s)", hipGetErrorString(he));

  pr_graph *g = new pr_graph();
  g->popts = o;
  g->n = csr->n;
  g->m = csr->m;
  g->weighted = csr->in_w != nullptr;
  int rc = PR_OK;
  hipDeviceProp_t prop;
  if (hipGetDevice(&g->device) != hipSuccess || hipGetDeviceProperties(&prop, g->device) != hipSuccess) {
    destroy(g);
    return pr_fail(PR_EDEVICE, "pr_graph_create: cannot query the current device");
  }
  g->n_cu = prop.multiProcessorCount;

  rc = [&]() -> int {
  // 1 / W_v, W_v summed over out-edges in out order
  const int64_t n = g->n;
  int rc2;
  std::vector<double> inv_w(n);
  for (int64_t v = 0; v < n; ++v) {
    double W;
    if (csr->out_w) {
      W = 0.0;
      for (int64_t e = csr->out_ptr[v]; e < csr->out_ptr[v + 1]; ++e) W += csr->out_w[e];
    } else {
      W = (double)csr->out_deg[v];
    }
    inv_w[v] = W > 0.0 ? 1.0 / W : 0.0;
    if (W == 0.0) g->n_dangling++;
  }
  if ((rc2 = upload(g, &g->inv_w, inv_w.data(), inv_w.size()))) return rc2;
  if ((rc2 = build_plan(g, g->fwd, n, csr->in_ptr, csr->in_src, csr->in_w, o))) return rc2;
  if (o.with_adjoint) {
    if ((rc2 = build_plan(g, g->adj, n, csr->out_ptr, csr->out_dst, csr->out_w, o))) return rc2;
    std::vector<uint32_t> op(n + 1);
    for (int64_t v = 0; v <= n; ++v) op[v] = (uint32_t)csr->out_ptr[v];
    if ((rc2 = upload(g, &g->out_ptr, op.data(), op.size()))) return rc2;
    g->has_adj = true;
  }
  if (hipStreamCreateWithFlags(&g->work, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void **)&g->host_st, sizeof(SweepState)) != hipSuccess)
    return pr_fail(PR_EDEVICE, "pr_graph_create: stream/event/pinned allocation failed");
  if ((rc2 = fpr_dev_alloc(g, (void **)&g->red_tmp, sizeof(double) * 4096))) return rc2;
  g->grid = fpr_grid_for(g);
  return PR_OK;
  }();
  if (rc != PR_OK) {
    destroy(g);
    return rc;
  }
  *out = g;
  return PR_OK;
}

extern "C" int pr_graph_stats_get(const pr_graph *g, pr_graph_stats *s) {
  pr_clear_error();
  if (!g || !s) return pr_fail(PR_EINVAL, "pr_graph_stats_get: NULL argument");
  memset(s, 0, sizeof(*s));
  s->n = g->n;
  s->m = g->m;
  s->n_light = g->fwd.n_light;
  s->n_medium = g->fwd.n_medium;
  s->n_heavy = g->fwd.n_heavy_rows;
  s->e_light = g->fwd.e_light;
  s->e_medium = g->fwd.e_medium;
  s->e_heavy = g->fwd.e_heavy;
  s->n_items = g->fwd.n_items;
  s->n_dangling = g->n_dangling;
  s->device_bytes = g->device_bytes;
  s->grid = g->grid;
  return PR_OK;
}
