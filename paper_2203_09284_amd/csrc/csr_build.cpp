// Canonical CSR construction on the host (pr_build_csr).
//
// The stored graph follows the paper's edge-centric layout (Section 3): an
// in-edge list per destination (the contributionList order), an out-edge
// list per source, and the offsetList that maps each out-edge to the slot of
// the same edge in the in-edge order.  Self-loops are dropped; repeated
// (src, dst) pairs become one edge whose weight is the sum of the repeats in
// input order.
//
// Method: counting sort of the input edges by source (stable, so each source
// bucket keeps input order), a per-bucket sort by (destination, input
// position) in parallel, a merge of equal destinations, then a stable
// counting sort of the out-edges by destination, which leaves the sources of
// every destination ascending.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

unsigned worker_count() {
  unsigned hw = std::thread::hardware_concurrency();
  if (hw == 0) hw = 4;
  if (hw > 64) hw = 64;
  return hw;
}

// Dynamic parallel loop over [0, count) in chunks.
template <typename F>
void parallel_chunks(int64_t count, int64_t chunk, F fn) {
  std::atomic<int64_t> next{0};
  unsigned nt = worker_count();
  if (count <= chunk) nt = 1;
  auto body = [&]() {
    for (;;) {
      int64_t b = next.fetch_add(chunk);
      if (b >= count) break;
      int64_t e = std::min(count, b + chunk);
      fn(b, e);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(body);
  body();
  for (auto &t : th) t.join();
}

template <typename T>
T *xalloc(size_t count) {
  return static_cast<T *>(malloc(sizeof(T) * (count > 0 ? count : 1)));
}

}  // namespace

extern "C" void pr_csr_free(pr_csr *c) {
  if (!c) return;
  free(c->in_ptr);
  free(c->in_src);
  free(c->in_w);
  free(c->out_ptr);
  free(c->out_dst);
  free(c->out_w);
  free(c->out_to_in);
  free(c->out_deg);
  free(c->in_deg);
  free(c->edge_map);
  memset(c, 0, sizeof(*c));
}

extern "C" int pr_build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const double *w, pr_csr *out) {
  pr_clear_error();
  if (!out) return pr_fail(PR_EINVAL, "pr_build_csr: out is NULL");
  memset(out, 0, sizeof(*out));
  if (n < 1 || n > INT32_MAX) return pr_fail(PR_EINVAL, "pr_build_csr: n=%lld out of range", (long long)n);
  if (m < 0 || m > (int64_t)UINT32_MAX - 2)
    return pr_fail(PR_EINVAL, "pr_build_csr: m=%lld out of range", (long long)m);
  if (m > 0 && (!src || !dst)) return pr_fail(PR_EINVAL, "pr_build_csr: NULL edge arrays");

  // validate ids and weights
  std::atomic<int64_t> bad{-1};
  parallel_chunks(m, 1 << 20, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      bool ok = src[i] >= 0 && src[i] < n && dst[i] >= 0 && dst[i] < n;
      if (ok && w) ok = isfinite(w[i]) && w[i] > 0.0;
      if (!ok) {
        bad.store(i);
        return;
      }
    }
  });
  if (bad.load() >= 0) {
    int64_t i = bad.load();
    if (w && !(isfinite(w[i]) && w[i] > 0.0))
      return pr_fail(PR_EINVAL, "pr_build_csr: weight %lld is not finite and positive", (long long)i);
    return pr_fail(PR_EINVAL, "pr_build_csr: edge %lld has an endpoint outside [0, %lld)",
                   (long long)i, (long long)n);
  }

  // 1. stable counting sort of non-self-loop edges by source
  std::vector<int64_t> bucket(n + 1, 0);
  for (int64_t i = 0; i < m; ++i)
    if (src[i] != dst[i]) bucket[src[i] + 1]++;
  for (int64_t v = 0; v < n; ++v) bucket[v + 1] += bucket[v];
  const int64_t k = bucket[n];
  struct Rec {
    int32_t dst;
    int64_t idx;
  };
  Rec *rec = xalloc<Rec>(k);
  int64_t *fill = xalloc<int64_t>(n);
  if (!rec || !fill) {
    free(rec);
    free(fill);
    return pr_fail(PR_ENOMEM, "pr_build_csr: out of host memory");
  }
  memcpy(fill, bucket.data(), sizeof(int64_t) * n);
  for (int64_t i = 0; i < m; ++i)
    if (src[i] != dst[i]) rec[fill[src[i]]++] = Rec{dst[i], i};
  free(fill);

  // 2. sort every source bucket by (dst, input position); count distinct dsts
  int32_t *out_deg = xalloc<int32_t>(n);
  if (!out_deg) {
    free(rec);
    return pr_fail(PR_ENOMEM, "pr_build_csr: out of host memory");
  }
  parallel_chunks(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      Rec *lo = rec + bucket[v], *hi = rec + bucket[v + 1];
      std::sort(lo, hi, [](const Rec &a, const Rec &c) {
        return a.dst != c.dst ? a.dst < c.dst : a.idx < c.idx;
      });
      int32_t cnt = 0;
      for (Rec *r = lo; r < hi; ++r)
        if (r == lo || r->dst != r[-1].dst) ++cnt;
      out_deg[v] = cnt;
    }
  });

  // 3. out-CSR with merged repeats
  int64_t *out_ptr = xalloc<int64_t>(n + 1);
  if (!out_ptr) {
    free(rec);
    free(out_deg);
    return pr_fail(PR_ENOMEM, "pr_build_csr: out of host memory");
  }
  out_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) out_ptr[v + 1] = out_ptr[v] + out_deg[v];
  const int64_t mu = out_ptr[n];
  int32_t *out_dst = xalloc<int32_t>(mu);
  double *out_w = w ? xalloc<double>(mu) : nullptr;
  int64_t *edge_map = xalloc<int64_t>(m);
  int32_t *in_deg = xalloc<int32_t>(n);
  int64_t *in_ptr = xalloc<int64_t>(n + 1);
  int32_t *in_src = xalloc<int32_t>(mu);
  double *in_w = w ? xalloc<double>(mu) : nullptr;
  int64_t *out_to_in = xalloc<int64_t>(mu);
  if (!out_dst || (w && !out_w) || !edge_map || !in_deg || !in_ptr || !in_src || (w && !in_w) ||
      !out_to_in) {
    free(rec);
    free(out_deg);
    free(out_ptr);
    free(out_dst);
    free(out_w);
    free(edge_map);
    free(in_deg);
    free(in_ptr);
    free(in_src);
    free(in_w);
    free(out_to_in);
    return pr_fail(PR_ENOMEM, "pr_build_csr: out of host memory");
  }
  parallel_chunks(m, 1 << 20, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) edge_map[i] = -1;
  });
  parallel_chunks(n, 4096, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int64_t o = out_ptr[v] - 1;
      for (int64_t r = bucket[v]; r < bucket[v + 1]; ++r) {
        if (r == bucket[v] || rec[r].dst != rec[r - 1].dst) {
          ++o;
          out_dst[o] = rec[r].dst;
          if (out_w) out_w[o] = w[rec[r].idx];
        } else if (out_w) {
          out_w[o] += w[rec[r].idx];
        }
        edge_map[rec[r].idx] = o;
      }
    }
  });
  free(rec);

  // 4. in-CSR: stable counting sort of out-edges by destination
  memset(in_deg, 0, sizeof(int32_t) * n);
  for (int64_t e = 0; e < mu; ++e) in_deg[out_dst[e]]++;
  in_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) in_ptr[v + 1] = in_ptr[v] + in_deg[v];
  int64_t *slot = xalloc<int64_t>(n);
  if (!slot) {
    out->n = n;
    pr_csr tmp{n, mu, in_ptr, in_src, in_w, out_ptr, out_dst, out_w, out_to_in, out_deg, in_deg, m, edge_map};
    pr_csr_free(&tmp);
    return pr_fail(PR_ENOMEM, "pr_build_csr: out of host memory");
  }
  memcpy(slot, in_ptr, sizeof(int64_t) * n);
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e) {
      int64_t s = slot[out_dst[e]]++;
      in_src[s] = (int32_t)v;
      if (in_w) in_w[s] = out_w[e];
      out_to_in[e] = s;
    }
  }
  free(slot);

  out->n = n;
  out->m = mu;
  out->in_ptr = in_ptr;
  out->in_src = in_src;
  out->in_w = in_w;
  out->out_ptr = out_ptr;
  out->out_dst = out_dst;
  out->out_w = out_w;
  out->out_to_in = out_to_in;
  out->out_deg = out_deg;
  out->in_deg = in_deg;
  out->m_input = m;
  out->edge_map = edge_map;
  return PR_OK;
}
