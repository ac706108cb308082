/*
 * oracle.c -- plain FP64 CPU PageRank oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or table with the GPU library.
 *
 * It computes the unique fixed point x* of
 *     x = F(x) := (1-d) p + d P x,
 * where P is column-stochastic: P[u][v] = w(v->u) / W(v) for every edge v->u,
 * W(v) = sum of v's out-weights (the out-degree when unweighted), and a
 * dangling column (W(v) = 0) is 1/n everywhere.  With p = 1/n this is the
 * paper's recurrence (Section 1, Eq. 1) with the dangling mass D spread
 * uniformly, D = sum of x over dangling vertices.
 *
 * The canonical graph follows the paper's edge-centric baseline (Section 3):
 *   - inList  : edges grouped by destination (destinations ascending), sources
 *               ascending within a destination; position e of this order is
 *               slot e of the paper's contributionList.
 *   - outList : edges grouped by source, destinations ascending.
 *   - offsetList[e_out] = contributionList slot of the same (src, dst) edge
 *               (Section 3, the offsetList/contributionList example, Fig. 1).
 * The iterations are written from the equations, not from the paper's
 * listings: they pull share_v = x_v / W_v over each inList.  The numbers they
 * add, and the order they add them in, are the ones the edge-centric layout
 * stores and sums.
 *
 * Routines (each names the passage it follows):
 *   orc_csr_count / orc_csr_build  canonical graph: self-loops dropped, repeated
 *                                  (src, dst) pairs merged, their weights summed in
 *                                  input order; offsetList.
 *   orc_jacobi        x <- F(x) (Eq. 1, per iteration Eq. 2): the fixed point's
 *                     plain definition iterated.
 *   orc_gauss_seidel  Eq. 9 in place, ascending vertex order (Seq-FusEd of
 *                     Section 6.3, the loop-fused form of Section 4); plus a
 *                     mass-scaled variant (see the function).
 *   orc_gauss_seidel_threads  the parallel loop-fused variant (Sections 4.3 and
 *                     6.3), host timing only.
 *   orc_apply_F       one application of F (certificates).
 *   orc_residual_edges ||F(x) - x||_1 from a plain edge list, no graph built
 *                     (certificates at sizes the CSR build cannot reach quickly).
 *   orc_adjoint       transposed fixed point (I - dP)^T lam = g and the
 *                     gradients dL/dp = (1-d) lam, dL/dw.
 *   orc_sample_in_lists  brute-force in-neighbour lists of chosen rows.
 *
 * The paper is silent on dangling vertices, uses the max-norm for its stop
 * rule (Eq. 3), and stops on error <= threshold.  This oracle spreads dangling
 * mass uniformly by default (LEAK mode reproduces the literal algorithms),
 * supports both L1 and max-norm residuals, and stops when residual < tol.
 *
 * A test-only mutation switch (orc_set_mutation) plants specific mistakes so
 * the tests can show that the pins catch them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

enum { ORC_NORM_L1 = 0, ORC_NORM_LINF = 1 };
enum { ORC_DANGLING_UNIFORM = 0, ORC_DANGLING_LEAK = 1 };

/* Mutations (0 = none): 1 drop the dangling term, 2 drop the teleport term,
 * 3 use in-degree instead of out-degree, 4 transpose the graph (gather over
 * out-edges), 5 wrong sign in the adjoint's normalisation term, 6 teleport
 * 1/n in place of the personalization vector p. */
static int g_mutation = 0;
void orc_set_mutation(int m) { g_mutation = m; }

#define CHUNK 4096 /* fixed reduction chunking: results do not depend on thread count */

/* ------------------------------------------------------------ CSR ----- */

typedef struct {
  int32_t s, t;
  int64_t idx;
} edge_rec;

static int cmp_dst_src(const void *a, const void *b) {
  const edge_rec *x = (const edge_rec *)a, *y = (const edge_rec *)b;
  if (x->t != y->t) return x->t < y->t ? -1 : 1;
  if (x->s != y->s) return x->s < y->s ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

static int cmp_src_dst(const void *a, const void *b) {
  const edge_rec *x = (const edge_rec *)a, *y = (const edge_rec *)b;
  if (x->s != y->s) return x->s < y->s ? -1 : 1;
  if (x->t != y->t) return x->t < y->t ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

/* Number of distinct non-self-loop edges, or -1 on a bad id / allocation failure. */
int64_t orc_csr_count(int64_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  edge_rec *r = (edge_rec *)malloc(sizeof(edge_rec) * (size_t)(m > 0 ? m : 1));
  if (!r) return -1;
  int64_t k = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(r); return -1; }
    if (src[i] == dst[i]) continue;
    r[k].s = src[i]; r[k].t = dst[i]; r[k].idx = i; ++k;
  }
  qsort(r, (size_t)k, sizeof(edge_rec), cmp_dst_src);
  int64_t u = 0;
  for (int64_t i = 0; i < k; ++i)
    if (i == 0 || r[i].s != r[i - 1].s || r[i].t != r[i - 1].t) ++u;
  free(r);
  return u;
}

/*
 * Build the canonical graph.  Output arrays are caller-allocated with the sizes
 * from orc_csr_count (mu = distinct edges):
 *   in_ptr[n+1], in_src[mu], in_w[mu] (nullable) -- inList / CL order
 *   out_ptr[n+1], out_dst[mu], out_w[mu] (nullable) -- outList order
 *   offset[mu]  -- offsetList: out position -> CL slot
 *   out_deg[n], in_deg[n]
 *   edge_map[m] (nullable) -- for each input edge, its outList position, -1 if a self-loop
 * w (nullable): input weights; repeated pairs get the sum of their weights in input order.
 */
int orc_csr_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                  int64_t *in_ptr, int32_t *in_src, double *in_w,
                  int64_t *out_ptr, int32_t *out_dst, double *out_w,
                  int64_t *offset, int32_t *out_deg, int32_t *in_deg, int64_t *edge_map) {
  edge_rec *r = (edge_rec *)malloc(sizeof(edge_rec) * (size_t)(m > 0 ? m : 1));
  if (!r) return -1;
  int64_t k = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(r); return -1; }
    if (edge_map) edge_map[i] = -1;
    if (src[i] == dst[i]) continue;
    r[k].s = src[i]; r[k].t = dst[i]; r[k].idx = i; ++k;
  }
  /* out order first: distinct (src, dst) pairs in ascending (src, dst) */
  qsort(r, (size_t)k, sizeof(edge_rec), cmp_src_dst);
  for (int64_t v = 0; v <= n; ++v) out_ptr[v] = 0;
  for (int64_t v = 0; v < n; ++v) { out_deg[v] = 0; in_deg[v] = 0; }
  int64_t mu = 0;
  for (int64_t i = 0; i < k; ++i) {
    int fresh = (i == 0 || r[i].s != r[i - 1].s || r[i].t != r[i - 1].t);
    if (fresh) {
      out_dst[mu] = r[i].t;
      if (out_w) out_w[mu] = w ? w[r[i].idx] : 1.0;
      out_deg[r[i].s]++;
      in_deg[r[i].t]++;
      ++mu;
    } else if (out_w && w) {
      out_w[mu - 1] += w[r[i].idx]; /* equal keys keep input order (idx tiebreak) */
    }
    if (edge_map) edge_map[r[i].idx] = mu - 1;
  }
  for (int64_t v = 0; v < n; ++v) out_ptr[v + 1] = out_ptr[v] + out_deg[v];
  for (int64_t v = 0; v < n; ++v) in_ptr[v + 1] = 0;
  in_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) in_ptr[v + 1] = in_ptr[v] + in_deg[v];
  /* inList / CL slots: walk out-edges in (src asc) order and drop each into its
   * destination's slice; sources then arrive ascending within every slice. */
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) { free(r); return -1; }
  for (int64_t v = 0; v < n; ++v) fill[v] = in_ptr[v];
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e) {
      int32_t t = out_dst[e];
      int64_t slot = fill[t]++;
      in_src[slot] = (int32_t)v;
      if (in_w) in_w[slot] = out_w ? out_w[e] : 1.0;
      offset[e] = slot;
    }
  }
  free(fill);
  free(r);
  return 0;
}

/* ------------------------------------------------ Eq. 1 pieces -------- */
/*
 * Notation (Section 1, Eq. 1, with the dangling reading described above):
 *   W_v      out-weight sum of v (out-degree when unweighted), summed in
 *            outList order;
 *   share_v  x_v / W_v, the rank v passes along each unit of out-weight
 *            (0 for a dangling vertex: its mass travels through D instead);
 *   D        total rank of the dangling vertices, spread as D/n everywhere;
 *   F(x)_u = (1-d) p_u + d ( sum_{v->u} w(v->u) share_v + D/n ).
 */

static void out_weight_sums(int64_t n, const int64_t *out_ptr, const double *out_w,
                            const int32_t *out_deg, double *W) {
  for (int64_t v = 0; v < n; ++v) {
    if (!out_w) { W[v] = (double)out_deg[v]; continue; }
    double s = 0.0;
    for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e) s += out_w[e];
    W[v] = s;
  }
}

/* Sum over fixed chunks, chunk partials added in order (thread-count independent). */
static double chunked_sum(int64_t n, const double *vals) {
  int64_t nc = (n + CHUNK - 1) / CHUNK;
  double *part = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
  if (!part) return NAN;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    double s = 0.0;
    int64_t hi = (c + 1) * CHUNK < n ? (c + 1) * CHUNK : n;
    for (int64_t i = c * CHUNK; i < hi; ++i) s += vals[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nc; ++c) s += part[c];
  free(part);
  return s;
}

static double dangling_total(int64_t n, const double *x, const double *W) {
  double D = 0.0;
  for (int64_t v = 0; v < n; ++v)
    if (W[v] == 0.0) D += x[v];
  return D;
}

static double plain_sum(int64_t n, const double *x) {
  double s = 0.0;
  for (int64_t v = 0; v < n; ++v) s += x[v];
  return s;
}

/* sum_{v->u} w(v->u) share_v over u's inList (sources ascending). */
static double pulled(int64_t u, const int64_t *in_ptr, const int32_t *in_src, const double *in_w,
                     const double *share) {
  double acc = 0.0;
  for (int64_t e = in_ptr[u]; e < in_ptr[u + 1]; ++e)
    acc += in_w ? share[in_src[e]] * in_w[e] : share[in_src[e]];
  return acc;
}

/* --------------------------------------------- Jacobi (Eq. 1 / Eq. 2) --- */
/*
 * The plain definition: x^{k+1} = F(x^k), every component computed from the
 * previous iterate only (the edge-centric baseline of Section 3 computes
 * exactly these numbers: the contributions it stores per edge are
 * w(v->u) share_v, and it sums each vertex's slice in inList order).  Stops
 * when the residual ||x^{k+1} - x^k|| (L1, or max-norm as Eq. 3) is below tol,
 * or after max_iter sweeps.
 *   x       start vector on entry, last iterate on exit
 *   p       personalization (nullable => 1/n)
 *   threads OpenMP threads over vertices (0 = the runtime's default); the
 *           result does not depend on it
 *   trace   (nullable, max_iter entries) residual after each sweep
 *   sums    (nullable, max_iter entries) sum of x after each sweep
 * Returns the sweeps executed (-1 on allocation failure); *res = last residual.
 */
int orc_jacobi(int64_t n, const int64_t *in_ptr, const int32_t *in_src, const double *in_w,
               const int64_t *out_ptr, const int32_t *out_dst, const double *out_w,
               const int32_t *out_deg, const int32_t *in_deg, const double *p, double d,
               double tol, int max_iter, int norm, int dangling, int threads, double *x,
               double *res, double *trace, double *sums) {
  if (threads > 0) omp_set_num_threads(threads);
  double *W = (double *)malloc(sizeof(double) * (size_t)n);
  double *share = (double *)malloc(sizeof(double) * (size_t)n);
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  double *change = (double *)malloc(sizeof(double) * (size_t)n);
  if (!W || !share || !y || !change) { free(W); free(share); free(y); free(change); return -1; }
  out_weight_sums(n, out_ptr, out_w, out_deg, W);
  if (g_mutation == 3)
    for (int64_t v = 0; v < n; ++v) W[v] = (double)in_deg[v];
  const double inv_n = 1.0 / (double)n;
  int sweeps = 0;
  double r = INFINITY;
  while (sweeps < max_iter) {
    const double D = (dangling == ORC_DANGLING_UNIFORM && g_mutation != 1) ? dangling_total(n, x, W) : 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) share[v] = W[v] != 0.0 ? x[v] / W[v] : 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; ++u) {
      double acc;
      if (g_mutation == 4) {
        /* planted mistake: the transposed operand (out-neighbours) */
        acc = 0.0;
        for (int64_t e = out_ptr[u]; e < out_ptr[u + 1]; ++e)
          acc += out_w ? share[out_dst[e]] * out_w[e] : share[out_dst[e]];
      } else {
        acc = pulled(u, in_ptr, in_src, in_w, share);
      }
      const double pu = (p && g_mutation != 6) ? p[u] : inv_n;
      const double teleport = (g_mutation == 2) ? 0.0 : (1.0 - d) * pu;
      y[u] = teleport + d * (acc + D * inv_n);
      change[u] = fabs(y[u] - x[u]);
    }
    memcpy(x, y, sizeof(double) * (size_t)n);
    ++sweeps;
    if (norm == ORC_NORM_LINF) {
      r = 0.0;
      for (int64_t u = 0; u < n; ++u) r = change[u] > r ? change[u] : r;
    } else {
      r = chunked_sum(n, change);
    }
    if (trace) trace[sweeps - 1] = r;
    if (sums) sums[sweeps - 1] = chunked_sum(n, x);
    if (r < tol) break;
  }
  *res = r;
  free(W); free(share); free(y); free(change);
  return sweeps;
}

/* ------------------------------------- Gauss-Seidel (Eq. 9, in place) --- */
/*
 * The loop-fused form of Section 4 reaches a vertex's new rank before the
 * vertices after it are pulled, so u reads x^{k+1}_v for in-neighbours v < u
 * and x^k_v for v >= u (Eq. 9), vertices taken in ascending id (Seq-FusEd).
 * Here x and share are overwritten in place, which is that recurrence.
 *
 * scaled = 0: the dangling total is recomputed at the start of each sweep and
 *   kept current as dangling vertices change (Gauss-Seidel on the full
 *   column-stochastic matrix).
 * scaled = 1: mass-scaled variant.  A Gauss-Seidel sweep does not conserve
 *   sum(x), and that drift is its slowest error mode.  Here D and the total
 *   mass S are the previous sweep's and the teleport term is scaled by S:
 *   x_u <- (1-d) p_u S + d (pulled + D/n).  Dividing the iterates by S turns
 *   this into Gauss-Seidel followed by renormalisation to sum 1 (the fixed
 *   point's sum when p sums to 1), so the fixed point is unchanged.  The
 *   residual is (||x' - x||_1 + |S' - S|) / S, a bound on the step of the
 *   normalised iterates, and x is normalised on exit.  Needs uniform dangling
 *   and the L1 norm.
 */
int orc_gauss_seidel(int64_t n, const int64_t *in_ptr, const int32_t *in_src, const double *in_w,
                     const int64_t *out_ptr, const double *out_w, const int32_t *out_deg,
                     const double *p, double d, double tol, int max_iter, int norm, int dangling,
                     int scaled, double *x, double *res, double *trace) {
  const int uniform = (dangling == ORC_DANGLING_UNIFORM);
  if (scaled && (!uniform || norm != ORC_NORM_L1)) return -2;
  double *W = (double *)malloc(sizeof(double) * (size_t)n);
  double *share = (double *)malloc(sizeof(double) * (size_t)n);
  if (!W || !share) { free(W); free(share); return -1; }
  out_weight_sums(n, out_ptr, out_w, out_deg, W);
  for (int64_t v = 0; v < n; ++v) share[v] = W[v] != 0.0 ? x[v] / W[v] : 0.0;
  const double inv_n = 1.0 / (double)n;
  int sweeps = 0;
  double r = INFINITY;
  while (sweeps < max_iter) {
    double D = uniform ? dangling_total(n, x, W) : 0.0;
    const double S = scaled ? plain_sum(n, x) : 1.0;
    double l1 = 0.0, linf = 0.0;
    for (int64_t u = 0; u < n; ++u) {
      const double acc = pulled(u, in_ptr, in_src, in_w, share);
      const double pu = p ? p[u] : inv_n;
      const double xn = (1.0 - d) * pu * S + d * (acc + D * inv_n);
      const double step = fabs(xn - x[u]);
      if (W[u] == 0.0) {
        if (uniform && !scaled) D += xn - x[u];
      } else {
        share[u] = xn / W[u];
      }
      x[u] = xn;
      l1 += step;
      if (step > linf) linf = step;
    }
    ++sweeps;
    r = scaled ? (l1 + fabs(plain_sum(n, x) - S)) / S : (norm == ORC_NORM_LINF ? linf : l1);
    if (trace) trace[sweeps - 1] = r;
    if (r < tol) break;
  }
  if (scaled) {
    const double S = plain_sum(n, x);
    for (int64_t v = 0; v < n; ++v) x[v] /= S;
  }
  *res = r;
  free(W); free(share);
  return sweeps;
}

/*
 * Par-FusEd: the paper's parallel loop-fused variant (Sections 4.3 and 6.3),
 * for host timing only (never a parity reference).  The vertices are split
 * statically over `threads` OpenMP threads; each thread applies Eq. 9 to its
 * own range in ascending order, in place on the shared share[] array, so it
 * reads whatever value another thread last stored (relaxed atomic loads and
 * stores: a value is old or new, never torn).  D is the one at the start of
 * each sweep; `scaled` selects the mass-scaled form described above.  With one
 * thread and scaled = 1 it computes what orc_gauss_seidel computes with
 * scaled = 1.  L1 residual only.
 */
int orc_gauss_seidel_threads(int64_t n, const int64_t *in_ptr, const int32_t *in_src,
                             const double *in_w, const int64_t *out_ptr, const double *out_w,
                             const int32_t *out_deg, const double *p, double d, double tol,
                             int max_iter, int dangling, int scaled, int threads, double *x,
                             double *res) {
  const int uniform = (dangling == ORC_DANGLING_UNIFORM);
  if (scaled && !uniform) return -2;
  double *W = (double *)malloc(sizeof(double) * (size_t)n);
  double *share = (double *)malloc(sizeof(double) * (size_t)n);
  if (!W || !share) { free(W); free(share); return -1; }
  out_weight_sums(n, out_ptr, out_w, out_deg, W);
  for (int64_t v = 0; v < n; ++v) share[v] = W[v] != 0.0 ? x[v] / W[v] : 0.0;
  const double inv_n = 1.0 / (double)n;
  int sweeps = 0;
  double r = INFINITY;
  while (sweeps < max_iter) {
    const double D = uniform ? dangling_total(n, x, W) : 0.0;
    const double S = scaled ? plain_sum(n, x) : 1.0;
    double l1 = 0.0;
#pragma omp parallel for schedule(static) num_threads(threads) reduction(+ : l1)
    for (int64_t u = 0; u < n; ++u) {
      double acc = 0.0;
      for (int64_t e = in_ptr[u]; e < in_ptr[u + 1]; ++e) {
        double s;
        __atomic_load(&share[in_src[e]], &s, __ATOMIC_RELAXED);
        acc += in_w ? s * in_w[e] : s;
      }
      const double pu = p ? p[u] : inv_n;
      const double xn = (1.0 - d) * pu * S + d * (acc + D * inv_n);
      if (W[u] != 0.0) {
        const double s = xn / W[u];
        __atomic_store(&share[u], &s, __ATOMIC_RELAXED);
      }
      l1 += fabs(xn - x[u]);
      x[u] = xn;
    }
    ++sweeps;
    r = scaled ? (l1 + fabs(plain_sum(n, x) - S)) / S : l1;
    if (r < tol) break;
  }
  if (scaled) {
    const double S = plain_sum(n, x);
    for (int64_t v = 0; v < n; ++v) x[v] /= S;
  }
  *res = r;
  free(W); free(share);
  return sweeps;
}

/* ------------------------------------------------ F and certificates --- */
/* y = F(x) over the inList (sources of each destination), FP64. */
int orc_apply_F(int64_t n, const int64_t *in_ptr, const int32_t *in_src, const double *in_w,
                const int64_t *out_ptr, const double *out_w, const int32_t *out_deg,
                const double *p, double d, int dangling, const double *x, double *y) {
  double *W = (double *)malloc(sizeof(double) * (size_t)n);
  if (!W) return -1;
  out_weight_sums(n, out_ptr, out_w, out_deg, W);
  const double D = (dangling == ORC_DANGLING_UNIFORM) ? dangling_total(n, x, W) : 0.0;
  const double inv_n = 1.0 / (double)n;
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < n; ++u) {
    double acc = 0.0;
    for (int64_t e = in_ptr[u]; e < in_ptr[u + 1]; ++e) {
      int32_t v = in_src[e];
      acc += (in_w ? in_w[e] : 1.0) * (x[v] / W[v]);
    }
    const double pu = p ? p[u] : inv_n;
    y[u] = (1.0 - d) * pu + d * (acc + D * inv_n);
  }
  free(W);
  return 0;
}

/*
 * ||F(x) - x||_1 straight from an edge list, without building any graph
 * structure: W_v is summed over the listed edges leaving v (their weights, or
 * 1 each), D over the vertices whose W_v is 0, and
 *     F(x)_u = (1-d) p_u + d ( sum over listed edges v->u of w x_v / W_v + D/n ).
 * Self-loops are skipped, as the canonical graph drops them.  A repeated
 * (src, dst) pair would be counted twice, so the list must hold each edge
 * once; a list that does not gives a value for a different graph, which makes
 * a comparison with the canonical graph's fixed point fail, never pass.
 * For every x, ||x - x*||_1 <= this / (1 - d) (F is a d-contraction in L1).
 *   w      edge weights (nullable: 1)
 *   p      personalization (nullable: 1/n)
 *   y      (nullable) receives F(x)
 *   threads edge-range partitions, each summing into its own array; the arrays
 *          are added in partition order, so the result depends only on
 *          `threads` (1 = one plain sequential pass)
 * Returns the residual, or NaN on allocation failure.
 */
double orc_residual_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          const double *w, const double *p, double d, const double *x,
                          double *y, int threads) {
  const int T = threads > 0 ? threads : 1;
  double *W = (double *)calloc((size_t)n, sizeof(double));
  double *acc = (double *)calloc((size_t)n * (size_t)T, sizeof(double));
  if (!W || !acc) { free(W); free(acc); return NAN; }
  const int transposed = (g_mutation == 4);
  for (int64_t i = 0; i < m; ++i) {
    const int32_t a = src[i], b = dst[i];
    if (a == b) continue;
    /* planted mistake 3: in-weight in place of out-weight */
    W[g_mutation == 3 ? b : a] += w ? w[i] : 1.0;
  }
  const double D = (g_mutation == 1) ? 0.0 : dangling_total(n, x, W);
#pragma omp parallel for schedule(static) num_threads(T)
  for (int t = 0; t < T; ++t) {
    double *mine = acc + (size_t)t * (size_t)n;
    const int64_t lo = m * t / T, hi = m * (t + 1) / T;
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t a = transposed ? dst[i] : src[i], b = transposed ? src[i] : dst[i];
      if (a == b || W[a] == 0.0) continue;
      mine[b] += (w ? w[i] : 1.0) * (x[a] / W[a]);
    }
  }
  const double inv_n = 1.0 / (double)n;
  double r = 0.0;
  for (int64_t u = 0; u < n; ++u) {
    double s = acc[u];
    for (int t = 1; t < T; ++t) s += acc[(size_t)t * (size_t)n + (size_t)u];
    const double pu = (p && g_mutation != 6) ? p[u] : inv_n;
    const double teleport = (g_mutation == 2) ? 0.0 : (1.0 - d) * pu;
    const double fu = teleport + d * (s + D * inv_n);
    if (y) y[u] = fu;
    r += fabs(fu - x[u]);
  }
  free(W); free(acc);
  return r;
}

/* ------------------------------------------------ adjoint ------------- */
/*
 * Transposed fixed point: lam = g + d P^T lam, where
 *   (P^T lam)_v = sum_{v->u} (w/W_v) lam_u      if W_v > 0
 *               = (sum_u lam_u) / n              if v is dangling.
 * Iterated (Jacobi) until max |lam' - lam| < tol.  Then, for L with dL/dx = g:
 *   dL/dp_u = (1-d) lam_u
 *   dL/dw(v->u) = d * x_v / W_v * (lam_u - (P^T lam)_v)   (outList order)
 * from dP[i][v]/dw(v->u) = [i = u]/W_v - w(v->i)/W_v^2.
 * Returns sweeps executed (or -1).
 */
int orc_adjoint(int64_t n, const int64_t *out_ptr, const int32_t *out_dst, const double *out_w,
                const int32_t *out_deg, const double *x, const double *g, double d, double tol,
                int max_iter, double *lam, double *grad_p, double *grad_w, double *res) {
  double *W = (double *)malloc(sizeof(double) * (size_t)n);
  double *nl = (double *)malloc(sizeof(double) * (size_t)n);
  double *ptl = (double *)malloc(sizeof(double) * (size_t)n);
  if (!W || !nl || !ptl) { free(W); free(nl); free(ptl); return -1; }
  out_weight_sums(n, out_ptr, out_w, out_deg, W);
  const double inv_n = 1.0 / (double)n;
  for (int64_t v = 0; v < n; ++v) lam[v] = g[v];
  int it = 0;
  double r = INFINITY;
  while (it < max_iter) {
    double S = chunked_sum(n, lam);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      double t;
      if (W[v] == 0.0) {
        t = S * inv_n;
      } else {
        double s = 0.0;
        for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e)
          s += (out_w ? out_w[e] : 1.0) * lam[out_dst[e]];
        t = s / W[v];
      }
      nl[v] = g[v] + d * t;
    }
    r = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      double dl = fabs(nl[v] - lam[v]);
      if (dl > r) r = dl;
      lam[v] = nl[v];
    }
    ++it;
    if (r < tol) break;
  }
  *res = r;
  for (int64_t v = 0; v < n; ++v) grad_p[v] = (1.0 - d) * lam[v];
  /* (P^T lam)_v over real out-edges, then per-edge gradient */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    if (W[v] == 0.0) { ptl[v] = 0.0; continue; }
    double s = 0.0;
    for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e)
      s += (out_w ? out_w[e] : 1.0) * lam[out_dst[e]];
    ptl[v] = s / W[v];
    double scale = d * x[v] / W[v];
    for (int64_t e = out_ptr[v]; e < out_ptr[v + 1]; ++e) {
      double corr = (g_mutation == 5) ? -ptl[v] : ptl[v];
      grad_w[e] = scale * (lam[out_dst[e]] - corr);
    }
  }
  free(W); free(nl); free(ptl);
  return it;
}

/* Brute-force in-neighbour lists of sampled rows straight from a raw edge list
 * (self-loops dropped, repeats merged), for spot checks on graphs too large for
 * orc_csr_build.  rows must be distinct; out_cnt[i] = distinct sources of rows[i];
 * out_src is filled row by row (ascending sources) up to cap entries in total.
 * Returns the total number of entries, or -1. */
int64_t orc_sample_in_lists(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            int64_t k, const int32_t *rows, int64_t cap, int64_t *out_cnt,
                            int32_t *out_src) {
  int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!slot) return -1;
  for (int64_t v = 0; v < n; ++v) slot[v] = -1;
  for (int64_t i = 0; i < k; ++i) slot[rows[i]] = (int32_t)i;
  /* collect (row slot, src) pairs */
  int64_t cnt = 0, alloc = 1024;
  edge_rec *acc = (edge_rec *)malloc(sizeof(edge_rec) * (size_t)alloc);
  if (!acc) { free(slot); return -1; }
  for (int64_t e = 0; e < m; ++e) {
    int32_t t = dst[e];
    if (t < 0 || t >= n || slot[t] < 0 || src[e] == t) continue;
    if (cnt == alloc) {
      alloc *= 2;
      edge_rec *na = (edge_rec *)realloc(acc, sizeof(edge_rec) * (size_t)alloc);
      if (!na) { free(acc); free(slot); return -1; }
      acc = na;
    }
    acc[cnt].t = slot[t]; acc[cnt].s = src[e]; acc[cnt].idx = e; ++cnt;
  }
  qsort(acc, (size_t)cnt, sizeof(edge_rec), cmp_dst_src);
  for (int64_t i = 0; i < k; ++i) out_cnt[i] = 0;
  int64_t total = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    if (i > 0 && acc[i].t == acc[i - 1].t && acc[i].s == acc[i - 1].s) continue;
    out_cnt[acc[i].t]++;
    if (total < cap) out_src[total] = acc[i].s;
    ++total;
  }
  free(acc); free(slot);
  return total;
}
