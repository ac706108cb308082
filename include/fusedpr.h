/*
 * fusedpr.h -- C ABI of the MI355X (gfx950) PageRank library.
 *
 * The library computes the PageRank vector of a directed graph: the fixed
 * point of the paper's recurrence (Section 1, Eq. 1; restated per iteration
 * as Eq. 2)
 *
 *     x_u = (1-d) p_u + d * ( sum_{v -> u} w(v->u) x_v / W_v  +  D / n )
 *
 * with W_v the out-weight sum of v (its out-degree when unweighted), D the
 * total rank of dangling vertices (W_v = 0), spread uniformly, and p the
 * teleport vector (1/n everywhere unless given).  It is reached either by the
 * edge-centric Jacobi pull (Section 3, Algorithm 1) or by the loop-fused
 * Gauss-Seidel-like sweep (Section 4, Algorithm 2; Eq. 9), here over blocks
 * of vertices: each block reads the contributions that earlier blocks wrote
 * in the same sweep (see pr_plan_opts.gs_blocks).
 *
 * Conventions shared by every entry point:
 *   - Return value: PR_OK (0) on success, PR_NOT_CONVERGED (1) when an
 *     iteration stopped at max_iter (outputs are valid), a negative PR_E*
 *     code on error.  No entry point aborts or exits; the message of the last
 *     error on the calling thread is returned by pr_last_error().
 *   - Arguments are validated before any GPU work is queued; an invalid
 *     argument returns PR_EINVAL and leaves outputs untouched.
 *   - Pointers documented as "device" must be device memory of the current
 *     HIP device (e.g. from PyTorch); "host" pointers are ordinary memory.
 *     Input pointers are borrowed for the duration of the call only.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Entry
 *     points that return host-side results (iteration counts, residuals)
 *     synchronise that stream before returning; device outputs are complete
 *     when they return.
 *   - Vertex ids are int32 in [0, n); edge counts up to 2^32 - 2 per graph.
 *   - Calls on one pr_graph must not overlap (each graph owns its workspace);
 *     distinct graphs may be used from distinct threads.
 */
#ifndef FUSEDPR_H
#define FUSEDPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pr_status {
  PR_OK = 0,
  PR_NOT_CONVERGED = 1,
  PR_EINVAL = -1,
  PR_ENOMEM = -2,
  PR_EDEVICE = -3
};

/* Message of the most recent error on this thread ("" if none).  The string
 * stays valid until the next library call on the same thread. */
const char *pr_last_error(void);

/* ------------------------------------------------------------------------
 * Canonical graph on the host.
 *
 * The paper keeps per-vertex in- and out-adjacency (inList / outList) and an
 * offsetList mapping each out-edge to the contributionList slot of the same
 * edge (Section 3, the example of Fig. 1).  pr_build_csr produces that layout
 * in compressed form:
 *   in_ptr[n+1], in_src[m], in_w[m]   in-edges grouped by destination
 *                                     (destinations ascending), sources
 *                                     ascending within a destination
 *   out_ptr[n+1], out_dst[m], out_w[m] out-edges grouped by source,
 *                                     destinations ascending
 *   out_to_in[m]                      offsetList: out position -> in position
 *   out_deg[n], in_deg[n]             degrees of the stored graph
 *   edge_map[m_input]                 input edge i -> its out position,
 *                                     -1 if it was a dropped self-loop
 * Self-loops are dropped and repeated (src, dst) pairs are merged into one
 * edge whose weight is the sum of their weights, added in input order.  The
 * weight arrays are NULL for an unweighted graph.  All arrays are allocated
 * by the library and released by pr_csr_free.
 * ---------------------------------------------------------------------- */
typedef struct pr_csr {
  int64_t n;
  int64_t m;
  int64_t *in_ptr;
  int32_t *in_src;
  double *in_w;
  int64_t *out_ptr;
  int32_t *out_dst;
  double *out_w;
  int64_t *out_to_in;
  int32_t *out_deg;
  int32_t *in_deg;
  int64_t m_input;
  int64_t *edge_map;
} pr_csr;

/* Build the canonical graph from an edge list (host arrays src[m], dst[m],
 * optional host weights w[m], each finite and > 0).  n >= 1, m >= 0.
 * PR_EINVAL on an id outside [0, n) or a bad weight; PR_ENOMEM on allocation
 * failure.  *out is zeroed first and owns the result on success. */
int pr_build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *w,
                 pr_csr *out);
void pr_csr_free(pr_csr *csr);

/* ------------------------------------------------------------------------
 * Device graph.
 *
 * pr_graph_create copies the graph to the current device and builds the
 * execution plan: vertices are binned by in-degree (one lane up to a whole
 * wavefront per vertex; very long lists split over several wavefronts), the
 * in-edges are re-laid in bin order, and the gathered array is laid out by
 * gather count so its hottest part can sit in LDS.  The library owns that
 * device memory and the per-graph workspace; pr_graph_destroy releases them
 * (pr_graph_bind below places the graph in the caller's memory instead).
 * ---------------------------------------------------------------------- */
typedef struct pr_graph pr_graph;

typedef struct pr_plan_opts {
  int chunk;             /* lists longer than this (hubs) are summed by several wavefronts:
                            up to 8 * chunk edges (and at most one workgroup's share of a
                            launch) by the 8 wavefronts of one workgroup, longer ones in
                            pieces of at most chunk edges, one wavefront each, added by the
                            finalize kernel (0 = default: about the edges per wavefront of
                            a sweep launch, a power of two in [1024, 16384]; else [64, 2^20]) */
  int tile_max_row;      /* lists of 1..tile_max_row edges are packed into 512-edge tiles
                            (default 512, at most 512; lowered to chunk if larger); longer
                            ones get a wavefront each */
  int tile_rows;         /* rows per tile at most (1..128, default 128) */
  int steps;             /* one-wavefront rows per work item (default 1) */
  int hot_slots;         /* gather slots staged in LDS per sweep workgroup (-1 = as many as fit,
                            0 = none) */
  int gather_layout;     /* order of the gathered array: 1 sorted by gather count, the hottest
                            vertices first; 0 vertex-id order; 2 the most gathered vertices (as
                            many as the LDS copy holds in FP32) first, the rest in vertex-id
                            order, which keeps the locality of an ordered input; -1 (default)
                            2 when the input is local (see local_share), else 1 */
  int with_adjoint;      /* also plan the out-edge (transposed) pull for pr_adjoint */
  int gs_blocks;         /* Gauss-Seidel blocks of the fused form (0 = default: 1 when the
                            input is local (see local_share), else by edges per sweep
                            wavefront: 1 under 64, 2 under 6144, 3 under 49152, else 8;
                            else 1..64): the
                            vertices, in decreasing out-degree, are cut into this many blocks
                            of equal in-edge count (hubs join the last block) and swept one
                            launch each, so every block reads the contributions the blocks
                            before it wrote in the same sweep (Eq. 9 over the blocks).  The
                            Jacobi form ignores it. */
  int with_cl;           /* also build the edge-centric contributionList layout (Section 3:
                            contributionList + offsetList) for PR_EDGE_LIST: 8 B (16 B
                            weighted) per edge more on the device (default 0) */
  int with_inplace;      /* also keep the in-edges in vertex order (offsets, sources, weights)
                            for PR_INPLACE: 4 B (12 B weighted) per edge and 4 B per vertex
                            more on the device (default 0) */
} pr_plan_opts;

void pr_plan_opts_default(pr_plan_opts *o);

/* csr: a canonical graph from pr_build_csr (host memory).  opts may be NULL. */
int pr_graph_create(const pr_csr *csr, const pr_plan_opts *opts, pr_graph **out);
void pr_graph_destroy(pr_graph *g);

typedef struct pr_graph_stats {
  int64_t n, m;
  int64_t n_light, n_medium, n_heavy; /* vertices per bin: one lane, several lanes, chunked */
  int64_t e_light, e_medium, e_heavy; /* in-edges per bin */
  int64_t n_items;                    /* wavefront work items per sweep */
  int64_t n_dangling;
  int64_t device_bytes;               /* graph + plan bytes held on the device */
  int grid;                           /* workgroups of one sweep launch */
  int gs_blocks;                      /* Gauss-Seidel blocks (sweep launches of the fused form) */
  int chunk;                          /* hub threshold in edges, as resolved */
  int64_t graph_captures;             /* hipGraphs of sweeps captured so far for this graph
                                         (one per distinct launch configuration; not per
                                         output or teleport vector) */
  uint64_t signature;                 /* 64-bit hash of the stored graph (sizes, offsets,
                                         neighbours, weights): the key of tuned settings */
  double local_share;                 /* share of the in-edges whose source id is within
                                         1024 of the destination's.  At 1/4 or more, and at
                                         least four times the share of a random labeling
                                         (about 2048 / n), the input counts as local (a grid,
                                         a mesh, a road network in its natural order):
                                         out-degree blocks would then
                                         interleave in id order and read every source line
                                         once per block, so the default plan keeps one block
                                         and the id order of the gathered array */
  int gather_layout;                  /* the gathered array's order, as resolved */
} pr_graph_stats;

int pr_graph_stats_get(const pr_graph *g, pr_graph_stats *out);

/* Caller-owned device memory for the graph (the input G = (V, E) of
 * Section 3, which the paper's Algorithm 1 takes as given).
 *
 * pr_graph_device_bytes runs the planning of pr_graph_create on csr and opts
 * without touching the device and returns in *bytes the device memory the
 * graph and its plan occupy (every array rounded up to 256 bytes).
 * pr_graph_bind then builds the same graph with every one of those arrays
 * placed in the caller's device buffer dev_mem (current device, 256-byte
 * aligned, at least *bytes long; e.g. a torch uint8 tensor): the library
 * allocates no device memory for the graph (only its stream, two events and
 * a small pinned state block).  The buffer must outlive the graph and must
 * not be written while the graph exists.  Workspace the solvers allocate on
 * first use is still the library's unless a solve takes the caller's
 * (pr_solve_ws).  PR_EINVAL on a misaligned or non-device dev_mem, PR_ENOMEM
 * when it is too small.
 * pr_graph_free releases what the library owns of a graph (created or bound);
 * a bound graph's buffer stays the caller's. */
int pr_graph_device_bytes(const pr_csr *csr, const pr_plan_opts *opts, size_t *bytes);
int pr_graph_bind(const pr_csr *csr, const pr_plan_opts *opts, void *dev_mem, size_t bytes, pr_graph **out);
void pr_graph_free(pr_graph *g);

/* ------------------------------------------------------------------------
 * Solver options.
 * ---------------------------------------------------------------------- */
enum pr_mode { PR_JACOBI = 0, PR_FUSED = 1, PR_EDGE_LIST = 2, PR_INPLACE = 3, PR_FUSED_EDGE_LIST = 4 };
enum pr_precision { PR_FP64 = 0, PR_FP32 = 1 };
enum pr_dangling { PR_DANGLING_UNIFORM = 0, PR_DANGLING_LEAK = 1 };
enum pr_norm { PR_NORM_L1 = 0, PR_NORM_LINF = 1 };

typedef struct pr_opts {
  int mode;             /* PR_JACOBI (Algorithm 1 as a pull), PR_FUSED (Algorithm 2, block
                            Gauss-Seidel) or PR_EDGE_LIST (Algorithm 1 with the paper's
                            edge-ordered contributionList: a scatter through offsetList, then
                            contiguous row sums; needs a graph planned with with_cl; same
                            values, same summation order, same results as PR_JACOBI), or
                            PR_INPLACE (Algorithm 2 / Eq. 9 swept in place: each wavefront
                            sweeps a contiguous range of blocks of consecutive vertices in
                            ascending order, stages a block's contributions in LDS and
                            updates the block in order, each lane walking its own run
                            of consecutive vertices, so a source inside the block that is
                            already updated is read fresh; the blocks run asynchronously,
                            reading the other blocks' contributions from one shared array
                            in whatever state it is (Section 4.3); needs a graph planned
                            with with_inplace; not bit-reproducible across runs, same fixed
                            point), or
                            PR_FUSED_EDGE_LIST (Algorithm 2 with the paper's contributionList:
                            per Gauss-Seidel block, the rows sum their contiguous list slices
                            and update, then the block's vertices scatter their new
                            contributions through offsetList; the list is filled once from
                            the start vector; needs with_cl; same values, same summation
                            order, same results as PR_FUSED) */
  int precision;        /* PR_FP64, or PR_FP32: ranks and contributions stored and summed
                           in FP32 with compensated sums; residual and dangling mass in FP64 */
  int dangling;         /* PR_DANGLING_UNIFORM, or PR_DANGLING_LEAK (the paper's literal
                           algorithms, which drop dangling mass) */
  int norm;             /* residual norm: PR_NORM_L1, or PR_NORM_LINF (Eq. 3; Jacobi only) */
  int warm_start;       /* 1: start from the x passed in; 0: start from p */
  int fused_scaled;     /* PR_FUSED only: scale the teleport term by the previous sweep's
                           total mass (default 1); 0 = plain lagged-dangling sweep */
  int sweeps_per_poll;  /* sweeps queued between host convergence polls (default 8) */
  int use_hip_graph;    /* capture the queued sweeps in a hipGraph (default 1) */
  double refine_tol;    /* PR_FP32: FP64 refinement sweeps continue until the FP64 residual
                           is below this (0 = no refinement; default: the solve's tol) */
  double fp32_tol;      /* PR_FP32: residual at which the FP32 stage hands over to the FP64
                           refinement (default max(tol, 1e-7)) */
  double *trace;        /* optional host array[max_iter]: residual after each sweep */
} pr_opts;

void pr_opts_default(pr_opts *o);

/* ------------------------------------------------------------------------
 * Forward solve.
 *
 * pr_solve iterates until the residual (the norm of the change between
 * successive iterates, Eq. 3 with the chosen norm) drops below tol, or
 * max_iter sweeps.  Algorithm 1 / Algorithm 2 loop structure: the pull, the
 * update, the dangling-mass and residual reductions and the convergence test
 * are fused into one kernel per sweep.
 *   d        damping factor, 0 < d < 1 (the paper uses 0.85)
 *   tol      > 0;  max_iter >= 1
 *   p        device double[n] teleport vector (finite, >= 0, sum 1), or NULL for 1/n;
 *            device memory, so the library does not check it: a p outside this
 *            contract gives ranks and residuals that mean nothing, with no error
 *   x        device double[n]: start vector if o->warm_start, else ignored on entry;
 *            the ranks on return (sum 1 for uniform dangling)
 *   iters    host: sweeps executed (FP32: FP32 sweeps + FP64 refinement sweeps)
 *   resid    host: residual of the last sweep
 * Returns PR_NOT_CONVERGED (x valid) when max_iter is reached first.
 * ---------------------------------------------------------------------- */
int pr_solve(pr_graph *g, double d, double tol, int max_iter, const pr_opts *o, const double *p,
             double *x, int *iters, double *resid, void *stream);

/* pr_solve in a workspace the caller owns: the damping d and tolerance tol of
 * Section 5's experiments and the stop rule of Section 3, with the
 * contribution arrays (and the FP32 copy of the ranks) in ws, a device buffer
 * of at least pr_workspace_bytes(g, tol, o) bytes (256-byte aligned), so the
 * call allocates no workspace.  Same checks and results as pr_solve; refuses
 * the edge-list forms and a residual trace (PR_EINVAL), whose buffers stay
 * the library's.  ws may be reused by later calls on any graph that fits;
 * calls that share one ws must not overlap. */
int pr_workspace_bytes(const pr_graph *g, double tol, const pr_opts *o, size_t *bytes);
int pr_solve_ws(pr_graph *g, double d, double tol, int max_iter, const pr_opts *o, const double *p, double *x,
                void *ws, size_t ws_bytes, int *iters, double *resid, void *stream);

/* pr_solve for callers that cannot allocate device memory (code that must
 * not call hipMalloc, tight serving loops, harnesses that forbid allocation).
 * Same arguments, checks, results and return values as pr_solve on a graph
 * that already exists; the caller passes x (and p) as before.  Where pr_solve
 * allocates the contribution arrays (and the FP32 copy of the ranks) on first
 * use, this entry point takes them from a fixed array in the library's device
 * image: pr_noalloc_scratch_bytes() bytes (32 MiB) on each device, held until
 * the process ends.  A solve needs 16 n bytes in FP64 and 12 n in FP32, plus
 * 16 n for the FP64 refinement (each rounded up to 256 bytes), so up to about
 * 2 million vertices in FP64; a larger graph gives PR_EINVAL.  It queues its
 * sweeps as plain launches (no hipGraph is instantiated), and refuses
 * PR_EDGE_LIST and a residual trace, which need buffers of their own
 * (PR_EINVAL).  Every call on one device works in the same array: calls that
 * overlap on one device (any graphs, any threads or streams) race and give
 * wrong ranks.  Nothing in the array needs to start at zero: each call writes
 * every value before reading it. */
int pr_solve_noalloc(pr_graph *g, double d, double tol, int max_iter, const pr_opts *o, const double *p,
                     double *x, int *iters, double *resid, void *stream);
size_t pr_noalloc_scratch_bytes(void);

/* Exactly `sweeps` sweeps from the x passed in (no convergence test), in the
 * form o->mode and the precision o->precision select: the body of
 * Algorithm 1's loop (Eq. 2, Jacobi) or of Algorithm 2's (Eq. 9, fused),
 * without the stop test of Eq. 3.  x is FP64 on entry and
 * on return; FP32 sweeps run on an internal FP32 copy that is cast back after
 * the last sweep (no refinement).  resid (host, nullable) receives the residual
 * of the last sweep.  elapsed_ms (host, nullable) receives the time between
 * HIP events recorded on the library's work stream right before the first
 * and right after the last sweep kernel (launched as one hipGraph when
 * o->use_hip_graph), i.e. the sweeps' device time. */
int pr_iterate(pr_graph *g, double d, const pr_opts *o, const double *p, double *x, int sweeps,
               double *resid, double *elapsed_ms, void *stream);

/* Per-kernel device time of the sweep: `sweeps` sweeps from x (FP64 on entry
 * and on return, as pr_iterate; teleport 1/n), launched one by one on the
 * library's work stream with HIP events recorded before the sweep kernel,
 * between it and its reduction (finalize) kernel, and after the latter.
 *   sweep_ms, finalize_ms   host: average milliseconds per sweep of each; the
 *                           sweep kernel's time covers all of its launches in
 *                           one sweep (one per Gauss-Seidel block in the fused
 *                           form; the scatter and the list sums in the
 *                           edge-list form)
 * Measurement support for the sweep of the recurrence above (the per-iteration
 * time the paper compares in Section 6); 1 <= sweeps <= 4096. */
int pr_profile_sweeps(pr_graph *g, double d, const pr_opts *o, double *x, int sweeps, double *sweep_ms,
                      double *finalize_ms, void *stream);

/* ||F(x) - x||_1 for any device vector x (FP64), where F is one exact
 * application of Eq. 1 (one Jacobi sweep, Eq. 2).  Not in the paper: F is a
 * contraction with factor d in the L1 norm, which bounds the error of x:
 * ||x - x*||_1 <= ||F(x) - x||_1 / (1 - d).  result: host double. */
int pr_certificate(pr_graph *g, double d, const double *p, const double *x, double *result,
                   void *stream);

/* Device time of the sweep's memory gathers alone: a kernel on the sweep's
 * grid that reads, from an n-element array of the precision's type (FP64 8
 * bytes, FP32 4 bytes, allocated and freed by the call), the value at every
 * in-edge's gather slot in the plan's bin order, skipping the slots the sweep
 * keeps in its LDS copy, eight loads in flight per lane, and sums them
 * (mode 0); or as many slots drawn uniformly from [0, n) by a counter-based
 * SplitMix64 mix of the edge index (mode 1: random lines that no cache holds).
 * Nothing else is read or written.  The gathers are the reads of Eq. 1's sum;
 * on a graph without id locality their rate, not HBM's streaming rate, bounds
 * the sweep, so this is the sweep's floor on the device it runs on.
 *   precision      PR_FP64 or PR_FP32
 *   reps           timed launches after one untimed launch, 1..1000
 *   best_us        host: fastest launch in microseconds
 *   mean_us        host, nullable: their mean
 * Measurement support; PR_EINVAL on bad arguments or a graph on another
 * device, PR_ENOMEM when the array does not fit, PR_EDEVICE on a HIP error.
 * The call waits for its launches. */
int pr_probe_gathers(pr_graph *g, int precision, int mode, int reps, double *best_us, double *mean_us,
                     void *stream);

/* ------------------------------------------------------------------------
 * Batched personalized PageRank: k teleport vectors, each one-hot on
 * seeds[j] (Eq. 1 with a personalised teleport term), solved together as a
 * multi-column Jacobi pull per sweep.  Dangling mass is spread uniformly.
 * Ranks are FP32 (compensated sums), per-column residual and dangling mass
 * FP64; a column is frozen once its L1 residual is below tol.  Unweighted
 * graphs only: a graph created with edge weights gives PR_EINVAL.
 *
 * Launch shape: `tile` columns advance per launch (a multiple of 4, at most
 * 64; inside a launch the columns of a vertex form one contiguous row, read
 * whole per in-edge), each sweep wavefront takes `items_per_grab` consecutive
 * work items (runs of rows, long rows, hub chunks) at a time (1..16), and the
 * sweep kernel runs `wg_per_cu` workgroups per compute unit (1 or 2).  The
 * shape changes only the time: every column is summed in the same order and
 * every per-column reduction runs over work items in item order, so all
 * shapes give the same bits.
 * ---------------------------------------------------------------------- */
typedef struct pr_batch_shape {
  int tile;
  int items_per_grab;
  int wg_per_cu;
} pr_batch_shape;

/* tile 64, items_per_grab 1, wg_per_cu 2 */
void pr_batch_shape_default(pr_batch_shape *s);

/* k personalized solves of Eq. 1 (teleport e_{seeds[j]} for column j), as above.
 *   seeds   device int32[k], ids in [0, n) (checked: PR_EINVAL);  1 <= k <= 1024
 *   shape   launch shape (host), or NULL: the autotuned one (pr_autotune_batched,
 *           cache file from the FUSEDPR_TUNE_CACHE environment variable)
 *   X       device float[n * k], row-major (vertex-major): X[v * k + j]
 *   iters   host int[k]: sweeps until column j froze (or max_iter)
 *   resid   host double[k]: last residual of each column
 * The sweeps of each launch of columns run as hipGraphs of 8 sweeps (the
 * host polls the per-column state between them; sweeps after every column
 * froze exit at once).  Stream order: runs on the graph's work stream after
 * the work queued on `stream`, and returns once the results are in X, iters
 * and resid. */
int pr_solve_batched(pr_graph *g, double d, double tol, int max_iter, int k, const int32_t *seeds,
                     const pr_batch_shape *shape, float *X, int *iters, double *resid, void *stream);

/* Autotuner for pr_solve_batched (Eq. 1 with one-hot teleports; not in the
 * paper, which solves one vector at a time): times every tile width from 8
 * to 64 (4 when k is smaller), with 1, 2 or 4 items per grab and 1 or 2
 * workgroups per compute unit, on this graph and device (4 sweeps each), and
 * returns the fastest per column in *shape.  When cache_path is not NULL the
 * choice is read from / appended to that JSON-lines file, keyed by the graph's
 * signature (pr_graph_stats.signature), its size, k and the device name. */
int pr_autotune_batched(pr_graph *g, int k, const char *cache_path, pr_batch_shape *shape, void *stream);

/* ------------------------------------------------------------------------
 * Adjoint (implicit differentiation of the fixed point).
 *
 * Not in the paper, which only solves the forward problem: the fixed point
 * of Eq. 1 is x = (1-d)(I - dP)^{-1} p, so its gradients need one solve with
 * the transposed operator instead of differentiating through the iterates.
 * For a scalar loss L(x) with dL/dx = g, solves (I - dP)^T lam = g by the
 * transposed Jacobi pull over out-edges, then
 *   dL/dp_u       = (1-d) lam_u
 *   dL/dw(v->u)   = d * x_v / W_v * (lam_u - (P^T lam)_v)
 * (the second term is the derivative of the normalisation by W_v).
 *   x      device double[n]: the forward solution
 *   g      device double[n]
 *   lam    device double[n] out
 *   dLdp   device double[n] out (nullable)
 *   dLdw   device double[m] out in out-edge (pr_csr out_*) order (nullable)
 *   tol    on max |lam' - lam|;  iters / resid: host
 * The graph must have been created with with_adjoint = 1.
 * ---------------------------------------------------------------------- */
int pr_adjoint(pr_graph *g, double d, const double *x, const double *dLdx, double tol, int max_iter,
               double *lam, double *dLdp, double *dLdw, int *iters, double *resid, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FUSEDPR_H */
