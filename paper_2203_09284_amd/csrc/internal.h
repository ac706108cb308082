// Internal declarations of the fusedpr library (host side and kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fusedpr.h"

// ----------------------------------------------------------------- errors --
int pr_fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void pr_clear_error();

#define PR_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return pr_fail(e_ == hipErrorOutOfMemory ? PR_ENOMEM : PR_EDEVICE, "%s: %s (%s:%d)", \
                     #call, hipGetErrorString(e_), __FILE__, __LINE__);               \
  } while (0)

// ------------------------------------------------------------- constants --
namespace fpr {

constexpr int kBlock = 256;          // threads per workgroup of the small kernels
constexpr int kWaves = kBlock / 64;
#ifndef FPR_SWEEP_BLOCK
#define FPR_SWEEP_BLOCK 512
#endif
#ifndef FPR_HOT_KB
#define FPR_HOT_KB 70
#endif
constexpr int kSweepBlock = FPR_SWEEP_BLOCK;  // threads per workgroup of the sweep
constexpr int kSweepWaves = kSweepBlock / 64;
constexpr int kFinBlock = 1024;  // threads of the one-workgroup finalize kernel
constexpr int kBatch = 8;                     // loads in flight per lane and batch
constexpr int kPrefetch = 4;                  // row rounds whose list bounds are loaded up front
constexpr int kHotBytes = FPR_HOT_KB * 1024;  // LDS holding the hottest gather slots, per workgroup
constexpr int kHotLayout = kHotBytes / 4;     // slots kept in gather-count order by gather_layout 2
constexpr int64_t kLocalSpan = 1024;          // id distance under which an in-edge counts as local
#ifndef FPR_IP_RUN
#define FPR_IP_RUN 4
#endif
// In-place form: a wavefront's block of 64 * kIpRun vertices is updated in
// kIpRun steps, lane l taking its run of consecutive vertices l * kIpRun + k
// (k = 0 .. kIpRun - 1).  The plan stores the block interleaved: vertex
// l * kIpRun + k sits at position 64 k + l, so every step reads and writes
// consecutive positions (the last, partial block keeps vertex order).
constexpr int kIpRun = FPR_IP_RUN;
constexpr int kIpVpb = 64 * kIpRun;
constexpr int kTileEdges = 512;               // edges of a tile: 8 consecutive per lane
constexpr int kTileRows = 128;                // rows of a tile at most (row sums staged in LDS)
constexpr int kVRunCost = 64;                 // batched: batch rounds per run of short rows

enum ItemKind : int { kTile = 0, kRows = 1, kHeavy = 2, kZero = 3, kHubWG = 4, kVLong = 5, kVQuad = 6 };

// Sweep flags (runtime, uniform across the grid)
enum SweepFlags : int {
  kFlagLeak = 1,      // no dangling term (the paper's literal algorithms)
  kFlagLinf = 2,      // max-norm residual instead of L1
  kFlagScaled = 4,    // teleport scaled by the previous sweep's total mass
  kFlagUniformP = 8,  // p == 1/n (p pointer unused)
  kFlagAdjoint = 16,  // transposed iteration: lam' = g + d (W^-1 sum w lam + [W = 0] sum(lam) / n)
  kFlagList = 32,     // edge-centric list form: no n-length contribution array
};

// Device-resident state of an iteration; one per graph and pull direction.
struct SweepState {
  int iter;           // sweeps completed
  int done;           // 1 once the residual is below tol or iter == max_iter
  int max_iter;
  double tol;
  double D;      // dangling mass of the current iterate
  double S;      // total mass of the current iterate
  double resid;  // residual of the last sweep
  double raw;    // unscaled L1 (or max) change of the last sweep
};

// Where the sweeps of one plan find the caller's vectors: the rank vector x
// (FP64 or FP32) and the teleport vector p (null = 1/n).  The block lives in
// device memory and the kernels read it when they start, so a captured
// hipGraph of sweeps serves every x and p without capturing again.
struct IoPtrs {
  void *x;
  const double *p;
};

// One binned pull layout: vertices grouped by degree, neighbours re-laid in
// bin order.  Used for the forward pull over in-edges and the transposed
// pull over out-edges.
struct DevPlan {
  int64_t n = 0, m = 0;
  uint32_t *rows = nullptr;   // [n] vertex ids in bin order
  uint32_t *rowpos = nullptr; // [n] gather-layout slot of rows[i]
  uint32_t *gpos = nullptr;   // [n] gather-layout slot of every vertex
  uint32_t *rptr = nullptr;   // [n+1] edge offsets (bin order)
  int32_t *idx = nullptr;     // [m] gather-layout slots of the neighbours
  double *w = nullptr;        // [m] edge weights or null
  int4 *items = nullptr;      // [n_items] sweep list: {kTile, tile} | {kRows, first, end, lanes per
                              // row} | {kHubWG, row} (whole workgroup) | {kHeavy, row, chunk, slot}
                              // | {kZero, first, end}
  int4 *bitems = nullptr;     // [n_bitems] batched list: {kHeavy, row, chunk, slot} (hub chunk) |
                              // {kVLong, row} (one long row) | {kVQuad, first run, runs (1..4)}
  int2 *vrun = nullptr;       // [n_vrun] batched row runs [first, end) of short and empty rows
  int4 *tiles = nullptr;      // [n_tiles] {first row, rows, edges, 0}
  int32_t *tidx = nullptr;    // [n_tiles * 512] tile edges, lane-transposed: [k][lane] = edge 8*lane+k
  double *tw = nullptr;       // [n_tiles * 512] their weights, same layout (or null)
  uint8_t *tmask = nullptr;   // [n_tiles * 64] per lane: bit k set if edge 8*lane+k starts a row
  int4 *hsplit = nullptr;     // [n_split] rows split into chunks: {row index, first slot, chunks, 0}
                              // (batched list: every hub)
  int4 *msplit = nullptr;     // [n_msplit] the hubs the sweep list splits into chunks (same slots)
  double *hpart = nullptr;    // [n_chunks] partial sums of the chunks of split rows
  double *wave_part = nullptr;  // [3][part_stride] per-workgroup change, dangling mass, total mass;
                                // block b's launch writes from b * (workgroups per launch)
  SweepState *st = nullptr;
  IoPtrs *io = nullptr;           // device block read by the sweep kernels
  IoPtrs io_last{nullptr, nullptr};  // what the last queued write put there
  bool io_valid = false;
  int n_items = 0;
  int n_bitems = 0;
  int n_vrun = 0;
  int n_tiles = 0;
  int n_heavy = 0;
  int n_split = 0;
  int n_msplit = 0;
  int n_chunks = 0;
  int chunk = 2048;
  int n_waves = 0;  // wavefronts of one sweep launch
  int part_stride = 0;
  int n_blocks = 1;               // Gauss-Seidel blocks of the fused form
  std::vector<int> block_items;   // [n_blocks + 1] first position of each block's sweep list
  int *block_pos = nullptr;       // the same on the device
  int *wave_cnt = nullptr;        // [n_blocks * n_waves] list length of each wavefront per block
  // contributionList layout (plan option with_cl): list position of every
  // edge = its position in tidx (tile rows) or cl_rows + its idx position
  int32_t *cl_src = nullptr;      // [m] source of each out-edge, grouped by the launch that
                                  // updates the source (cl_group), out-CSR order inside a group
  int32_t *cl_pos = nullptr;      // [m] its list position
  double *cl_w = nullptr;         // [m] its weight (weighted graphs)
  int64_t cl_size = 0;            // list positions (tiles * 512 + m)
  uint32_t cl_rows = 0;           // first position of the idx region
  // in-place form (plan option with_inplace): the in-edges by position
  // (vertex order, interleaved inside each block: kIpRun)
  uint32_t *ip_ptr = nullptr;     // [n+1] offsets, in position order
  int32_t *ip_src = nullptr;      // [m] source positions
  double *ip_w = nullptr;         // [m] weights (weighted graphs)
  uint32_t *ip_pos = nullptr;     // [n] position of each vertex
  double *ip_iw = nullptr;        // [n] 1/W in position order
  int32_t *ip_range = nullptr;    // [W+1] first block of each sweep wavefront (equal cost)
  std::vector<int64_t> cl_group;  // [n_blocks + 2] first scatter entry of each group: sources
                                  // updated by block b's launch, then by the finalize kernel
  std::vector<uint8_t> upd_launch;  // host, during planning: the launch that updates each vertex
  std::vector<int64_t> inpos;     // host, during planning: in-CSR edge -> list position
  std::vector<int> block_slots;   // [n_blocks + 1] first gather slot of each block's non-hub
                                  // vertices (the hubs' slots come before block 0's)
  int64_t n_light = 0, n_medium = 0, n_heavy_rows = 0;  // rows in tiles, one wavefront each, chunked
  int64_t e_light = 0, e_medium = 0, e_heavy = 0;
  int64_t bytes = 0;
};

}  // namespace fpr

// A hipGraph of queued sweeps, keyed by the bytes of its launch arguments.
struct GraphEntry {
  std::vector<unsigned char> key;
  hipGraphExec_t exec;
};

struct pr_graph {
  int device = 0;
  int n_cu = 0;
  double local_share = 0.0;  // in-edges whose source id is within kLocalSpan of the destination
  int64_t n = 0, m = 0;
  bool weighted = false;
  pr_plan_opts popts{};
  fpr::DevPlan fwd, adj;
  bool has_adj = false;
  double *inv_w = nullptr;      // [n] 1 / W_v, 0 for dangling vertices
  uint32_t *out_ptr = nullptr;  // [n+1] out-edge offsets (adjoint gradient layout)
  int32_t *out_dst = nullptr;   // [m] out-edge destinations in pr_csr order (adjoint gradients)
  double *out_w = nullptr;      // [m] their weights (or null)
  double *ca64[2] = {nullptr, nullptr};  // adjoint gather buffers
  int64_t n_dangling = 0;
  int grid = 0;  // persistent workgroups per sweep
  hipStream_t work = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // workspace (allocated on first use)
  double *c64[2] = {nullptr, nullptr};
  float *c32[2] = {nullptr, nullptr};
  float *x32 = nullptr;
  double *cl64 = nullptr;       // contributionList buffers of the edge-centric form
  float *cl32 = nullptr;
  double *xtmp = nullptr;
  double *trace_dev = nullptr;
  int trace_cap = 0;
  fpr::SweepState *host_st = nullptr;  // pinned mirror of the state
  double *red_tmp = nullptr;           // small reduction scratch
  // batched workspace
  float *Xb[2] = {nullptr, nullptr};
  size_t Xb_elems = 0;
  double *bstate = nullptr;  // per-column state
  double *bpart = nullptr;   // per-item per-column partials
  size_t bpart_elems = 0;
  int *bhost = nullptr;
  void *vwork = nullptr;  // batched workspace bookkeeping (batched.hip)
  struct TuneMemo {
    int k, tile, ipw, wg;
  };
  std::vector<TuneMemo> tune_memo;  // autotuned batched launch shapes of this graph
  uint64_t signature = 0;           // hash of the graph (size, offsets, neighbours, weights)
  // hipGraphs of sweeps captured for this graph; calls on one graph never
  // overlap, so they need no lock
  std::vector<GraphEntry> graph_cache;
  int64_t graph_captures = 0;
  int64_t device_bytes = 0;
  std::vector<void *> owned;  // device allocations released by pr_graph_destroy
  // Where fpr_dev_alloc takes device memory from: the library's own hipMalloc
  // (kMemOwn), a count of the bytes only, with no device work (kMemCount; the
  // planning run behind pr_graph_device_bytes), or the caller's buffer
  // (kMemArena; pr_graph_bind), carved in 256-byte aligned pieces.
  int mem_mode = 0;
  unsigned char *arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
};

enum { kMemOwn = 0, kMemCount = 1, kMemArena = 2 };

// plan.hip
int fpr_dev_alloc(pr_graph *g, void **p, size_t bytes);
// sweep.hip
int fpr_grid_for(pr_graph *g);
void fpr_sweep_release(pr_graph *g);    // drops cached hipGraphs of g
// batched.hip
void fpr_batched_release(pr_graph *g);  // drops g's batched workspace bookkeeping
// adjoint.hip: dL/dp = (1-d) lam and dL/dw (out-edge order) from the converged lam
int fpr_adjoint_gradients(pr_graph *g, double d, const double *x, const double *lam, double *dLdp,
                          double *dLdw, hipStream_t s);
