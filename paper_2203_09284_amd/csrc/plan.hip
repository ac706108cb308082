// Device graph and execution plan (pr_graph_create).
//
// The sweep pulls, for every vertex, over a list (in-edges for the forward
// pull, out-edges for the transposed pull of the adjoint).  Every work item
// runs on one wavefront.  The plan bins vertices by list length L:
//   L = 0            zero rows: lane per vertex, no gathers (the update only).
//   1 <= L <= tmax   tiles: consecutive rows packed into 512-edge tiles, at
//                    most 128 rows each.  Lane l takes edges 8l..8l+7 of the
//                    tile; the tile's edge ids are stored lane-transposed so
//                    each load instruction reads 256 contiguous bytes, with a
//                    bit per edge marking row starts.  A segmented scan
//                    across the lanes completes rows that span lanes.
//   tmax < L <= chunk  a wavefront per vertex, lanes striding the list.
//   L > chunk        hubs: each chunk of `chunk` edges is one item; the
//                    chunk sums go to per-chunk slots and the sweep's
//                    finalize kernel adds them in chunk order.
// The vertices are first cut into Gauss-Seidel blocks for the fused form
// (gs_blocks; block 0 holds the highest out-degree vertices, the hubs go to
// the last block).
// Rows are laid out block by block, and inside a block hubs, one-wavefront
// rows, tile rows, zero rows (vertex ids ascending inside each bin); that is
// also the order work items run in.
//
// Gather layout: the array the pull gathers from (contributions forward,
// adjoint values backward) is stored hubs first, then block by block, each
// group with its vertices sorted by how often they are gathered (descending,
// ties by id); the neighbour lists hold those slots.  On power-law graphs the
// few vertices that feed most edges then pack into the first slots, which
// each sweep workgroup keeps in LDS, and the slots of each block form one
// range.  Values are unchanged; only addresses move.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <queue>
#include <vector>

#include "internal.h"

using namespace fpr;

extern "C" void pr_plan_opts_default(pr_plan_opts *o) {
  if (!o) return;
  o->chunk = 0;
  o->tile_max_row = kTileEdges;
  o->tile_rows = kTileRows;
  o->steps = 1;
  o->hot_slots = -1;
  o->gather_layout = -1;
  o->with_adjoint = 0;
  o->gs_blocks = 0;
  o->with_cl = 0;
  o->with_inplace = 0;
}

int fpr_dev_alloc(pr_graph *g, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (g->mem_mode != kMemOwn) {
    const size_t piece = (bytes + 255) & ~(size_t)255;
    if (g->mem_mode == kMemArena && g->arena_used + piece > g->arena_bytes)
      return pr_fail(PR_ENOMEM, "pr_graph_bind: the device buffer (%zu bytes) is too small (%zu more needed)",
                     g->arena_bytes, g->arena_used + piece - g->arena_bytes);
    // counting: a distinct dummy address per piece (never dereferenced)
    *p = g->mem_mode == kMemArena ? (void *)(g->arena + g->arena_used) : (void *)(uintptr_t)(4096 + g->arena_used);
    g->arena_used += piece;
    g->device_bytes += (int64_t)bytes;
    return PR_OK;
  }
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
  if (count && g->mem_mode != kMemCount) PR_HIP(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return PR_OK;
}

// Build one binned pull plan from a CSR (ptr[n+1], nbr[m], w[m] nullable).
static int build_plan(pr_graph *g, DevPlan &P, int64_t n, const int64_t *ptr, const int32_t *nbr,
                      const double *w, const pr_plan_opts &o, bool want_cl) {
  P.n = n;
  P.m = ptr[n];
  P.chunk = o.chunk;
  const int64_t m = P.m;
  // Gauss-Seidel blocks of the fused form: the vertices other than the
  // chunked rows (hubs), in decreasing gather count, are cut where the running
  // in-edge count passes b/B of all edges (equal work per block); the hubs
  // join the last block, whose chunk sums the finalize kernel adds.  Every
  // vertex of block b is updated before any vertex of block b+1 reads.
  std::vector<uint32_t> freq(n, 0), order(n);
  for (int64_t e = 0; e < m; ++e) freq[nbr[e]]++;
  for (int64_t v = 0; v < n; ++v) order[v] = (uint32_t)v;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return freq[a] > freq[b]; });
  auto bin_of = [&](int64_t v) {
    const int64_t L = ptr[v + 1] - ptr[v];
    return L > o.chunk ? 0 : L > o.tile_max_row ? 1 : L > 0 ? 2 : 3;
  };
  const int B = std::max(1, std::min<int>(o.gs_blocks, 64));
  std::vector<uint8_t> blk(n, 0);
  {
    int64_t cum = 0;
    for (int64_t k = 0; k < n; ++k) {
      const uint32_t v = order[k];
      if (bin_of(v) == 0) {
        blk[v] = (uint8_t)(B - 1);
        continue;
      }
      blk[v] = (uint8_t)std::min<int64_t>(B - 1, m > 0 ? (cum * B) / m : 0);
      cum += ptr[v + 1] - ptr[v];
    }
  }
  // Gather layout: the hubs first, then the other vertices block by block;
  // inside each group by decreasing gather count (gather_layout = 1), by
  // vertex id (0), or (2) the group's vertices among the kHotLayout most
  // gathered ones first, by decreasing gather count, then the rest by vertex
  // id (keeps the locality of an ordered input for the gathers that miss the
  // LDS copy).  block_slots[b] = first slot of block b's non-hub vertices, so
  // the slots block b+1 reads fresh are [block_slots[0], block_slots[b+1]).
  std::vector<uint32_t> pos(n);
  {
    std::vector<uint32_t> rank(n);
    for (int64_t k = 0; k < n; ++k) rank[order[k]] = (uint32_t)k;
    auto group = [&](uint32_t v) { return bin_of(v) == 0 ? -1 : (int)blk[v]; };
    auto key = [&](uint32_t v) -> uint64_t {  // order inside a group
      if (o.gather_layout == 1) return rank[v];
      if (o.gather_layout == 2 && rank[v] < (uint32_t)kHotLayout) return rank[v];
      return (uint64_t)kHotLayout + v;
    };
    std::vector<uint32_t> lay(n);
    for (int64_t k = 0; k < n; ++k) lay[k] = (uint32_t)k;
    std::sort(lay.begin(), lay.end(), [&](uint32_t a, uint32_t b) {
      const int ga = group(a), gb = group(b);
      return ga != gb ? ga < gb : key(a) < key(b);
    });
    for (int64_t k = 0; k < n; ++k) pos[lay[k]] = (uint32_t)k;
    P.block_slots.assign(B + 1, (int)n);
    for (int64_t k = n - 1; k >= 0; --k)
      if (group(lay[k]) >= 0) P.block_slots[group(lay[k])] = (int)k;
    for (int b = B - 1; b >= 0; --b) P.block_slots[b] = std::min(P.block_slots[b], P.block_slots[b + 1]);
  }
  // bins per block: 0 hubs, 1 one-wavefront rows, 2 tile rows, 3 zero rows
  std::vector<std::vector<uint32_t>> bins((size_t)B * 4);
  for (int64_t v = 0; v < n; ++v) bins[(size_t)blk[v] * 4 + bin_of(v)].push_back((uint32_t)v);
  for (int b = 0; b < B; ++b)  // one-wavefront rows longest first: long items start early
    std::stable_sort(bins[(size_t)b * 4 + 1].begin(), bins[(size_t)b * 4 + 1].end(),
                     [&](uint32_t a, uint32_t c) { return ptr[a + 1] - ptr[a] > ptr[c + 1] - ptr[c]; });
  std::vector<uint32_t> rows;
  rows.reserve(n);
  for (auto &b : bins) rows.insert(rows.end(), b.begin(), b.end());
  std::vector<uint32_t> rptr(n + 1);
  rptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t v = rows[i];
    rptr[i + 1] = rptr[i] + (uint32_t)(ptr[v + 1] - ptr[v]);
  }
  std::vector<uint32_t> rowpos(n);
  for (int64_t i = 0; i < n; ++i) rowpos[i] = pos[rows[i]];
  std::vector<int32_t> idx(m);
  std::vector<double> wv(w ? m : 0);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t v = rows[i];
    int64_t L = ptr[v + 1] - ptr[v];
    for (int64_t k = 0; k < L; ++k) idx[rptr[i] + k] = (int32_t)pos[nbr[ptr[v] + k]];
    if (w) memcpy(&wv[rptr[i]], w + ptr[v], sizeof(double) * L);
  }

  if (want_cl) {
    P.inpos.assign((size_t)m, -1);
    // the launch that updates each vertex: its block's, or the finalize
    // kernel's (B) for the hubs split into chunks (set below)
    P.upd_launch.assign(blk.begin(), blk.end());
  }
  // Work items.  Per block, in launch order: hubs, one-wavefront rows (longest
  // first), tiles, zero rows.  Two lists share the rows and tiles:
  //  * the sweep list: a hub of at most 8 * chunk edges is one item of a
  //    whole workgroup (all 8 of its wavefronts), a longer hub is split into
  //    `chunk`-edge items whose sums the finalize kernel adds (msplit /
  //    hpart); the items are dealt to wavefronts per block (below);
  //  * the batched list: each hub is split into `chunk`-edge items whose sums
  //    the batched finalize kernel adds (hsplit / hpart); each row of the
  //    one-wavefront bin is an item of its own; the short and empty rows are
  //    cut into runs of about kVRunCost batch rounds, four runs to an item.
  const int W = g->grid * kSweepWaves;
  std::vector<int4> items, bitems, hsplit, msplit, tiles;
  std::vector<int2> vrun;
  std::vector<int> wave_cnt;
  // No single item may outlast the launch that holds it.  A whole-workgroup
  // hub takes at most 8 chunks and at most a workgroup's share of a launch's
  // edges (longer hubs are split); a split hub's pieces are the smallest
  // power of two, at least 1024, that covers a wavefront's share (at most
  // `chunk`).
  const int64_t share = m / ((int64_t)B * W);
  const int64_t wg_max =
      std::max<int64_t>(o.chunk, std::min<int64_t>((int64_t)kSweepWaves * o.chunk, share * kSweepWaves));
  int64_t piece = o.chunk;
  while (piece > 1024 && piece / 2 >= share) piece /= 2;
  P.chunk = (int)piece;
  std::vector<int32_t> tidx;
  std::vector<double> tw;
  std::vector<uint8_t> tmask;
  int64_t i = 0, chunks = 0;
  P.block_items.assign(1, 0);
  for (int b = 0; b < B; ++b) {
    std::vector<int4> rest;  // the block's items other than hubs, in order
    const auto &hubs = bins[(size_t)b * 4 + 0];
    const int64_t hub0 = i;
    std::vector<int4> mega;  // chunk items of the hubs longer than wg_max
    for (size_t h = 0; h < hubs.size(); ++h, ++i) {
      int64_t L = rptr[i + 1] - rptr[i];
      int64_t nch = (L + piece - 1) / piece;
      int slot = (int)chunks;
      hsplit.push_back(make_int4((int)i, slot, (int)nch, 0));
      if (L > wg_max) {
        msplit.push_back(make_int4((int)i, slot, (int)nch, 0));
        if (want_cl) P.upd_launch[rows[i]] = (uint8_t)B;
      }
      chunks += nch;
      for (int64_t c = 0; c < nch; ++c) {
        bitems.push_back(make_int4(kHeavy, (int)i, (int)c, slot));
        if (L > wg_max) mega.push_back(make_int4(kHeavy, (int)i, (int)c, slot));
      }
      P.e_heavy += L;
    }
    P.n_heavy_rows += (int64_t)hubs.size();
    const int64_t long0 = i;  // the block's one-wavefront, short and empty rows: [long0, short0), [short0, ...)
    {
      const int64_t end = i + (int64_t)bins[(size_t)b * 4 + 1].size();
      for (int64_t i0 = i; i0 < end; i0 += o.steps)
        rest.push_back(make_int4(kRows, (int)i0, (int)std::min(end, i0 + o.steps), 64));
      P.n_medium += end - i;
      P.e_medium += rptr[end] - rptr[i];
      i = end;
    }
    const int64_t short0 = i;
    {
      const int64_t end = i + (int64_t)bins[(size_t)b * 4 + 2].size();
      P.n_light += end - i;
      P.e_light += rptr[end] - rptr[i];
      while (i < end) {
        const int64_t r0 = i;
        int64_t edges = 0;
        while (i < end && i - r0 < o.tile_rows) {
          const int64_t L = rptr[i + 1] - rptr[i];
          if (edges + L > kTileEdges) break;
          edges += L;
          ++i;
        }
        const int t = (int)tiles.size();
        tiles.push_back(make_int4((int)r0, (int)(i - r0), (int)edges, 0));
        // the tile's first row, rows and edges travel in the item (one load less)
        rest.push_back(make_int4(kTile, t, (int)r0, (int)(((i - r0) << 16) | edges)));
        tidx.resize((size_t)(t + 1) * kTileEdges, 0);
        if (w) tw.resize((size_t)(t + 1) * kTileEdges, 0.0);
        tmask.resize((size_t)(t + 1) * 64, 0);
        int64_t j = 0;
        for (int64_t r = r0; r < i; ++r) {
          tmask[(size_t)t * 64 + (j >> 3)] |= (uint8_t)(1u << (j & 7));
          for (uint32_t e = rptr[r]; e < rptr[r + 1]; ++e, ++j) {
            const size_t at = (size_t)t * kTileEdges + (size_t)(j & 7) * 64 + (size_t)(j >> 3);
            tidx[at] = idx[e];
            if (w) tw[at] = wv[e];
            if (want_cl) P.inpos[(size_t)(ptr[rows[r]] + (e - rptr[r]))] = (int64_t)at;
          }
        }
      }
    }
    {
      const int64_t end = i + (int64_t)bins[(size_t)b * 4 + 3].size();
      for (int64_t i0 = i; i0 < end; i0 += 256)
        rest.push_back(make_int4(kZero, (int)i0, (int)std::min(end, i0 + 256), 0));
      P.n_light += end - i;
      i = end;
    }
    // batched list: the long rows one by one, then the short and empty rows
    // in runs (a run's cost: a round of up to 8 gathers per 8 edges, and one
    // for the update), four runs to an item
    for (int64_t r = long0; r < short0; ++r) bitems.push_back(make_int4(kVLong, (int)r, 0, 0));
    {
      std::vector<int2> runs;
      for (int64_t r = short0; r < i;) {
        const int64_t r0 = r;
        int64_t c = 0;
        while (r < i) {
          const int64_t cr = (int64_t)(rptr[r + 1] - rptr[r] + 7) / 8 + 1;
          if (c > 0 && c + cr > kVRunCost) break;
          c += cr;
          ++r;
        }
        runs.push_back(make_int2((int)r0, (int)r));
      }
      for (size_t q = 0; q < runs.size(); q += 4)
        bitems.push_back(make_int4(kVQuad, (int)(vrun.size() + q), (int)std::min<size_t>(4, runs.size() - q), 0));
      vrun.insert(vrun.end(), runs.begin(), runs.end());
    }
    // The sweep list of this block: work items are dealt to the W
    // wavefronts of a launch by longest-processing-time first, with a cost
    // model in 512-edge gather rounds.  Hubs go first, each to all 8
    // wavefronts of the least loaded workgroup (so every wavefront of that
    // workgroup meets the hub's barrier at the same list index); then every
    // other item, longest first, to the least loaded wavefront.  Wavefront w's
    // k-th item sits at position base + k * W + w; wave_cnt[b * W + w] is the
    // length of its list (positions past it are never read).
    {
      auto rounds = [&](int64_t L, int64_t per) { return (double)((L + per - 1) / per); };
      auto cost = [&](const int4 &it) -> double {
        switch (it.x) {
          case kTile: return 1.25;
          case kRows: {
            double c = 0.0;
            for (int r = it.y; r < it.z; ++r) c += rounds(rptr[r + 1] - rptr[r], 512) + 0.25;
            return c;
          }
          case kHeavy: return rounds(std::min<int64_t>(piece, rptr[it.y + 1] - rptr[it.y] - (int64_t)it.z * piece), 512);
          case kZero: return 0.25 + (it.z - it.y) / 512.0;
          default: return 1.0;
        }
      };
      const int G = W / kSweepWaves;
      std::vector<double> load(W, 0.0);
      std::vector<std::vector<int4>> lists(W);
      // hubs, heaviest first, to whole workgroups
      std::vector<int64_t> wgh;
      for (size_t h = 0; h < hubs.size(); ++h)
        if (rptr[hub0 + h + 1] - rptr[hub0 + h] <= wg_max) wgh.push_back(hub0 + (int64_t)h);
      std::stable_sort(wgh.begin(), wgh.end(), [&](int64_t a2, int64_t b2) {
        return rptr[a2 + 1] - rptr[a2] > rptr[b2 + 1] - rptr[b2];
      });
      {
        using E = std::pair<double, int>;
        std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
        for (int q = 0; q < G; ++q) heap.push(E(0.0, q));
        for (int64_t r : wgh) {
          E e = heap.top();
          heap.pop();
          const double c = rounds(rptr[r + 1] - rptr[r], (int64_t)kSweepWaves * 512) + 0.5;
          for (int k = 0; k < kSweepWaves; ++k) {
            lists[e.second * kSweepWaves + k].push_back(make_int4(kHubWG, (int)r, 0, 0));
            load[e.second * kSweepWaves + k] += c;
          }
          heap.push(E(e.first + c, e.second));
        }
      }
      std::vector<int4> other(mega);
      other.insert(other.end(), rest.begin(), rest.end());
      std::vector<double> oc(other.size());
      for (size_t k = 0; k < other.size(); ++k) oc[k] = cost(other[k]);
      std::vector<size_t> ord(other.size());
      for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
      std::stable_sort(ord.begin(), ord.end(), [&](size_t a2, size_t b2) { return oc[a2] > oc[b2]; });
      {
        using E = std::pair<double, int>;
        std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
        for (int w2 = 0; w2 < W; ++w2) heap.push(E(load[w2], w2));
        for (size_t k : ord) {
          E e = heap.top();
          heap.pop();
          lists[e.second].push_back(other[k]);
          heap.push(E(e.first + oc[k], e.second));
        }
      }
      size_t kmax = 0;
      for (auto &l : lists) kmax = std::max(kmax, l.size());
      const size_t base = items.size();
      items.resize(base + kmax * (size_t)W, make_int4(kZero, 0, 0, 0));
      for (int w2 = 0; w2 < W; ++w2) {
        for (size_t k = 0; k < lists[w2].size(); ++k) items[base + k * (size_t)W + w2] = lists[w2][k];
        wave_cnt.push_back((int)lists[w2].size());
      }
    }
    P.block_items.push_back((int)items.size());
  }
  if (want_cl) {
    // contributionList positions: tile edges keep their tidx position, the
    // other lists follow the tiles at their idx position
    P.cl_rows = (uint32_t)(tiles.size() * (size_t)kTileEdges);
    P.cl_size = (int64_t)P.cl_rows + m;
    if (P.cl_size >= INT32_MAX) return pr_fail(PR_EINVAL, "pr_graph_create: contributionList too large");
    for (int64_t r = 0; r < n; ++r) {
      const uint32_t v = rows[r];
      for (int64_t k = 0; k < (int64_t)(ptr[v + 1] - ptr[v]); ++k)
        if (P.inpos[(size_t)(ptr[v] + k)] < 0) P.inpos[(size_t)(ptr[v] + k)] = (int64_t)P.cl_rows + rptr[r] + k;
    }
  }
  P.n_blocks = B;
  for (int b = 0; b + 1 < B; ++b)  // the last block's launch holds the hubs
    if (!bins[(size_t)b * 4].empty()) return pr_fail(PR_EDEVICE, "pr_graph_create: hub outside the last block");
  P.n_items = (int)items.size();
  P.n_bitems = (int)bitems.size();
  P.n_vrun = (int)vrun.size();
  P.n_tiles = (int)tiles.size();
  P.n_heavy = (int)P.n_heavy_rows;
  P.n_split = (int)hsplit.size();
  P.n_msplit = (int)msplit.size();
  P.n_chunks = (int)chunks;

  // host-side check of what the kernels assume
  auto check = [&](const int4 &it) {
    if (it.x == kHeavy)
      return it.y >= 0 && it.y < n && it.w >= 0 && it.w + it.z < chunks &&
             (int64_t)it.z * piece < (int64_t)(rptr[it.y + 1] - rptr[it.y]);
    if (it.x == kHubWG)
      return it.y >= 0 && it.y < n && (int64_t)(rptr[it.y + 1] - rptr[it.y]) > o.chunk &&
             (int64_t)(rptr[it.y + 1] - rptr[it.y]) <= wg_max;
    if (it.x == kRows) return it.y >= 0 && it.y < it.z && it.z <= n;
    if (it.x == kZero) return it.y >= 0 && it.y <= it.z && it.z <= n;
    if (it.x == kTile) {
      const int4 d = tiles[it.y];
      return d.x == it.z && d.y == (it.w >> 16) && d.z == (it.w & 0xffff) &&
             d.x >= 0 && d.y >= 1 && d.y <= kTileRows && d.x + d.y <= n && d.z >= d.y && d.z <= kTileEdges &&
             (int64_t)(rptr[d.x + d.y] - rptr[d.x]) == d.z;
    }
    return false;
  };
  for (const int4 &it : items)
    if (!check(it)) return pr_fail(PR_EDEVICE, "pr_graph_create: internal plan check failed");
  for (const int4 &it : bitems) {
    bool ok;
    if (it.x == kVLong) ok = it.y >= 0 && it.y < n && rptr[it.y + 1] > rptr[it.y];
    else if (it.x == kVQuad) ok = it.y >= 0 && it.z >= 1 && it.z <= 4 && (int64_t)it.y + it.z <= (int64_t)vrun.size();
    else ok = it.x == kHeavy && check(it);
    if (!ok) return pr_fail(PR_EDEVICE, "pr_graph_create: internal plan check failed (batched item)");
  }
  for (const int2 &rr : vrun)
    if (!(rr.x >= 0 && rr.x < rr.y && rr.y <= n))
      return pr_fail(PR_EDEVICE, "pr_graph_create: internal plan check failed (batched run)");
  // every wavefront of a workgroup meets each of its hub items at the same
  // list index
  for (int b = 0; b < B; ++b)
    for (int w2 = 0; w2 < W; ++w2)
      for (int k = 0; k < wave_cnt[(size_t)b * W + w2]; ++k) {
        const int4 &it = items[(size_t)P.block_items[b] + (size_t)k * W + w2];
        if (it.x != kHubWG) continue;
        const int w0 = w2 - w2 % kSweepWaves;
        for (int j = 0; j < kSweepWaves; ++j) {
          const int4 &o2 = items[(size_t)P.block_items[b] + (size_t)k * W + w0 + j];
          if (k >= wave_cnt[(size_t)b * W + w0 + j] || o2.x != kHubWG || o2.y != it.y)
            return pr_fail(PR_EDEVICE, "pr_graph_create: internal plan check failed (hub item)");
        }
      }

  int64_t before = g->device_bytes;
  int rc;
  if ((rc = upload(g, &P.rows, rows.data(), rows.size()))) return rc;
  if ((rc = upload(g, &P.rowpos, rowpos.data(), rowpos.size()))) return rc;
  if ((rc = upload(g, &P.gpos, pos.data(), pos.size()))) return rc;
  if ((rc = upload(g, &P.rptr, rptr.data(), rptr.size()))) return rc;
  if ((rc = upload(g, &P.idx, idx.data(), idx.size()))) return rc;
  if (w && (rc = upload(g, &P.w, wv.data(), wv.size()))) return rc;
  if ((rc = upload(g, &P.items, items.data(), items.size()))) return rc;
  if ((rc = upload(g, &P.bitems, bitems.data(), bitems.size()))) return rc;
  if ((rc = upload(g, &P.wave_cnt, wave_cnt.data(), wave_cnt.size()))) return rc;
  {
    std::vector<int> bpos(P.block_items.begin(), P.block_items.end());
    if ((rc = upload(g, &P.block_pos, bpos.data(), bpos.size()))) return rc;
  }
  if ((rc = upload(g, &P.hsplit, hsplit.data(), hsplit.size()))) return rc;
  if ((rc = upload(g, &P.vrun, vrun.data(), vrun.size()))) return rc;
  if ((rc = upload(g, &P.msplit, msplit.data(), msplit.size()))) return rc;
  if ((rc = upload(g, &P.tiles, tiles.data(), tiles.size()))) return rc;
  if ((rc = upload(g, &P.tidx, tidx.data(), tidx.size()))) return rc;
  if (w && (rc = upload(g, &P.tw, tw.data(), tw.size()))) return rc;
  if ((rc = upload(g, &P.tmask, tmask.data(), tmask.size()))) return rc;
  if ((rc = fpr_dev_alloc(g, (void **)&P.hpart, sizeof(double) * (chunks > 0 ? chunks : 1)))) return rc;
  P.n_waves = W;
  P.part_stride = B * g->grid;  // one partial per sweep workgroup and block
  if ((rc = fpr_dev_alloc(g, (void **)&P.wave_part, sizeof(double) * 3 * (size_t)P.part_stride))) return rc;
  if ((rc = fpr_dev_alloc(g, (void **)&P.st, sizeof(SweepState)))) return rc;
  if (g->mem_mode != kMemCount) PR_HIP(hipMemset(P.st, 0, sizeof(SweepState)));
  if ((rc = fpr_dev_alloc(g, (void **)&P.io, sizeof(IoPtrs)))) return rc;
  if (g->mem_mode != kMemCount) PR_HIP(hipMemset(P.io, 0, sizeof(IoPtrs)));
  P.bytes = g->device_bytes - before;
  return PR_OK;
}

// 64-bit FNV-1a over 8-byte words of the stored graph: n, m, the in-edge
// offsets, neighbours and weights.  Graphs of equal size but different edges
// get different keys for their tuned settings.
static uint64_t graph_signature(const pr_csr *c) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto mix = [&](uint64_t v) { h = (h ^ v) * 0x100000001b3ull; };
  mix((uint64_t)c->n);
  mix((uint64_t)c->m);
  for (int64_t v = 0; v <= c->n; ++v) mix((uint64_t)c->in_ptr[v]);
  for (int64_t e = 0; e < c->m; ++e) mix((uint64_t)(uint32_t)c->in_src[e] | ((uint64_t)e << 32));
  if (c->in_w)
    for (int64_t e = 0; e < c->m; ++e) {
      uint64_t b;
      memcpy(&b, &c->in_w[e], sizeof(b));
      mix(b);
    }
  return h;
}

static void destroy(pr_graph *g) {
  if (!g) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  if (g->work) (void)hipStreamSynchronize(g->work);
  fpr_sweep_release(g);
  fpr_batched_release(g);
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

// pr_graph_create (kMemOwn), the sizing run of pr_graph_device_bytes
// (kMemCount: *out receives a graph holding only the count) and pr_graph_bind
// (kMemArena: the device arrays in the caller's buffer).
static int create_impl(const pr_csr *csr, const pr_plan_opts *opts, int mem_mode, void *arena, size_t arena_bytes,
                       pr_graph **out) {
  if (!out) return pr_fail(PR_EINVAL, "pr_graph_create: out is NULL");
  *out = nullptr;
  if (!csr || !csr->in_ptr || !csr->out_ptr || !csr->out_deg || csr->n < 1 || csr->m < 0 ||
      (csr->m > 0 && (!csr->in_src || !csr->out_dst || !csr->out_to_in)) || (!csr->in_w != !csr->out_w))
    return pr_fail(PR_EINVAL, "pr_graph_create: csr is not a pr_build_csr result");
  if (csr->m > (int64_t)UINT32_MAX - 2)
    return pr_fail(PR_EINVAL, "pr_graph_create: %lld edges exceed the per-graph limit",
                   (long long)csr->m);
  pr_plan_opts o;
  pr_plan_opts_default(&o);
  if (opts) o = *opts;
  if ((o.chunk != 0 && (o.chunk < 64 || o.chunk > (1 << 20))) || o.tile_max_row < 0 || o.tile_max_row > kTileEdges ||
      o.tile_rows < 1 || o.tile_rows > kTileRows || o.steps < 1 || o.steps > 64 || o.gs_blocks < 0 ||
      o.gs_blocks > 64 || o.gather_layout < -1 || o.gather_layout > 2)
    return pr_fail(PR_EINVAL,
                   "pr_graph_create: need chunk = 0 or 64 <= chunk <= 2^20, 0 <= tile_max_row <= 512, "
                   "1 <= tile_rows <= 128, 1 <= steps <= 64, 0 <= gs_blocks <= 64, gather_layout 0..2");
  {
    // the plan indexes with these arrays: offsets must be a monotone cover of
    // [0, m] and every id must be a vertex, else the graph is refused
    const int64_t n = csr->n, m = csr->m;
    if (csr->in_ptr[0] != 0 || csr->in_ptr[n] != m || csr->out_ptr[0] != 0 || csr->out_ptr[n] != m)
      return pr_fail(PR_EINVAL, "pr_graph_create: in_ptr / out_ptr do not span [0, m]");
    for (int64_t v = 0; v < n; ++v) {
      if (csr->in_ptr[v + 1] < csr->in_ptr[v] || csr->out_ptr[v + 1] < csr->out_ptr[v])
        return pr_fail(PR_EINVAL, "pr_graph_create: decreasing offsets at vertex %lld", (long long)v);
      if (csr->out_deg[v] != csr->out_ptr[v + 1] - csr->out_ptr[v])
        return pr_fail(PR_EINVAL, "pr_graph_create: out_deg[%lld] disagrees with out_ptr", (long long)v);
    }
    for (int64_t e = 0; e < m; ++e)
      if ((uint32_t)csr->in_src[e] >= (uint64_t)n || (uint32_t)csr->out_dst[e] >= (uint64_t)n)
        return pr_fail(PR_EINVAL, "pr_graph_create: edge %lld names a vertex outside [0, n)", (long long)e);
  }
  int dev_count = 0;
  hipError_t he = hipGetDeviceCount(&dev_count);
  if (he != hipSuccess || dev_count < 1)
    return pr_fail(PR_EDEVICE, "pr_graph_create: no HIP device (%s)", hipGetErrorString(he));

  pr_graph *g = new pr_graph();
  g->mem_mode = mem_mode;
  g->arena = static_cast<unsigned char *>(arena);
  g->arena_bytes = arena_bytes;
  g->popts = o;
  g->n = csr->n;
  g->m = csr->m;
  g->weighted = csr->in_w != nullptr;
  g->signature = graph_signature(csr);
  int rc = PR_OK;
  hipDeviceProp_t prop;
  if (hipGetDevice(&g->device) != hipSuccess || hipGetDeviceProperties(&prop, g->device) != hipSuccess) {
    destroy(g);
    return pr_fail(PR_EDEVICE, "pr_graph_create: cannot query the current device");
  }
  g->n_cu = prop.multiProcessorCount;
  g->grid = fpr_grid_for(g);
  if (o.chunk == 0) {
    // hubs start at about the average edge share of one sweep wavefront
    // (a power of two in [1024, 16384]): a longer list on one wavefront would
    // be the launch's critical path
    const int64_t W = (int64_t)g->grid * kSweepWaves;
    int64_t c = 1024;
    while (c < 16384 && 2 * c <= csr->m / W) c *= 2;
    o.chunk = (int)c;
  }
  o.tile_max_row = std::min(o.tile_max_row, o.chunk);
  {
    // share of in-edges whose source id lies within kLocalSpan of the
    // destination's: the input's own order already groups the sources of
    // neighbouring rows
    int64_t near = 0;
    for (int64_t u = 0; u < csr->n; ++u)
      for (int64_t e = csr->in_ptr[u]; e < csr->in_ptr[u + 1]; ++e) {
        const int64_t dv = (int64_t)csr->in_src[e] - u;
        near += (dv < kLocalSpan && dv > -kLocalSpan) ? 1 : 0;
      }
    g->local_share = csr->m > 0 ? (double)near / (double)csr->m : 0.0;
  }
  // local: a quarter of the in-edges or more, and at least four times the
  // share a random labeling gives (about 2 kLocalSpan / n)
  const double random_share = std::min(1.0, (double)(2 * kLocalSpan - 1) / (double)csr->n);
  const bool local = g->local_share >= 0.25 && g->local_share >= 4.0 * random_share;
  if (o.gather_layout < 0) o.gather_layout = local ? 2 : 1;
  if (o.gs_blocks == 0 && local) o.gs_blocks = 1;
  if (o.gs_blocks == 0) {
    // Each block costs a launch (ramp and tail, about 10 us) and saves
    // sweeps; the longer a sweep, the more blocks pay off.  By edges per
    // sweep wavefront: under 64 one block, under 6144 two (R-MAT-20), under
    // 49152 three (R-MAT-21 to 23), else eight (R-MAT-24), the fastest
    // measured counts at those sizes.
    const int64_t epw = csr->m / ((int64_t)g->grid * kSweepWaves);
    o.gs_blocks = epw < 64 ? 1 : epw < 6144 ? 2 : epw < 49152 ? 3 : 8;
  }
  g->popts = o;
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
    if ((rc2 = build_plan(g, g->fwd, n, csr->in_ptr, csr->in_src, csr->in_w, o, o.with_cl != 0))) return rc2;
    if (o.with_cl) {
      // out-edge order: source, list position and weight of every edge
      const int64_t m = csr->m;
      std::vector<int32_t> src((size_t)m), pos((size_t)m);
      std::vector<double> wv(csr->in_w ? (size_t)m : 0);
      for (int64_t v = 0; v < n; ++v)
        for (int64_t e = csr->out_ptr[v]; e < csr->out_ptr[v + 1]; ++e) {
          const int64_t ie = csr->out_to_in[e];
          if (ie < 0 || ie >= m)
            return pr_fail(PR_EINVAL, "pr_graph_create: out_to_in[%lld] = %lld is not an in-edge position",
                           (long long)e, (long long)ie);
          const int64_t p = g->fwd.inpos[(size_t)ie];
          if (p < 0 || p >= g->fwd.cl_size)
            return pr_fail(PR_EDEVICE, "pr_graph_create: internal plan check failed (list position)");
          src[(size_t)e] = (int32_t)v;
          pos[(size_t)e] = (int32_t)p;
          if (csr->in_w) wv[(size_t)e] = csr->in_w[ie];
        }
      std::vector<int64_t>().swap(g->fwd.inpos);
      // grouped by the launch that updates the source (stable, so out-edge
      // order inside a group): the loop-fused list form scatters group b
      // right after block b's launch, the split hubs' group after the
      // finalize kernel
      {
        const int B = g->fwd.n_blocks;
        const std::vector<uint8_t> &ul = g->fwd.upd_launch;
        std::vector<int64_t> off(B + 2, 0);
        for (int64_t e = 0; e < m; ++e) off[ul[(size_t)src[(size_t)e]] + 1]++;
        for (int b = 0; b <= B; ++b) off[b + 1] += off[b];
        g->fwd.cl_group = off;
        std::vector<int32_t> s2((size_t)m), p2((size_t)m);
        std::vector<double> w2(wv.size());
        for (int64_t e = 0; e < m; ++e) {
          const int64_t at = off[ul[(size_t)src[(size_t)e]]]++;
          s2[(size_t)at] = src[(size_t)e];
          p2[(size_t)at] = pos[(size_t)e];
          if (!wv.empty()) w2[(size_t)at] = wv[(size_t)e];
        }
        src.swap(s2);
        pos.swap(p2);
        wv.swap(w2);
        std::vector<uint8_t>().swap(g->fwd.upd_launch);
      }
      if ((rc2 = upload(g, &g->fwd.cl_src, src.data(), src.size()))) return rc2;
      if ((rc2 = upload(g, &g->fwd.cl_pos, pos.data(), pos.size()))) return rc2;
      if (csr->in_w && (rc2 = upload(g, &g->fwd.cl_w, wv.data(), wv.size()))) return rc2;
    }
    if (o.with_inplace) {
      // the canonical in-lists, rows and sources renumbered by position:
      // inside a full block of kIpVpb vertices, vertex b0 + l * kIpRun + k
      // sits at position b0 + 64 k + l; the last, partial block keeps
      // vertex order
      std::vector<uint32_t> pos(n), vert(n);
      for (int64_t b0 = 0; b0 < n; b0 += kIpVpb) {
        const int64_t nb = std::min<int64_t>(kIpVpb, n - b0);
        for (int64_t i = 0; i < nb; ++i) {
          const int64_t v = nb == kIpVpb ? b0 + (i % 64) * kIpRun + i / 64 : b0 + i;
          pos[v] = (uint32_t)(b0 + i);
          vert[b0 + i] = (uint32_t)v;
        }
      }
      std::vector<uint32_t> ip(n + 1);
      std::vector<int32_t> isrc((size_t)csr->m);
      std::vector<double> iwt(csr->in_w ? (size_t)csr->m : 0), iiw(n);
      ip[0] = 0;
      for (int64_t q = 0; q < n; ++q) {
        const int64_t v = vert[q];
        uint32_t at = ip[q];
        for (int64_t e = csr->in_ptr[v]; e < csr->in_ptr[v + 1]; ++e, ++at) {
          isrc[at] = (int32_t)pos[csr->in_src[e]];
          if (csr->in_w) iwt[at] = csr->in_w[e];
        }
        ip[q + 1] = at;
        iiw[q] = inv_w[v];
      }
      if ((rc2 = upload(g, &g->fwd.ip_ptr, ip.data(), ip.size()))) return rc2;
      if ((rc2 = upload(g, &g->fwd.ip_src, isrc.data(), isrc.size()))) return rc2;
      if (csr->in_w && (rc2 = upload(g, &g->fwd.ip_w, iwt.data(), iwt.size()))) return rc2;
      if ((rc2 = upload(g, &g->fwd.ip_pos, pos.data(), pos.size()))) return rc2;
      if ((rc2 = upload(g, &g->fwd.ip_iw, iiw.data(), iiw.size()))) return rc2;
      // each sweep wavefront takes a contiguous range of blocks of about equal
      // cost (in-edges, plus two per vertex for the update), in ascending order
      {
        const int64_t nblocks = (n + kIpVpb - 1) / kIpVpb;
        const int64_t W = (int64_t)g->grid * kSweepWaves;
        std::vector<double> cum(nblocks + 1, 0.0);
        for (int64_t b = 0; b < nblocks; ++b) {
          const int64_t lo = b * kIpVpb, hi = std::min<int64_t>(n, lo + kIpVpb);
          cum[b + 1] = cum[b] + (double)(ip[hi] - ip[lo]) + 2.0 * (double)(hi - lo);
        }
        std::vector<int32_t> range(W + 1);
        int64_t b = 0;
        for (int64_t w2 = 0; w2 <= W; ++w2) {
          const double target = cum[nblocks] * (double)w2 / (double)W;
          while (b < nblocks && cum[b] < target) ++b;
          range[w2] = (int32_t)b;
        }
        range[W] = (int32_t)nblocks;
        if ((rc2 = upload(g, &g->fwd.ip_range, range.data(), range.size()))) return rc2;
      }
    }
    if (o.with_adjoint) {
      if ((rc2 = build_plan(g, g->adj, n, csr->out_ptr, csr->out_dst, csr->out_w, o, false))) return rc2;
      std::vector<uint32_t> op(n + 1);
      for (int64_t v = 0; v <= n; ++v) op[v] = (uint32_t)csr->out_ptr[v];
      if ((rc2 = upload(g, &g->out_ptr, op.data(), op.size()))) return rc2;
      if ((rc2 = upload(g, &g->out_dst, csr->out_dst, (size_t)csr->m))) return rc2;
      if (csr->out_w && (rc2 = upload(g, &g->out_w, csr->out_w, (size_t)csr->m))) return rc2;
      g->has_adj = true;
    }
    if ((rc2 = fpr_dev_alloc(g, (void **)&g->red_tmp, sizeof(double) * 4096))) return rc2;
    if (g->mem_mode == kMemCount) return PR_OK;  // sizes only: no stream, events or pinned state
    if (hipStreamCreateWithFlags(&g->work, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&g->host_st, sizeof(SweepState)) != hipSuccess)
      return pr_fail(PR_EDEVICE, "pr_graph_create: stream/event/pinned allocation failed");
    return PR_OK;
  }();
  if (rc != PR_OK) {
    destroy(g);
    return rc;
  }
  // later (lazy) workspace allocations of a bound graph are the library's own
  if (mem_mode == kMemArena) g->mem_mode = kMemOwn;
  *out = g;
  return PR_OK;
}

extern "C" int pr_graph_create(const pr_csr *csr, const pr_plan_opts *opts, pr_graph **out) {
  pr_clear_error();
  return create_impl(csr, opts, kMemOwn, nullptr, 0, out);
}

extern "C" int pr_graph_device_bytes(const pr_csr *csr, const pr_plan_opts *opts, size_t *bytes) {
  pr_clear_error();
  if (!bytes) return pr_fail(PR_EINVAL, "pr_graph_device_bytes: bytes is NULL");
  pr_graph *g = nullptr;
  int rc = create_impl(csr, opts, kMemCount, nullptr, 0, &g);
  if (rc != PR_OK) return rc;
  *bytes = g->arena_used;
  g->owned.clear();
  destroy(g);
  return PR_OK;
}

extern "C" int pr_graph_bind(const pr_csr *csr, const pr_plan_opts *opts, void *dev_mem, size_t bytes,
                             pr_graph **out) {
  pr_clear_error();
  if (!dev_mem || ((uintptr_t)dev_mem & 255) != 0)
    return pr_fail(PR_EINVAL, "pr_graph_bind: dev_mem must be a 256-byte aligned device pointer");
  hipPointerAttribute_t attr;
  const hipError_t pe = hipPointerGetAttributes(&attr, dev_mem);
  (void)hipGetLastError();  // a pointer HIP does not know leaves an error behind: clear it
  if (pe != hipSuccess || attr.type != hipMemoryTypeDevice)
    return pr_fail(PR_EINVAL, "pr_graph_bind: dev_mem is not device memory");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || attr.device != cur)
    return pr_fail(PR_EINVAL, "pr_graph_bind: dev_mem lives on device %d, device %d is current", attr.device, cur);
  return create_impl(csr, opts, kMemArena, dev_mem, bytes, out);
}

extern "C" void pr_graph_free(pr_graph *g) { destroy(g); }

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
  s->gs_blocks = g->fwd.n_blocks;
  s->chunk = g->fwd.chunk;
  s->graph_captures = g->graph_captures;
  s->signature = g->signature;
  s->local_share = g->local_share;
  s->gather_layout = g->popts.gather_layout;
  return PR_OK;
}
