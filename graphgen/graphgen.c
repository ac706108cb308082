/*
 * graphgen.c -- seeded synthetic graph inputs.
 *
 * This module produces INPUTS only: edge lists, vertex permutations, edge
 * weights and seed vertices.  It holds none of the PageRank arithmetic, and
 * both the CPU oracle and the GPU library consume what it writes.
 *
 * Random numbers come from one counter-based generator, SplitMix64
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): the i-th output (i = 0, 1, ...) of a stream whose key is K is
 *     mix64(K + (i + 1) * 0x9E3779B97F4A7C15)
 * with mix64 the SplitMix64 finaliser.  A stream key is derived from the user
 * seed and a stream number as  K(seed, stream) = mix64(mix64(seed + G) ^ (stream * C)).
 * A uniform double in [0, 1) is (u64 >> 11) * 2^-53.
 *
 * Generators
 *   - Erdos-Renyi G(n, m): ordered pairs (src, dst) drawn uniformly from
 *     stream 1 (src from output 2i, dst from output 2i+1); self-loops and
 *     repeated pairs are rejected until exactly m distinct edges exist.
 *   - R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004; the generator behind the
 *     paper's synthetic graphs, Section 6.2): per edge e and level l (most
 *     significant bit first) one uniform u = U(stream 1, e*scale + l) picks a
 *     quadrant: u < a -> (0,0); u < a+b -> (src 0, dst 1); u < a+b+c ->
 *     (src 1, dst 0); else (1,1).  No noise.
 *   - Fisher-Yates permutation from stream 2: for i = n-1 .. 1, the
 *     (n-1-i)-th uniform u picks j = floor(u * (i+1)) and swaps p[i], p[j].
 *   - Deduplication: sort by (src, dst), drop repeats and self-loops.
 *   - BFS relabel on the undirected view: start at the vertex of largest
 *     total degree (smallest id on ties), visit neighbours in ascending id,
 *     restart at the smallest unvisited id when the queue empties.
 *   - Weights: w_i = lo + (hi - lo) * U(stream, i).
 *   - Distinct sample of k vertices: draws floor(U * n) in order, skipping repeats.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL
#define GG_STREAM_MUL 0xD1B54A32D192ED03ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed + GG_GAMMA) ^ (stream * GG_STREAM_MUL));
}

static inline uint64_t gg_u64(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GG_GAMMA); }

static inline double gg_unif(uint64_t key, uint64_t i) {
  return (double)(gg_u64(key, i) >> 11) * (1.0 / 9007199254740992.0);
}

/* Raw 64-bit output i of the stream with key `key` (pins the published SplitMix64 sequence). */
uint64_t gg_raw(uint64_t key, uint64_t i) { return gg_u64(key, i); }

/* First `count` outputs of stream (seed, stream) as uniforms; lets tests pin the generator. */
void gg_uniforms(uint64_t seed, uint64_t stream, int64_t count, double *out) {
  uint64_t key = gg_stream_key(seed, stream);
  for (int64_t i = 0; i < count; ++i) out[i] = gg_unif(key, (uint64_t)i);
}

static inline int32_t gg_pick(uint64_t key, uint64_t i, int64_t n) {
  int64_t v = (int64_t)(gg_unif(key, i) * (double)n);
  return (int32_t)(v >= n ? n - 1 : v);
}

/* ---------------------------------------------------------------- ER ---- */
/* Returns 0 on success, -1 if m is not attainable. */
int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t *src, int32_t *dst) {
  if (n < 2 || m < 0 || m > n * (n - 1)) return -1;
  uint64_t cap = 16;
  while (cap < (uint64_t)(4 * m + 16)) cap <<= 1;
  uint64_t *table = (uint64_t *)malloc(cap * sizeof(uint64_t));
  if (!table) return -1;
  const uint64_t EMPTY = ~0ULL;
  for (uint64_t i = 0; i < cap; ++i) table[i] = EMPTY;
  uint64_t key = gg_stream_key(seed, 1);
  int64_t got = 0;
  for (uint64_t draw = 0; got < m; ++draw) {
    int32_t s = gg_pick(key, 2 * draw, n);
    int32_t t = gg_pick(key, 2 * draw + 1, n);
    if (s == t) continue;
    uint64_t k = (uint64_t)s * (uint64_t)n + (uint64_t)t;
    uint64_t h = mix64(k) & (cap - 1);
    int dup = 0;
    while (table[h] != EMPTY) {
      if (table[h] == k) { dup = 1; break; }
      h = (h + 1) & (cap - 1);
    }
    if (dup) continue;
    table[h] = k;
    src[got] = s;
    dst[got] = t;
    ++got;
  }
  free(table);
  return 0;
}

/* -------------------------------------------------------------- R-MAT --- */
void gg_rmat(int scale, int64_t m, double a, double b, double c, uint64_t seed,
             int32_t *src, int32_t *dst) {
  uint64_t key = gg_stream_key(seed, 1);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t s = 0, t = 0;
    uint64_t base = (uint64_t)e * (uint64_t)scale;
    for (int l = 0; l < scale; ++l) {
      double u = gg_unif(key, base + (uint64_t)l);
      uint32_t sb, tb;
      if (u < a) { sb = 0; tb = 0; }
      else if (u < ab) { sb = 0; tb = 1; }
      else if (u < abc) { sb = 1; tb = 0; }
      else { sb = 1; tb = 1; }
      s = (s << 1) | sb;
      t = (t << 1) | tb;
    }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)t;
  }
}

/* ------------------------------------------------------- permutation --- */
void gg_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
  uint64_t key = gg_stream_key(seed, stream);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i >= 1; --i) {
    int64_t j = (int64_t)(gg_unif(key, (uint64_t)(n - 1 - i)) * (double)(i + 1));
    if (j > i) j = i;
    int32_t tmp = perm[i];
    perm[i] = perm[j];
    perm[j] = tmp;
  }
}

void gg_relabel(int64_t m, const int32_t *label, int32_t *src, int32_t *dst) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    src[e] = label[src[e]];
    dst[e] = label[dst[e]];
  }
}

/* ------------------------------------------------ parallel radix sort --- */
/* Stable LSD radix sort of 64-bit keys, 16-bit digits, only the digits
 * needed for keys below 2^bits.  Sorted keys end in `keys`. */
static int radix_sort_u64(uint64_t *keys, int64_t cnt, int bits) {
  if (cnt <= 1) return 0;
  uint64_t *tmp = (uint64_t *)malloc((size_t)cnt * sizeof(uint64_t));
  if (!tmp) return -1;
  int nthr = omp_get_max_threads();
  if (nthr > 64) nthr = 64;
  const int R = 1 << 16;
  int64_t *hist = (int64_t *)calloc((size_t)nthr * R, sizeof(int64_t));
  if (!hist) { free(tmp); return -1; }
  uint64_t *in = keys, *out = tmp;
  int passes = (bits + 15) / 16;
  for (int p = 0; p < passes; ++p) {
    int shift = 16 * p;
    memset(hist, 0, (size_t)nthr * R * sizeof(int64_t));
#pragma omp parallel num_threads(nthr)
    {
      int t = omp_get_thread_num();
      int nt = omp_get_num_threads();
      int64_t lo = cnt * t / nt, hi = cnt * (t + 1) / nt;
      int64_t *h = hist + (size_t)t * R;
      for (int64_t i = lo; i < hi; ++i) h[(in[i] >> shift) & 0xFFFF]++;
#pragma omp barrier
#pragma omp single
      {
        int64_t run = 0;
        for (int dgt = 0; dgt < R; ++dgt)
          for (int tt = 0; tt < nt; ++tt) {
            int64_t v = hist[(size_t)tt * R + dgt];
            hist[(size_t)tt * R + dgt] = run;
            run += v;
          }
      }
      for (int64_t i = lo; i < hi; ++i) {
        uint64_t k = in[i];
        out[h[(k >> shift) & 0xFFFF]++] = k;
      }
    }
    uint64_t *sw = in; in = out; out = sw;
  }
  if (in != keys) memcpy(keys, in, (size_t)cnt * sizeof(uint64_t));
  free(hist);
  free(tmp);
  return 0;
}

static int bits_for(uint64_t maxv) {
  int b = 1;
  while (b < 64 && (maxv >> b) != 0) ++b;
  return b;
}

/* Sort edges by (src, dst), drop self-loops and repeats, in place.
 * Returns the new edge count, or -1 on allocation failure. */
int64_t gg_dedup(int64_t n, int64_t m, int32_t *src, int32_t *dst) {
  uint64_t *keys = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  if (!keys) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) keys[e] = (uint64_t)src[e] * (uint64_t)n + (uint64_t)dst[e];
  uint64_t maxk = (uint64_t)n * (uint64_t)n;
  if (radix_sort_u64(keys, m, bits_for(maxk)) != 0) { free(keys); return -1; }
  int64_t out = 0;
  for (int64_t e = 0; e < m; ++e) {
    uint64_t k = keys[e];
    if (e > 0 && k == keys[e - 1]) continue;
    int32_t s = (int32_t)(k / (uint64_t)n), t = (int32_t)(k % (uint64_t)n);
    if (s == t) continue;
    src[out] = s;
    dst[out] = t;
    ++out;
  }
  free(keys);
  return out;
}

/* ---------------------------------------------------- BFS relabel ------ */
/* Input: edges sorted by (src, dst), distinct, no self-loops (gg_dedup output).
 * Output: label[v] = BFS visit index of v on the undirected view. */
int gg_bfs_order(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *label) {
  int64_t *optr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *iptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *isrc = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!optr || !iptr || !isrc || !queue) {
    free(optr); free(iptr); free(isrc); free(queue);
    return -1;
  }
  for (int64_t e = 0; e < m; ++e) {
    optr[src[e] + 1]++;
    iptr[dst[e] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) {
    optr[v + 1] += optr[v];
    iptr[v + 1] += iptr[v];
  }
  /* stable scatter by dst: edges arrive in ascending src, so each in-list is ascending */
  {
    int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!fill) { free(optr); free(iptr); free(isrc); free(queue); return -1; }
    memcpy(fill, iptr, (size_t)n * sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) isrc[fill[dst[e]]++] = src[e];
    free(fill);
  }
  for (int64_t v = 0; v < n; ++v) label[v] = -1;
  int64_t start = 0, best = -1;
  for (int64_t v = 0; v < n; ++v) {
    int64_t deg = (optr[v + 1] - optr[v]) + (iptr[v + 1] - iptr[v]);
    if (deg > best) { best = deg; start = v; }
  }
  int64_t head = 0, tail = 0, next_label = 0, scan = 0;
  int64_t root = start;
  while (next_label < n) {
    if (root < 0) {
      while (scan < n && label[scan] >= 0) ++scan;
      root = scan;
    }
    label[root] = (int32_t)next_label++;
    queue[tail++] = (int32_t)root;
    root = -1;
    while (head < tail) {
      int32_t v = queue[head++];
      /* merge ascending out-neighbours and ascending in-neighbours */
      int64_t a = optr[v], ae = optr[v + 1], b = iptr[v], be = iptr[v + 1];
      while (a < ae || b < be) {
        int32_t u;
        if (b >= be || (a < ae && dst[a] <= isrc[b])) u = dst[a++];
        else u = isrc[b++];
        if (label[u] < 0) {
          label[u] = (int32_t)next_label++;
          queue[tail++] = u;
        }
      }
    }
  }
  free(optr); free(iptr); free(isrc); free(queue);
  return 0;
}

/* ----------------------------------------------------------- values --- */
void gg_weights(int64_t m, uint64_t seed, uint64_t stream, double lo, double hi, double *w) {
  uint64_t key = gg_stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) w[i] = lo + (hi - lo) * gg_unif(key, (uint64_t)i);
}

/* k distinct vertices in [0, n), in draw order.  Returns 0, or -1 if k > n. */
int gg_sample_distinct(int64_t n, int64_t k, uint64_t seed, uint64_t stream, int32_t *out) {
  if (k > n || k < 0) return -1;
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  if (!seen) return -1;
  uint64_t key = gg_stream_key(seed, stream);
  int64_t got = 0;
  for (uint64_t i = 0; got < k; ++i) {
    int32_t v = gg_pick(key, i, n);
    if (seen[v]) continue;
    seen[v] = 1;
    out[got++] = v;
  }
  free(seen);
  return 0;
}
