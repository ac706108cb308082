"""Seeded synthetic graph inputs shared by the CPU oracle, the GPU library's
tests and the benchmark.

This package only produces inputs (edge lists, permutations, weights, seed
vertices); it holds none of the PageRank arithmetic.  The heavy lifting is in
``graphgen.c`` (counter-based SplitMix64 streams, R-MAT, Fisher-Yates, radix
dedup, BFS relabel), compiled with gcc into ``_graphgen.so`` next to it.

Stream numbers used by the named workloads: 1 = edge endpoints, 2 = vertex
permutation, 3 = edge weights, 4 = sampled vertices (seeds, loss targets).

The named workloads mirror the paper's inputs (Section 6.2, Table 3): R-MAT
graphs from the Graph500-style generator it cites stand in for its web and
social graphs, with randomly permuted ids (locality-free, social-graph-like)
or BFS order (web-crawl-like locality).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_SO = os.path.join(_HERE, "_graphgen.so")
_LIB = None

STREAM_EDGES = 1
STREAM_PERM = 2
STREAM_WEIGHTS = 3
STREAM_SAMPLE = 4

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = True) -> str:
    """Compile graphgen.c into _graphgen.so (gcc, OpenMP)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_SO)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i64, u64, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.gg_er.argtypes = [i64, i64, u64, i32p, i32p]
    lib.gg_er.restype = ctypes.c_int
    lib.gg_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, i32p, i32p]
    lib.gg_rmat.restype = None
    lib.gg_permutation.argtypes = [i64, u64, u64, i32p]
    lib.gg_permutation.restype = None
    lib.gg_relabel.argtypes = [i64, i32p, i32p, i32p]
    lib.gg_relabel.restype = None
    lib.gg_dedup.argtypes = [i64, i64, i32p, i32p]
    lib.gg_dedup.restype = i64
    lib.gg_bfs_order.argtypes = [i64, i64, i32p, i32p, i32p]
    lib.gg_bfs_order.restype = ctypes.c_int
    lib.gg_weights.argtypes = [i64, u64, u64, dbl, dbl, f64p]
    lib.gg_weights.restype = None
    lib.gg_sample_distinct.argtypes = [i64, i64, u64, u64, i32p]
    lib.gg_sample_distinct.restype = ctypes.c_int
    lib.gg_uniforms.argtypes = [u64, u64, i64, f64p]
    lib.gg_uniforms.restype = None
    lib.gg_stream_key.argtypes = [u64, u64]
    lib.gg_stream_key.restype = u64
    lib.gg_raw.argtypes = [u64, u64]
    lib.gg_raw.restype = u64
    _LIB = lib
    return lib


# ----------------------------------------------------------------- basics --

def raw(key: int, i: int) -> int:
    return int(_lib().gg_raw(key, i))


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.empty(count, np.float64)
    _lib().gg_uniforms(seed, stream, count, out)
    return out


def er(n: int, m: int, seed: int):
    """Directed G(n, m): exactly m distinct edges, no self-loops."""
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    if _lib().gg_er(n, m, seed, src, dst) != 0:
        raise ValueError("G(n=%d, m=%d) cannot be drawn" % (n, m))
    return src, dst


def permutation(n: int, seed: int, stream: int = STREAM_PERM) -> np.ndarray:
    perm = np.empty(n, np.int32)
    _lib().gg_permutation(n, seed, stream, perm)
    return perm


def relabel(label: np.ndarray, src: np.ndarray, dst: np.ndarray):
    src = np.ascontiguousarray(src, np.int32).copy()
    dst = np.ascontiguousarray(dst, np.int32).copy()
    _lib().gg_relabel(len(src), np.ascontiguousarray(label, np.int32), src, dst)
    return src, dst


def rmat(scale: int, edge_factor: int = 16, seed: int = 0, a: float = RMAT_A, b: float = RMAT_B,
         c: float = RMAT_C, permute: bool = True):
    """Raw R-MAT edge list (repeats and self-loops kept), ids optionally permuted."""
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _lib().gg_rmat(scale, m, a, b, c, seed, src, dst)
    if permute:
        perm = permutation(n, seed, STREAM_PERM)
        _lib().gg_relabel(m, perm, src, dst)
    return src, dst


def dedup(n: int, src: np.ndarray, dst: np.ndarray):
    """Distinct, self-loop-free edges sorted by (src, dst)."""
    src = np.ascontiguousarray(src, np.int32).copy()
    dst = np.ascontiguousarray(dst, np.int32).copy()
    m2 = _lib().gg_dedup(n, len(src), src, dst)
    if m2 < 0:
        raise MemoryError("gg_dedup")
    return src[:m2].copy(), dst[:m2].copy()


def bfs_labels(n: int, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """BFS visit order on the undirected view (input must come from dedup())."""
    label = np.empty(n, np.int32)
    if _lib().gg_bfs_order(n, len(src), np.ascontiguousarray(src, np.int32),
                           np.ascontiguousarray(dst, np.int32), label) != 0:
        raise MemoryError("gg_bfs_order")
    return label


def weights(m: int, seed: int, stream: int = STREAM_WEIGHTS, lo: float = 0.5, hi: float = 1.5):
    w = np.empty(m, np.float64)
    _lib().gg_weights(m, seed, stream, lo, hi, w)
    return w


def sample_distinct(n: int, k: int, seed: int, stream: int = STREAM_SAMPLE) -> np.ndarray:
    out = np.empty(k, np.int32)
    if _lib().gg_sample_distinct(n, k, seed, stream, out) != 0:
        raise ValueError("cannot sample %d distinct of %d" % (k, n))
    return out


# ------------------------------------------------------ named workloads ---

def er_10k():
    """Directed Erdos-Renyi, n=10,000, exactly 80,000 distinct edges, seed 1."""
    n = 10_000
    src, dst = er(n, 80_000, seed=1)
    return dict(name="er-10k", n=n, src=src, dst=dst)


def rmat_permuted(scale: int, seed: int, edge_factor: int = 16):
    """R-MAT (a=.57, b=c=.19), ids randomly permuted; raw list (repeats kept)."""
    n = 1 << scale
    src, dst = rmat(scale, edge_factor, seed=seed, permute=True)
    return dict(name="rmat%d-perm" % scale, n=n, src=src, dst=dst)


def rmat20():
    """R-MAT scale 20, edge factor 16, seed 2, permuted ids."""
    return rmat_permuted(20, seed=2)


def ppr_seeds(n: int, k: int = 64, seed: int = 3) -> np.ndarray:
    """k distinct one-hot seed vertices drawn uniformly (seed 3 for the k=64 batch)."""
    return sample_distinct(n, k, seed, STREAM_SAMPLE)


def rmat_weighted(scale: int, seed: int, n_targets: int = 1024, edge_factor: int = 16):
    """Weighted R-MAT: deduplicated canonical (src, dst) order, weights U[0.5, 1.5]
    assigned in that order, plus loss targets drawn without replacement."""
    n = 1 << scale
    src, dst = rmat(scale, edge_factor, seed=seed, permute=True)
    src, dst = dedup(n, src, dst)
    w = weights(len(src), seed, STREAM_WEIGHTS, 0.5, 1.5)
    targets = sample_distinct(n, n_targets, seed, STREAM_SAMPLE)
    return dict(name="rmat%d-weighted" % scale, n=n, src=src, dst=dst, w=w, targets=targets)


def rmat18_weighted():
    return rmat_weighted(18, seed=4)


def rmat_bfs(scale: int, seed: int, edge_factor: int = 16):
    """R-MAT, deduplicated, then relabelled in BFS order (web-crawl-like locality)."""
    n = 1 << scale
    src, dst = rmat(scale, edge_factor, seed=seed, permute=True)
    src, dst = dedup(n, src, dst)
    label = bfs_labels(n, src, dst)
    _lib().gg_relabel(len(src), label, src, dst)
    return dict(name="rmat%d-bfs" % scale, n=n, src=src, dst=dst)


def rmat24_bfs():
    return rmat_bfs(24, seed=5)


# ------------------------------------------------- small shaped graphs ---

def road_grid(side: int, seed: int, keep: float = 0.75, one_way: float = 0.1):
    """Road-network-shaped graph: a side x side street grid, vertex r * side + c
    (row-major ids, so grid neighbours are near in id).  Each grid segment is
    kept with probability `keep`; a kept segment is one-way with probability
    `one_way` (direction chosen by a fair coin), else two-way.  Low degree (about
    2.8 out-edges per vertex), no hubs, diameter about 2 * side.  Stream 1
    draws three uniforms per candidate segment, right segments first, then down
    segments, in vertex order."""
    n = side * side
    r, c = np.divmod(np.arange(n, dtype=np.int64), side)
    right = np.nonzero(c + 1 < side)[0]
    down = np.nonzero(r + 1 < side)[0]
    a = np.concatenate([right, down])
    b = np.concatenate([right + 1, down + side])
    u = uniforms(seed, STREAM_EDGES, 3 * len(a))
    kept = u[0::3] < keep
    oneway = u[1::3] < one_way
    fwd = u[2::3] < 0.5
    a, b, oneway, fwd = a[kept], b[kept], oneway[kept], fwd[kept]
    both = ~oneway
    src = np.concatenate([a[both], b[both], np.where(fwd[oneway], a[oneway], b[oneway])])
    dst = np.concatenate([b[both], a[both], np.where(fwd[oneway], b[oneway], a[oneway])])
    return src.astype(np.int32), dst.astype(np.int32)


def road8m():
    """The road-network stand-in of the benchmark: a 2896 x 2896 grid (8.4 M
    vertices), seed 6."""
    src, dst = road_grid(2896, seed=6)
    return dict(name="road8m", n=2896 * 2896, src=src, dst=dst)


def cycle(n: int):
    s = np.arange(n, dtype=np.int32)
    return s, ((s + 1) % n).astype(np.int32)


def complete(n: int):
    s, t = np.meshgrid(np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), indexing="ij")
    keep = s != t
    return s[keep].astype(np.int32), t[keep].astype(np.int32)


def in_star(n: int):
    """Leaves 1..n-1 point to hub 0."""
    leaves = np.arange(1, n, dtype=np.int32)
    return leaves, np.zeros(n - 1, np.int32)


def out_star(n: int):
    """Hub 0 points to leaves 1..n-1."""
    leaves = np.arange(1, n, dtype=np.int32)
    return np.zeros(n - 1, np.int32), leaves


def bi_star(n: int):
    a, b = in_star(n)
    c, d = out_star(n)
    return np.concatenate([a, c]), np.concatenate([b, d])


def path(n: int):
    s = np.arange(n - 1, dtype=np.int32)
    return s, s + 1


def random_dag(n: int, m: int, seed: int):
    """Edges only from lower to higher id (ids are a topological order)."""
    u = uniforms(seed, STREAM_EDGES, 2 * m)
    a = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
    b = np.minimum((u[1::2] * n).astype(np.int64), n - 1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keep = lo != hi
    return lo[keep].astype(np.int32), hi[keep].astype(np.int32)


def random_graph(n: int, m: int, seed: int, self_loops: bool = True):
    """Uniform multigraph draw (repeats and, optionally, self-loops kept) for
    exercising the CSR builder's deduplication."""
    u = uniforms(seed, STREAM_EDGES, 2 * m)
    a = np.minimum((u[0::2] * n).astype(np.int64), n - 1).astype(np.int32)
    b = np.minimum((u[1::2] * n).astype(np.int64), n - 1).astype(np.int32)
    if not self_loops:
        keep = a != b
        a, b = a[keep], b[keep]
    return a, b
