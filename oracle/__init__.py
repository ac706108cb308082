"""Plain FP64 CPU PageRank oracle -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library
(``paper_2203_09284_amd``) and never imports it.

``oracle.c`` holds the arithmetic (the Jacobi iteration of Eq. 1, the in-place
Gauss-Seidel recurrence of Eq. 9 that the loop-fused algorithm computes, F(x)
and its residual, the adjoint); ``dense.py`` holds the dense-matrix checks for
graphs of at most a few thousand vertices.  This module only marshals
arguments.

Parity pins (tests/test_oracle_pins.py): dense solve, closed forms, the
sum(x) = 1 invariant, the contraction bound, the DAG forward-substitution case,
brute-force adjacency sets, Eq. 9 and Eq. 2 written as small pure-Python loops,
the offsetList example of Section 3, the edge-list residual against a dense
F(x), finite differences and the duality / homogeneity identities of the
adjoint.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_oracle.so")
_LIB = None

NORM = {"l1": 0, "linf": 1}
DANGLING = {"uniform": 0, "leak": 1}


def build(force: bool = True) -> str:
    """Compile oracle.c (gcc -O3, the paper's flag; FP contraction off)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11",
           "-Wall", "-o", tmp, _SRC, "-lm"]
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
    vp = ctypes.c_void_p
    i64, dbl, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.orc_csr_count.argtypes = [i64, i64, vp, vp]
    lib.orc_csr_count.restype = i64
    lib.orc_csr_build.argtypes = [i64, i64, vp, vp, vp] + [vp] * 10
    lib.orc_csr_build.restype = cint
    lib.orc_jacobi.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, cint, cint,
                               cint, cint, vp, vp, vp, vp]
    lib.orc_jacobi.restype = cint
    lib.orc_gauss_seidel.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, cint, cint,
                                     cint, cint, vp, vp, vp]
    lib.orc_gauss_seidel.restype = cint
    lib.orc_gauss_seidel_threads.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, cint, cint,
                                             cint, cint, vp, vp]
    lib.orc_gauss_seidel_threads.restype = cint
    lib.orc_apply_F.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, dbl, cint, vp, vp]
    lib.orc_apply_F.restype = cint
    lib.orc_residual_edges.argtypes = [i64, i64, vp, vp, vp, vp, dbl, vp, vp, cint]
    lib.orc_residual_edges.restype = dbl
    lib.orc_adjoint.argtypes = [i64, vp, vp, vp, vp, vp, vp, dbl, dbl, cint, vp, vp, vp, vp]
    lib.orc_adjoint.restype = cint
    lib.orc_sample_in_lists.argtypes = [i64, i64, vp, vp, i64, vp, i64, vp, vp]
    lib.orc_sample_in_lists.restype = i64
    lib.orc_set_mutation.argtypes = [cint]
    lib.orc_set_mutation.restype = None
    _LIB = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def set_mutation(code: int) -> None:
    """Plant a known mistake in the oracle (tests of the pins only)."""
    _lib().orc_set_mutation(int(code))


@dataclass
class Graph:
    """Canonical graph in the paper's edge-centric layout (Section 3)."""
    n: int
    m: int
    in_ptr: np.ndarray
    in_src: np.ndarray
    in_w: np.ndarray | None
    out_ptr: np.ndarray
    out_dst: np.ndarray
    out_w: np.ndarray | None
    offset: np.ndarray
    out_deg: np.ndarray
    in_deg: np.ndarray
    edge_map: np.ndarray

    @property
    def W(self) -> np.ndarray:
        """Out-weight sums in outList order (out-degree when unweighted)."""
        if self.out_w is None:
            return self.out_deg.astype(np.float64)
        W = np.zeros(self.n)
        for v in range(self.n):
            s = 0.0
            for e in range(self.out_ptr[v], self.out_ptr[v + 1]):
                s += self.out_w[e]
            W[v] = s
        return W


def csr(n: int, src, dst, w=None) -> Graph:
    """Canonical CSR: self-loops dropped, repeated pairs merged (weights summed)."""
    lib = _lib()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    m_in = len(src)
    if w is not None:
        w = np.ascontiguousarray(w, np.float64)
    mu = lib.orc_csr_count(n, m_in, _p(src), _p(dst))
    if mu < 0:
        raise ValueError("vertex id out of range")
    in_ptr = np.zeros(n + 1, np.int64)
    out_ptr = np.zeros(n + 1, np.int64)
    in_src = np.zeros(max(mu, 1), np.int32)
    out_dst = np.zeros(max(mu, 1), np.int32)
    in_w = np.zeros(max(mu, 1), np.float64) if w is not None else None
    out_w = np.zeros(max(mu, 1), np.float64) if w is not None else None
    offset = np.zeros(max(mu, 1), np.int64)
    out_deg = np.zeros(n, np.int32)
    in_deg = np.zeros(n, np.int32)
    edge_map = np.zeros(max(m_in, 1), np.int64)
    rc = lib.orc_csr_build(n, m_in, _p(src), _p(dst), _p(w), _p(in_ptr), _p(in_src), _p(in_w),
                           _p(out_ptr), _p(out_dst), _p(out_w), _p(offset), _p(out_deg),
                           _p(in_deg), _p(edge_map))
    if rc != 0:
        raise MemoryError("orc_csr_build")
    return Graph(n, mu, in_ptr, in_src[:mu], None if in_w is None else in_w[:mu], out_ptr,
                 out_dst[:mu], None if out_w is None else out_w[:mu], offset[:mu], out_deg,
                 in_deg, edge_map[:m_in])


def _start(g: Graph, p, x0):
    if x0 is not None:
        return np.array(x0, np.float64, copy=True)
    if p is not None:
        return np.array(p, np.float64, copy=True)
    return np.full(g.n, 1.0 / g.n)


def jacobi(g: Graph, d: float = 0.85, tol: float = 1e-10, max_iter: int = 1000, p=None,
           x0=None, norm: str = "l1", dangling: str = "uniform", threads: int = 1,
           trace: bool = False):
    """x <- F(x) until the residual is below tol (Eq. 1 / Eq. 2).
    Returns (x, sweeps, residual[, trace, sums])."""
    x = _start(g, p, x0)
    p = None if p is None else np.ascontiguousarray(p, np.float64)
    res = np.zeros(1)
    tr = np.zeros(max_iter) if trace else None
    sm = np.zeros(max_iter) if trace else None
    it = _lib().orc_jacobi(g.n, _p(g.in_ptr), _p(g.in_src), _p(g.in_w), _p(g.out_ptr),
                           _p(g.out_dst), _p(g.out_w), _p(g.out_deg), _p(g.in_deg), _p(p), d,
                           tol, max_iter, NORM[norm], DANGLING[dangling], threads, _p(x),
                           _p(res), _p(tr), _p(sm))
    if it < 0:
        raise MemoryError("orc_jacobi")
    if trace:
        return x, it, float(res[0]), tr[:it], sm[:it]
    return x, it, float(res[0])


def gauss_seidel(g: Graph, d: float = 0.85, tol: float = 1e-10, max_iter: int = 1000, p=None,
                 x0=None, norm: str = "l1", dangling: str = "uniform", trace: bool = False,
                 scaled: bool = False):
    """Eq. 9 in place, ascending vertex order (Seq-FusEd); scaled=True is the
    mass-scaled variant.  Returns (x, sweeps, residual[, trace])."""
    x = _start(g, p, x0)
    p = None if p is None else np.ascontiguousarray(p, np.float64)
    res = np.zeros(1)
    tr = np.zeros(max_iter) if trace else None
    it = _lib().orc_gauss_seidel(g.n, _p(g.in_ptr), _p(g.in_src), _p(g.in_w), _p(g.out_ptr),
                                 _p(g.out_w), _p(g.out_deg), _p(p), d, tol, max_iter, NORM[norm],
                                 DANGLING[dangling], int(scaled), _p(x), _p(res), _p(tr))
    if it == -2:
        raise ValueError("the mass-scaled variant needs uniform dangling and the L1 norm")
    if it < 0:
        raise MemoryError("orc_gauss_seidel")
    if trace:
        return x, it, float(res[0]), tr[:it]
    return x, it, float(res[0])


def gauss_seidel_threads(g: Graph, d: float = 0.85, tol: float = 1e-10, max_iter: int = 1000,
                         p=None, x0=None, dangling: str = "uniform", scaled: bool = True,
                         threads: int = 1):
    """The paper's parallel fused variant (Sections 4.3, 6.3) on `threads` host
    threads, in place and asynchronous across threads; host timing only.
    Returns (x, sweeps, residual)."""
    x = _start(g, p, x0)
    p = None if p is None else np.ascontiguousarray(p, np.float64)
    res = np.zeros(1)
    it = _lib().orc_gauss_seidel_threads(g.n, _p(g.in_ptr), _p(g.in_src), _p(g.in_w),
                                         _p(g.out_ptr), _p(g.out_w), _p(g.out_deg), _p(p), d, tol,
                                         max_iter, DANGLING[dangling], int(scaled), int(threads),
                                         _p(x), _p(res))
    if it == -2:
        raise ValueError("the mass-scaled variant needs uniform dangling")
    if it < 0:
        raise MemoryError("orc_gauss_seidel_threads")
    return x, it, float(res[0])


def apply_F(g: Graph, x, d: float = 0.85, p=None, dangling: str = "uniform") -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    p = None if p is None else np.ascontiguousarray(p, np.float64)
    y = np.zeros(g.n)
    if _lib().orc_apply_F(g.n, _p(g.in_ptr), _p(g.in_src), _p(g.in_w), _p(g.out_ptr),
                          _p(g.out_w), _p(g.out_deg), _p(p), d, DANGLING[dangling], _p(x),
                          _p(y)) != 0:
        raise MemoryError("orc_apply_F")
    return y


def certificate(g: Graph, x, d: float = 0.85, p=None) -> float:
    """Upper bound on ||x - x*||_1: ||F(x) - x||_1 / (1 - d), since ||dP||_1 = d."""
    x = np.asarray(x, np.float64)
    return float(np.abs(apply_F(g, x, d, p) - x).sum() / (1.0 - d))


def adjoint(g: Graph, x, dLdx, d: float = 0.85, tol: float = 1e-14, max_iter: int = 10_000):
    """Returns (lam, dL/dp, dL/dw in outList order, sweeps, residual)."""
    x = np.ascontiguousarray(x, np.float64)
    gv = np.ascontiguousarray(dLdx, np.float64)
    lam = np.zeros(g.n)
    gp = np.zeros(g.n)
    gw = np.zeros(max(g.m, 1))
    res = np.zeros(1)
    it = _lib().orc_adjoint(g.n, _p(g.out_ptr), _p(g.out_dst), _p(g.out_w), _p(g.out_deg), _p(x),
                            _p(gv), d, tol, max_iter, _p(lam), _p(gp), _p(gw), _p(res))
    if it < 0:
        raise MemoryError("orc_adjoint")
    return lam, gp, gw[:g.m], it, float(res[0])


def sample_in_lists(n: int, src, dst, rows):
    """Distinct, ascending in-neighbour lists of the given rows, by brute force
    over the raw edge list.  Returns a list of int32 arrays."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    rows = np.ascontiguousarray(rows, np.int32)
    cnt = np.zeros(len(rows), np.int64)
    lib = _lib()
    total = lib.orc_sample_in_lists(n, len(src), _p(src), _p(dst), len(rows), _p(rows), 0,
                                    _p(cnt), None)
    if total < 0:
        raise MemoryError("orc_sample_in_lists")
    buf = np.zeros(max(total, 1), np.int32)
    lib.orc_sample_in_lists(n, len(src), _p(src), _p(dst), len(rows), _p(rows), total, _p(cnt),
                            _p(buf))
    out, pos = [], 0
    for c in cnt:
        out.append(buf[pos:pos + c].copy())
        pos += c
    return out


def residual_edges(n: int, src, dst, x, d: float = 0.85, p=None, w=None, threads: int = 1,
                   want_F: bool = False):
    """||F(x) - x||_1 from the raw edge list (self-loops skipped; each (src, dst)
    pair must appear once), with no graph built.  ||x - x*||_1 is at most this
    / (1 - d).  Returns the residual, or (residual, F(x)) with want_F."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    x = np.ascontiguousarray(x, np.float64)
    w = None if w is None else np.ascontiguousarray(w, np.float64)
    p = None if p is None else np.ascontiguousarray(p, np.float64)
    if len(src) != len(dst) or len(x) != n or (w is not None and len(w) != len(src)):
        raise ValueError("edge list / vector sizes disagree")
    y = np.zeros(n) if want_F else None
    r = _lib().orc_residual_edges(n, len(src), _p(src), _p(dst), _p(w), _p(p), d, _p(x), _p(y),
                                  int(threads))
    if r != r:
        raise MemoryError("orc_residual_edges")
    return (float(r), y) if want_F else float(r)
