"""Dense-matrix checks for small graphs (n up to a few thousand) -- TEST
INFRASTRUCTURE, like the rest of ``oracle/``.

Everything here is built straight from the raw edge list with Python sets and
numpy, independently of ``oracle.c``:

  A[u, v]   = weight of edge v->u (repeated pairs: weights summed; unweighted
              repeats collapse to one edge); self-loops dropped
  W[v]      = column sums of A (out-weight sums)
  P[:, v]   = A[:, v] / W[v], or 1/n everywhere for a dangling column
              (0 in LEAK mode, the paper's literal algorithms)
  x*        = solve((I - d P) x = (1 - d) p)          (Section 1, Eq. 1 as a linear system)
  lam       = solve((I - d P)^T lam = g)               (adjoint of L = g^T x)

``cond_1(I - dP) <= (1 + d) / (1 - d)``, so a dense solve is accurate to a few
ulps times that -- far below every tolerance the tests use.
"""
from __future__ import annotations

import numpy as np


def adjacency(n: int, src, dst, w=None) -> np.ndarray:
    A = np.zeros((n, n))
    seen = set()
    for i, (s, t) in enumerate(zip(np.asarray(src).tolist(), np.asarray(dst).tolist())):
        if s == t:
            continue
        if w is None:
            if (s, t) in seen:
                continue
            seen.add((s, t))
            A[t, s] = 1.0
        else:
            A[t, s] += float(w[i])
    return A


def transition(n: int, src, dst, w=None, dangling: str = "uniform") -> np.ndarray:
    A = adjacency(n, src, dst, w)
    W = A.sum(axis=0)
    P = np.zeros((n, n))
    for v in range(n):
        if W[v] > 0:
            P[:, v] = A[:, v] / W[v]
        elif dangling == "uniform":
            P[:, v] = 1.0 / n
    return P


def solve(n: int, src, dst, w=None, d: float = 0.85, p=None, dangling: str = "uniform"):
    P = transition(n, src, dst, w, dangling)
    p = np.full(n, 1.0 / n) if p is None else np.asarray(p, np.float64)
    M = np.eye(n) - d * P
    return np.linalg.solve(M, (1.0 - d) * p)


def adjoint(n: int, src, dst, w=None, d: float = 0.85, g=None):
    P = transition(n, src, dst, w)
    M = np.eye(n) - d * P
    return np.linalg.solve(M.T, np.asarray(g, np.float64))


def loss(n: int, src, dst, w, d: float, p, g) -> float:
    return float(np.dot(g, solve(n, src, dst, w, d, p)))


def gradient_fd_weight(n: int, src, dst, w, d: float, p, g, edge: int, rel_h: float = 1e-5):
    """Central finite difference of L = g^T x w.r.t. input weight `edge`."""
    w = np.asarray(w, np.float64)
    h = rel_h * w[edge]
    wp = w.copy(); wp[edge] += h
    wm = w.copy(); wm[edge] -= h
    return (loss(n, src, dst, wp, d, p, g) - loss(n, src, dst, wm, d, p, g)) / (2.0 * h)


def gradient_fd_p(n: int, src, dst, w, d: float, p, g, u: int, h: float = 1e-4):
    p = np.asarray(p, np.float64)
    pp = p.copy(); pp[u] += h
    pm = p.copy(); pm[u] -= h
    return (loss(n, src, dst, w, d, pp, g) - loss(n, src, dst, w, d, pm, g)) / (2.0 * h)


def gradient_weights(n: int, src, dst, w, d: float, p, g):
    """dL/dw for each distinct edge, by differentiating the dense matrix: for the
    edge v->u, dP/dw changes column v only, by (e_u - P[:, v]) / W[v]; then
    dL/dw = lam^T (d dP/dw) x.  Returns {(v, u): gradient}."""
    A = adjacency(n, src, dst, w)
    W = A.sum(axis=0)
    P = transition(n, src, dst, w)
    p = np.full(n, 1.0 / n) if p is None else np.asarray(p, np.float64)
    M = np.eye(n) - d * P
    x = np.linalg.solve(M, (1.0 - d) * p)
    lam = np.linalg.solve(M.T, np.asarray(g, np.float64))
    out = {}
    vs, us = np.nonzero(A.T)  # A.T[v, u] = w(v->u)
    for v, u in zip(vs.tolist(), us.tolist()):
        dcol = -P[:, v].copy()
        dcol[u] += 1.0
        dcol /= W[v]
        out[(v, u)] = float(d * x[v] * np.dot(lam, dcol))
    return out
