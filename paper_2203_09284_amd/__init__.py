"""FusEd-PageRank on MI355X (gfx950): the per-iteration sparse pull of
PageRank in the paper's edge-centric Jacobi form (Algorithm 1) and its
loop-fused Gauss-Seidel-like form (Algorithm 2: over vertex blocks, or swept
in place with asynchronous blocks), as hand-written HIP kernels behind a C ABI
(include/fusedpr.h), plus batched personalized PageRank and an
implicit-differentiation adjoint.

    import paper_2203_09284_amd as fpr
    g = fpr.Graph(n, src, dst)                     # canonical CSR + device plan
    x, sweeps, resid, ok = g.solve(tol=1e-8, mode="fused")

The library is built in-tree by ``__graft_entry__.build()``; importing the
solvers without it raises ImportError (there is no CPU fallback).
"""
from ._lib import FusedPRError, lib  # noqa: F401
from .graph import CanonicalCSR, Graph, build_csr  # noqa: F401
from .autograd import PageRankFn, pagerank_with_grad  # noqa: F401


def pagerank(n, src, dst, d=0.85, tol=1e-8, max_iter=1000, mode="jacobi", precision="fp64",
             personalization=None, weights=None):
    """One-shot convenience: build the graph (with the arrays the form needs),
    solve, return (x, sweeps)."""
    plan = dict(with_inplace=1 if mode == "inplace" else 0,
                with_cl=1 if mode in ("edge_list", "fused_edge_list") else 0)
    g = Graph(n, src, dst, weights, plan=plan)
    try:
        x, it, _, _ = g.solve(d=d, tol=tol, max_iter=max_iter, mode=mode, precision=precision,
                              p=personalization)
        return x, it
    finally:
        g.close()
