"""Implicit differentiation of the PageRank fixed point.

x* solves (I - dP) x = (1 - d) p.  For a loss L(x*) with upstream gradient
g = dL/dx*, the backward pass solves the transposed system
(I - dP)^T lam = g on the GPU (pr_adjoint, a transposed pull over out-edges)
instead of differentiating through the iterates, and returns
    dL/dp = (1 - d) lam
    dL/dw(v->u) = d x_v / W_v (lam_u - (P^T lam)_v)
mapped back to the caller's edge order (repeated edges share the gradient of
their merged edge, self-loops get 0).
"""
from __future__ import annotations

import torch


class PageRankFn(torch.autograd.Function):
    """x = PageRankFn.apply(p, w, graph, d, tol, max_iter).

    p: teleport vector (float64, CUDA, sums to 1); w: the edge weights the
    graph was built with (float64, CUDA, caller's edge order) -- the forward
    solve uses the graph's copy, w is the handle gradients flow to.  The graph
    must be built with with_adjoint=True."""

    @staticmethod
    def forward(ctx, p, w, graph, d=0.85, tol=1e-12, max_iter=10_000):
        if not graph.with_adjoint:
            raise ValueError("the graph was built without the adjoint plan (with_adjoint=True)")
        x, _, _, ok = graph.solve(d=d, tol=tol, max_iter=max_iter, p=p.detach().contiguous())
        if not ok:
            raise RuntimeError("forward PageRank did not reach tol=%g in %d sweeps" % (tol, max_iter))
        ctx.graph = graph
        ctx.d = d
        ctx.tol = tol
        ctx.max_iter = max_iter
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        g = ctx.graph
        need_p, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        lam, gp, gw, _, _ = g.adjoint(x, gx.detach().to(torch.float64).contiguous(), d=ctx.d,
                                      tol=min(ctx.tol, 1e-12), max_iter=ctx.max_iter,
                                      want_p=need_p, want_w=need_w)
        grad_w = None
        if need_w:
            emap = g.edge_map.to(gw.device)
            keep = emap >= 0
            grad_w = torch.zeros(emap.numel(), dtype=torch.float64, device=gw.device)
            grad_w[keep] = gw[emap[keep]]
        return gp, grad_w, None, None, None, None


def pagerank_with_grad(graph, p, w, d=0.85, tol=1e-12, max_iter=10_000):
    return PageRankFn.apply(p, w, graph, d, tol, max_iter)
