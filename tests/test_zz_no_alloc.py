"""The no-allocation solve (pr_solve_noalloc, scratch in a fixed device array)
against pr_solve: the same ranks, bit for bit, and the oracle's fixed point
within L1 1e-9 (FP64) / 1e-5 (FP32), on two calls in a row, the second on a
smaller graph, in every precision and form it takes; sizes beyond its scratch
are refused."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
D = 0.85


def _fpr():
    import paper_2203_09284_amd as fpr
    return fpr


def l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def _case(scale, seed):
    n = 1 << scale
    s, t = gg.rmat(scale, 16, seed=seed)
    og = oracle.csr(n, s, t)
    xr, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=5000, threads=8)
    return n, s, t, xr


@pytest.mark.timeout(300)
def test_noalloc_matches_pr_solve_on_two_calls_in_a_row():
    fpr = _fpr()
    # the larger graph first, then a smaller one: the second call reuses the
    # scratch the first one filled
    for scale, seed in ((17, 41), (12, 42)):
        n, s, t, xr = _case(scale, seed)
        g = fpr.Graph(n, s, t)
        for mode in ("jacobi", "fused"):
            for prec, bar in (("fp64", 1e-9), ("fp32", 1e-9)):
                x0, it0, r0, ok0 = g.solve(d=D, tol=1e-12, max_iter=1000, mode=mode, precision=prec)
                x1, it1, r1, ok1 = g.solve(d=D, tol=1e-12, max_iter=1000, mode=mode, precision=prec,
                                           no_alloc=True)
                a, b = x0.cpu().numpy(), x1.cpu().numpy()
                print("n=%d %s %s: sweeps %d / %d, L1 vs oracle %.2e" % (n, mode, prec, it0, it1, l1(b, xr)),
                      flush=True)
                assert ok1 and it1 == it0 and r1 == r0, (scale, mode, prec)
                assert np.array_equal(a, b), (scale, mode, prec)
                assert l1(b, xr) <= bar
            # FP32 without refinement: the FP32 bar
            x2, _, _, _ = g.solve(d=D, tol=1e-7, max_iter=1000, mode=mode, precision="fp32", refine_tol=0,
                                  no_alloc=True)
            assert l1(x2.cpu().numpy(), xr) <= 1e-5
        g.close()


@pytest.mark.timeout(300)
def test_noalloc_inplace_form_reaches_the_fixed_point():
    """The in-place form keeps its interleaved ranks in the scratch's second
    contribution buffer; it is asynchronous, so the check is the oracle's fixed
    point (not the bits of pr_solve), again on two calls in a row."""
    fpr = _fpr()
    for scale, seed in ((17, 44), (12, 45)):
        n, s, t, xr = _case(scale, seed)
        g = fpr.Graph(n, s, t, plan=dict(with_inplace=1))
        for prec in ("fp64", "fp32"):
            x, it, r, ok = g.solve(d=D, tol=1e-12, max_iter=1000, mode="inplace", precision=prec, no_alloc=True)
            print("n=%d inplace %s: sweeps %d, L1 vs oracle %.2e" % (n, prec, it, l1(x.cpu().numpy(), xr)),
                  flush=True)
            assert ok and l1(x.cpu().numpy(), xr) <= 1e-9, (scale, prec)
        g.close()


def test_noalloc_refuses_what_it_cannot_hold():
    fpr = _fpr()
    from paper_2203_09284_amd._lib import FusedPRError
    L = fpr.lib()
    assert L.pr_noalloc_scratch_bytes() == 32 << 20
    n = 3_000_000  # 48 MB of FP64 contributions: more than the scratch
    s = np.arange(0, 1000, dtype=np.int32)
    g = fpr.Graph(n, s, (s + 1).astype(np.int32))
    with pytest.raises(FusedPRError, match="scratch"):
        g.solve(d=D, tol=1e-8, max_iter=100, no_alloc=True)
    g.close()
    s, t = gg.rmat(10, 8, seed=43)
    g = fpr.Graph(1 << 10, s, t, plan=dict(with_cl=1))
    with pytest.raises(FusedPRError, match="edge-list"):
        g.solve(d=D, tol=1e-8, mode="edge_list", no_alloc=True)
    with pytest.raises(FusedPRError, match="trace"):
        g.solve(d=D, tol=1e-8, trace=True, no_alloc=True)
    x, it, r, ok = g.solve(d=D, tol=1e-12, no_alloc=True)
    assert ok
    g.close()
