"""GPU parity of the in-place form (PR_INPLACE: Algorithm 2 / Eq. 9 swept in
place in LDS-staged vertex blocks, asynchronous across blocks) against the
FP64 oracle's fixed point: L1 <= 1e-9 in FP64 and after FP32 + FP64
refinement, L1 <= 1e-5 for FP32 alone, on every test graph (weighted,
personalized, hubs, road grid, empty and ragged blocks) and every plan shape
the other forms are tested with.  The asynchronous trajectory is not
reproducible, so only the fixed point is compared."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

from test_gpu_forward import CASES, PLANS, _p_dev, _ref

pytestmark = pytest.mark.gpu
D = 0.85


def _fpr():
    import paper_2203_09284_amd as fpr
    return fpr


def say(msg):
    print(msg, flush=True)


def l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def _plan(k):
    return dict(PLANS[k] or {}, with_inplace=1)


@pytest.mark.parametrize("plan", range(len(PLANS)))
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_inplace_fixed_point(case, plan):
    name, n, src, dst, w, p = CASES[case]
    say("case %s plan %d inplace" % (name, plan))
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=_plan(plan))
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace", p=_p_dev(p))
    err = l1(x.cpu().numpy(), xr)
    say("  fp64 sweeps=%d resid=%.2e L1=%.2e" % (it, res, err))
    assert ok and err <= 1e-9
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace", precision="fp32", p=_p_dev(p))
    err = l1(x.cpu().numpy(), xr)
    say("  fp32+refine sweeps=%d L1=%.2e" % (it, err))
    assert ok and err <= 1e-9
    x, it, res, ok = g.solve(d=D, tol=1e-7, max_iter=3000, mode="inplace", precision="fp32", refine_tol=0.0,
                             p=_p_dev(p))
    assert l1(x.cpu().numpy(), xr) <= 1e-5
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_inplace_plain_lagged_form(case):
    name, n, src, dst, w, p = CASES[case]
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=dict(with_inplace=1))
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=5000, mode="inplace", fused_scaled=False, p=_p_dev(p))
    assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
    g.close()


@pytest.mark.parametrize("n,edges", [(1, []), (5, []), (3, [(0, 1), (1, 2), (2, 0)]), (2049, [(2048, 0), (0, 2048)]),
                                     (1025, [(i, 1024) for i in range(1024)])])
def test_inplace_edge_cases(n, edges):
    """A single vertex, no edges, a cycle, a vertex alone in the last block, a
    row whose sources fill a whole block."""
    fpr = _fpr()
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    _, xr = _ref(n, src, dst, None, None)
    g = fpr.Graph(n, src, dst, plan=dict(with_inplace=1))
    for prec in ("fp64", "fp32"):
        x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace", precision=prec)
        assert ok and l1(x.cpu().numpy(), xr) <= 1e-9, prec
    g.close()


def test_inplace_hub_and_long_rows():
    """Rows far longer than one lane's share (summed by the whole wavefront),
    inside and across blocks."""
    fpr = _fpr()
    n = 5000
    rng_src = gg.sample_distinct(n, 4000, 51, 4)
    src = np.concatenate([rng_src, np.arange(1, n, dtype=np.int32), gg.sample_distinct(n, 300, 52, 4)])
    dst = np.concatenate([np.zeros(4000, np.int32), np.arange(0, n - 1, dtype=np.int32),
                          np.full(300, 2500, np.int32)])
    keep = src != dst
    src, dst = src[keep].astype(np.int32), dst[keep].astype(np.int32)
    _, xr = _ref(n, src, dst, None, None)
    g = fpr.Graph(n, src, dst, plan=dict(with_inplace=1))
    for prec in ("fp64", "fp32"):
        x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace", precision=prec)
        assert ok and l1(x.cpu().numpy(), xr) <= 1e-9, prec
    g.close()


def test_inplace_needs_its_plan_and_rejects_linf():
    fpr = _fpr()
    from paper_2203_09284_amd._lib import FusedPRError
    s, t = gg.cycle(10)
    g = fpr.Graph(10, s, t)
    with pytest.raises(FusedPRError, match="with_inplace"):
        g.solve(mode="inplace")
    g.close()
    g = fpr.Graph(10, s, t, plan=dict(with_inplace=1))
    with pytest.raises(FusedPRError):
        g.solve(mode="inplace", norm="linf")
    g.close()


def test_inplace_road_grid_needs_fewer_sweeps_than_jacobi():
    """On a road-shaped grid (row-major ids) each lane's left neighbour is
    already updated when it is read: fewer sweeps than Jacobi (soft check of
    the Gauss-Seidel effect), same fixed point."""
    fpr = _fpr()
    side = 200
    s, t = gg.road_grid(side, seed=53)
    n = side * side
    _, xr = _ref(n, s, t, None, None)
    g = fpr.Graph(n, s, t, plan=dict(with_inplace=1))
    _, it_j, _, _ = g.solve(d=D, tol=1e-10, max_iter=3000, mode="jacobi")
    x, it_i, _, ok = g.solve(d=D, tol=1e-10, max_iter=3000, mode="inplace")
    say("road200: jacobi %d sweeps, inplace %d" % (it_j, it_i))
    assert ok and it_i < it_j
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace")
    assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
    g.close()


@pytest.mark.parametrize("kind", ["weighted", "personalized", "road"])
def test_inplace_interleaved_blocks(kind):
    """Graphs of several full blocks and a partial last one, so the plan's
    interleaved layout (inside a full block, lane l's k-th vertex at
    position 64 k + l) is exercised together with what is read by vertex: the
    edge weights, the teleport vector and the caller's start vector.  FP64 and
    FP32 + refinement reach the oracle's fixed point; a warm start from that
    point converges at once; pr_iterate from 1/n, run long enough, lands on
    it too."""
    fpr = _fpr()
    n, w, p = 3000, None, None
    if kind == "road":
        side = 61
        src, dst = gg.road_grid(side, seed=91)
        n = side * side
    else:
        src, dst = gg.random_graph(n, 6 * n, 91)
    if kind == "weighted":
        w = gg.weights(len(src), 92)
    if kind == "personalized":
        p = gg.uniforms(93, 9, n)
        p = p / p.sum()
    say("interleaved %s n=%d (full blocks: %d)" % (kind, n, n // 512))
    assert n // 512 >= 5 and n % 512 != 0
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=dict(with_inplace=1))
    for prec in ("fp64", "fp32"):
        x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode="inplace", precision=prec, p=_p_dev(p))
        say("  %s sweeps=%d L1=%.2e" % (prec, it, l1(x.cpu().numpy(), xr)))
        assert ok and l1(x.cpu().numpy(), xr) <= 1e-9, prec
    x0 = torch.tensor(xr, dtype=torch.float64, device="cuda")
    x, it, res, ok = g.solve(d=D, tol=1e-11, max_iter=3000, mode="inplace", p=_p_dev(p), x=x0.clone(),
                             warm_start=True)
    assert ok and it <= 3 and l1(x.cpu().numpy(), xr) <= 1e-9, it
    xi = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    g.iterate(xi, 400, d=D, mode="inplace", p=_p_dev(p))
    assert l1(xi.cpu().numpy(), xr) <= 1e-9
    # FP32 sweeps alone (no refinement): the ranks read back from the FP32
    # contributions meet the FP32 bar
    xf = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    g.iterate(xf, 400, d=D, mode="inplace", precision="fp32", p=_p_dev(p))
    say("  fp32 iterate L1=%.2e" % l1(xf.cpu().numpy(), xr))
    assert l1(xf.cpu().numpy(), xr) <= 1e-5
    g.close()
