"""GPU parity of the forward solve (Jacobi and fused forms, FP64 and FP32)
against the FP64 CPU oracle's fixed point.  Bar: L1 <= 1e-9 (FP64),
L1 <= 1e-5 (FP32); CSR and degrees are checked bit-exact on the host side.
"""
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


def say(msg):
    print(msg, flush=True)


def l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


def cases():
    out = []
    src, dst = gg.random_graph(300, 1500, 11)
    out.append(("random300", 300, src, dst, None, None))
    s, t = gg.rmat(10, 8, seed=12)
    out.append(("rmat10", 1024, s, t, None, None))
    src, dst = gg.random_graph(500, 2500, 13)
    out.append(("weighted500", 500, src, dst, gg.weights(len(src), 13), None))
    src, dst = gg.random_graph(400, 1200, 14)
    p = gg.uniforms(14, 9, 400)
    out.append(("personalized400", 400, src, dst, None, p / p.sum()))
    s, t = gg.rmat(14, 16, seed=2)
    out.append(("rmat14", 1 << 14, s, t, None, None))
    d = gg.er_10k()
    out.append(("er10k", d["n"], d["src"], d["dst"], None, None))
    s, t = gg.road_grid(48, seed=16)
    out.append(("road48", 48 * 48, s, t, None, None))
    return out


CASES = cases()
# plans that force every bin, many heavy chunks, ragged tiles and several
# Gauss-Seidel block counts (the fused form launches one sweep per block) on
# small graphs
PLANS = [None, dict(chunk=64, tile_max_row=9, tile_rows=5, steps=3, hot_slots=100, gs_blocks=3),
         dict(chunk=256, tile_max_row=0, steps=1, hot_slots=0, gather_layout=0, gs_blocks=1),
         dict(chunk=96, tile_max_row=90, tile_rows=128, steps=2, hot_slots=7, gs_blocks=7, gather_layout=2)]


def _ref(n, src, dst, w, p, tol=1e-15):
    og = oracle.csr(n, src, dst, w)
    x, _, _ = oracle.jacobi(og, D, tol=tol, max_iter=5000, p=p)
    return og, x


def _p_dev(p):
    return None if p is None else torch.tensor(p, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("plan", range(len(PLANS)))
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", ["jacobi", "fused"])
def test_fp64_fixed_point(case, plan, mode):
    name, n, src, dst, w, p = CASES[case]
    say("case %s plan %d mode %s" % (name, plan, mode))
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=PLANS[plan])
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=3000, mode=mode, p=_p_dev(p))
    assert ok, (it, res)
    err = l1(x.cpu().numpy(), xr)
    say("  sweeps=%d resid=%.2e L1=%.2e" % (it, res, err))
    assert err <= 1e-9
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_fused_plain_lagged_form(case):
    name, n, src, dst, w, p = CASES[case]
    say("case %s fused unscaled" % name)
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w)
    x, it, res, ok = g.solve(d=D, tol=1e-13, max_iter=5000, mode="fused", fused_scaled=False,
                             p=_p_dev(p))
    assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", ["jacobi", "fused"])
def test_fp32(case, mode):
    name, n, src, dst, w, p = CASES[case]
    say("case %s fp32 %s" % (name, mode))
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w)
    # FP32 only (no refinement): within the FP32 bar
    x, it, res, ok = g.solve(d=D, tol=1e-7, max_iter=3000, mode=mode, precision="fp32",
                             refine_tol=0.0, p=_p_dev(p))
    e32 = l1(x.cpu().numpy(), xr)
    # FP32 then FP64 refinement: within the FP64 bar
    x2, it2, res2, ok2 = g.solve(d=D, tol=1e-13, max_iter=3000, mode=mode, precision="fp32",
                                 p=_p_dev(p))
    e64 = l1(x2.cpu().numpy(), xr)
    say("  fp32 sweeps=%d L1=%.2e | refined sweeps=%d L1=%.2e" % (it, e32, it2, e64))
    assert e32 <= 1e-5
    assert ok2 and e64 <= 1e-9
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_one_sweep_equals_oracle_F(case):
    name, n, src, dst, w, p = CASES[case]
    say("case %s one sweep" % name)
    fpr = _fpr()
    og = oracle.csr(n, src, dst, w)
    x0 = gg.uniforms(99, 1, n)
    x0 /= x0.sum()
    want = oracle.apply_F(og, x0, D, p)
    g = fpr.Graph(n, src, dst, w, plan=PLANS[1])
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    r = g.iterate(x, 1, d=D, p=_p_dev(p))
    got = x.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))
    assert abs(r - np.abs(want - x0).sum()) <= 1e-12 * max(r, 1e-300)
    cert = g.certificate(torch.tensor(x0, dtype=torch.float64, device="cuda"), d=D, p=_p_dev(p))
    assert abs(cert - np.abs(want - x0).sum()) <= 1e-12 * cert
    g.close()


CLOSED = [("cycle", gg.cycle(9), lambda n: np.full(n, 1.0 / n)),
          ("in_star", gg.in_star(65), None), ("out_star", gg.out_star(65), None),
          ("bi_star", gg.bi_star(65), None)]


def _closed(name, n):
    if name == "in_star":
        xh = (1 + (n - 1) * D) / (n + (n - 1) * D)
        return np.array([xh] + [((1 - D) + D * xh) / n] * (n - 1))
    if name == "out_star":
        return np.array([1.0 / (n + D)] + [(n + D - 1) / ((n + D) * (n - 1))] * (n - 1))
    if name == "bi_star":
        xh = (D + (1 - D) / n) / (1 + D)
        return np.array([xh] + [(1 - xh) / (n - 1)] * (n - 1))
    return np.full(n, 1.0 / n)


@pytest.mark.parametrize("ci", range(len(CLOSED)), ids=[c[0] for c in CLOSED])
@pytest.mark.parametrize("mode", ["jacobi", "fused"])
def test_closed_forms(ci, mode):
    name, (s, t), _ = CLOSED[ci]
    n = int(max(s.max(), t.max())) + 1
    say("closed form %s %s" % (name, mode))
    fpr = _fpr()
    g = fpr.Graph(n, s, t)
    x, it, res, ok = g.solve(d=D, tol=1e-15, max_iter=500, mode=mode)
    want = _closed(name, n)
    assert np.max(np.abs(x.cpu().numpy() - want)) <= 1e-15 * max(1.0, n * want.max())
    g.close()


def test_path_leak_mode_and_linf():
    fpr = _fpr()
    n = 40
    s, t = gg.path(n)
    say("path leak")
    g = fpr.Graph(n, s, t)
    want = np.array([(1 - D ** (i + 1)) / n for i in range(n)])
    x, it, res, ok = g.solve(d=D, tol=1e-17, max_iter=500, dangling="leak", norm="linf")
    assert ok and np.max(np.abs(x.cpu().numpy() - want)) <= 1e-15 * want.max()
    og = oracle.csr(n, s, t)
    _, ito, _ = oracle.jacobi(og, D, tol=1e-17, max_iter=500, dangling="leak", norm="linf")
    assert abs(it - ito) <= 1
    g.close()


def test_leak_mode_iterates_follow_the_oracle():
    fpr = _fpr()
    s, t = gg.rmat(12, 8, seed=3)
    n = 1 << 12
    og = oracle.csr(n, s, t)
    say("leak trajectory")
    g = fpr.Graph(n, s, t, plan=PLANS[1])
    for sweeps in (1, 3, 10):
        xr, _, _ = oracle.jacobi(og, D, tol=0.0, max_iter=sweeps, dangling="leak")
        x = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        g.iterate(x, sweeps, d=D, dangling="leak")
        assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-14 * xr.max()
    g.close()


@pytest.mark.parametrize("n,edges", [(1, ([], [])), (7, ([], [])), (3, ([1, 1], [1, 1])),
                                     (2, ([0], [1])), (5, ([0, 0, 0, 4], [1, 1, 1, 1]))])
def test_edge_cases(n, edges):
    fpr = _fpr()
    s = np.array(edges[0], np.int32)
    t = np.array(edges[1], np.int32)
    say("edge case n=%d m=%d" % (n, len(s)))
    xr = oracle.jacobi(oracle.csr(n, s, t), D, tol=1e-16, max_iter=500)[0]
    g = fpr.Graph(n, s, t)
    for mode in ("jacobi", "fused"):
        for prec in ("fp64", "fp32"):
            x, it, res, ok = g.solve(d=D, tol=1e-14, max_iter=500, mode=mode, precision=prec)
            assert l1(x.cpu().numpy(), xr) <= 1e-12, (mode, prec)
    g.close()


def test_gather_layout_does_not_change_jacobi_bits():
    """The gather layout only moves addresses: same values, same summation order."""
    fpr = _fpr()
    s, t = gg.rmat(14, 16, seed=9)
    n = 1 << 14
    say("gather layout")
    a = fpr.Graph(n, s, t, plan=dict(gather_layout=1))
    b = fpr.Graph(n, s, t, plan=dict(gather_layout=0))
    xa = a.solve(d=D, tol=1e-12, mode="jacobi")
    xb = b.solve(d=D, tol=1e-12, mode="jacobi")
    assert torch.equal(xa[0], xb[0]) and xa[1] == xb[1]
    a.close()
    b.close()


def test_jacobi_is_bit_reproducible_and_graph_capture_neutral():
    fpr = _fpr()
    s, t = gg.rmat(14, 16, seed=5)
    n = 1 << 14
    say("determinism")
    g = fpr.Graph(n, s, t)
    a = g.solve(d=D, tol=1e-12, mode="jacobi")
    b = g.solve(d=D, tol=1e-12, mode="jacobi")
    c = g.solve(d=D, tol=1e-12, mode="jacobi", use_hip_graph=False, sweeps_per_poll=3)
    assert torch.equal(a[0], b[0]) and torch.equal(a[0], c[0]) and a[1] == b[1] == c[1]
    g.close()


def test_fused_across_schedules():
    """The fused form's trajectory depends on the schedule; its fixed point must not."""
    fpr = _fpr()
    s, t = gg.rmat(13, 16, seed=6)
    n = 1 << 13
    _, xr = _ref(n, s, t, None, None)
    say("fused schedules")
    for plan in PLANS:
        g = fpr.Graph(n, s, t, plan=plan)
        for rep in range(3):
            x, it, res, ok = g.solve(d=D, tol=1e-13, mode="fused", sweeps_per_poll=1 + rep)
            assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
        g.close()


@pytest.mark.parametrize("plan", range(len(PLANS)))
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_edge_list_form_equals_jacobi_bits(case, plan):
    """Algorithm 1 with the edge-ordered contributionList (scatter, then
    contiguous row sums) adds the same values in the same order as the pull,
    so its iterates are bit-identical to the Jacobi form's."""
    name, n, src, dst, w, p = CASES[case]
    say("case %s plan %d edge list" % (name, plan))
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=dict(PLANS[plan] or {}, with_cl=1))
    for prec in ("fp64", "fp32"):
        xa, ia, ra, oka = g.solve(d=D, tol=1e-12, max_iter=3000, mode="jacobi", precision=prec, p=_p_dev(p))
        xb, ib, rb, okb = g.solve(d=D, tol=1e-12, max_iter=3000, mode="edge_list", precision=prec, p=_p_dev(p))
        assert oka and okb and ia == ib and ra == rb, (prec, ia, ib, ra, rb)
        assert torch.equal(xa, xb), prec
        assert l1(xb.cpu().numpy(), xr) <= 1e-9
    # a fixed number of sweeps through pr_iterate, both precisions
    for prec in ("fp64", "fp32"):
        x0 = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        x1 = x0.clone()
        g.iterate(x0, 5, d=D, mode="jacobi", precision=prec, p=_p_dev(p))
        g.iterate(x1, 5, d=D, mode="edge_list", precision=prec, p=_p_dev(p))
        assert torch.equal(x0, x1), prec
    g.close()


@pytest.mark.parametrize("plan", range(len(PLANS)))
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_fused_edge_list_form_equals_fused_bits(case, plan):
    """Algorithm 2 with the edge-ordered contributionList (per Gauss-Seidel
    block: contiguous row sums and the update, then the block's fused scatter
    through offsetList) reads this sweep's contributions of the earlier blocks
    and the previous sweep's of the others, as the block Gauss-Seidel pull
    does, and adds them in the same order: bit-identical iterates, in both
    precisions, mass-scaled and plain, through pr_solve and pr_iterate."""
    name, n, src, dst, w, p = CASES[case]
    say("case %s plan %d fused edge list" % (name, plan))
    fpr = _fpr()
    _, xr = _ref(n, src, dst, w, p)
    g = fpr.Graph(n, src, dst, w, plan=dict(PLANS[plan] or {}, with_cl=1))
    for prec in ("fp64", "fp32"):
        for scaled in (True, False):
            kw = dict(d=D, tol=1e-12, max_iter=3000, precision=prec, p=_p_dev(p), fused_scaled=scaled)
            xa, ia, ra, oka = g.solve(mode="fused", **kw)
            xb, ib, rb, okb = g.solve(mode="fused_edge_list", **kw)
            assert oka and okb and ia == ib and ra == rb, (prec, scaled, ia, ib, ra, rb)
            assert torch.equal(xa, xb), (prec, scaled)
            assert l1(xb.cpu().numpy(), xr) <= 1e-9
    for prec in ("fp64", "fp32"):
        x0 = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        x1 = x0.clone()
        g.iterate(x0, 5, d=D, mode="fused", precision=prec, p=_p_dev(p))
        g.iterate(x1, 5, d=D, mode="fused_edge_list", precision=prec, p=_p_dev(p))
        assert torch.equal(x0, x1), prec
    g.close()


def test_edge_list_form_needs_its_plan():
    fpr = _fpr()
    from paper_2203_09284_amd._lib import FusedPRError
    s, t = gg.cycle(10)
    g = fpr.Graph(10, s, t)
    with pytest.raises(FusedPRError):
        g.solve(mode="edge_list")
    with pytest.raises(FusedPRError):
        g.solve(mode="fused_edge_list")
    g.close()


def test_local_input_keeps_one_block_and_id_order():
    """The default plan measures the share of in-edges whose source id is
    within 1024 of the destination's.  A street grid in row-major order is
    local (about half its in-edges join horizontal neighbours): the default plan
    keeps one Gauss-Seidel block and the hot-first, then id-order gathered
    array, and solves with the same bits as that plan asked for explicitly.  A
    permuted R-MAT graph is not local and keeps the plan by edges per sweep
    wavefront and gather-count order."""
    fpr = _fpr()
    side = 300
    s, t = gg.road_grid(side, seed=81)
    n = side * side
    _, xr = _ref(n, s, t, None, None)
    g = fpr.Graph(n, s, t)
    st = g.stats()
    say("road grid: local share %.3f, blocks %d, layout %d" % (st["local_share"], st["gs_blocks"], st["gather_layout"]))
    assert st["local_share"] >= 0.25 and st["gs_blocks"] == 1 and st["gather_layout"] == 2
    e = fpr.Graph(n, s, t, plan=dict(gs_blocks=1, gather_layout=2))
    for mode in ("jacobi", "fused"):
        a = g.solve(d=D, tol=1e-12, mode=mode)
        b = e.solve(d=D, tol=1e-12, mode=mode)
        assert a[1] == b[1] and torch.equal(a[0], b[0]), mode
        assert l1(a[0].cpu().numpy(), xr) <= 1e-9
    g.close()
    e.close()
    s, t = gg.rmat(14, 16, seed=2)
    g = fpr.Graph(1 << 14, s, t)
    st = g.stats()
    say("rmat14: local share %.3f, blocks %d, layout %d" % (st["local_share"], st["gs_blocks"], st["gather_layout"]))
    assert st["local_share"] < 0.25 and st["gather_layout"] == 1
    g.close()


def test_gauss_seidel_blocks_cut_sweeps():
    """Block Gauss-Seidel over out-degree-ordered blocks needs fewer sweeps than
    Jacobi (Stein-Rosenberg for the regular splitting; soft check), and every
    block count reaches the same fixed point."""
    fpr = _fpr()
    s, t = gg.rmat(14, 16, seed=2)
    n = 1 << 14
    _, xr = _ref(n, s, t, None, None)
    say("gs blocks")
    g = fpr.Graph(n, s, t)
    _, it_j, _, _ = g.solve(d=D, tol=1e-10, mode="jacobi")
    g.close()
    for B in (1, 2, 4, 16, 64):
        g = fpr.Graph(n, s, t, plan=dict(gs_blocks=B))
        x, it, res, ok = g.solve(d=D, tol=1e-10, mode="fused")
        say("  blocks=%d sweeps=%d (jacobi %d)" % (B, it, it_j))
        assert ok and it <= it_j
        if B >= 4:
            assert it < it_j
        x, it, res, ok = g.solve(d=D, tol=1e-13, mode="fused")
        assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
        g.close()


def test_trace_and_warm_start():
    fpr = _fpr()
    s, t = gg.rmat(12, 16, seed=7)
    n = 1 << 12
    og, xr = _ref(n, s, t, None, None)
    say("trace / warm start")
    g = fpr.Graph(n, s, t)
    x, it, res, ok, tr = g.solve(d=D, tol=1e-4, trace=True)
    _, ito, _, tro, _ = oracle.jacobi(og, D, tol=1e-4, max_iter=1000, trace=True)
    assert len(tr) == it and abs(it - ito) <= 1
    assert np.allclose(tr[:min(it, ito)], tro[:min(it, ito)], rtol=1e-9, atol=1e-18)
    # checkpoint at 1e-4, resume to 1e-12 == direct solve
    x2, it2, res2, ok2 = g.solve(d=D, tol=1e-12, x=x.clone(), warm_start=True)
    assert ok2 and l1(x2.cpu().numpy(), xr) <= 1e-9
    g.close()


def test_not_converged_status():
    fpr = _fpr()
    s, t = gg.rmat(12, 16, seed=8)
    say("max_iter")
    g = fpr.Graph(1 << 12, s, t)
    x, it, res, ok = g.solve(d=D, tol=1e-14, max_iter=3)
    assert not ok and it == 3 and res > 1e-14
    g.close()


def test_invalid_arguments():
    fpr = _fpr()
    from paper_2203_09284_amd._lib import FusedPRError
    s, t = gg.cycle(10)
    say("invalid args")
    g = fpr.Graph(10, s, t)
    for kw in (dict(d=1.0), dict(d=0.0), dict(tol=0.0), dict(max_iter=0)):
        with pytest.raises(FusedPRError):
            g.solve(**kw)
    with pytest.raises(FusedPRError):
        g.solve(mode="fused", norm="linf")
    with pytest.raises(FusedPRError):
        g.solve(mode="fused", dangling="leak")
    with pytest.raises(ValueError):
        g.solve(p=torch.zeros(3, dtype=torch.float64, device="cuda"))
    g.close()
    for plan in (dict(gs_blocks=-1), dict(gs_blocks=65), dict(chunk=32), dict(tile_rows=129), dict(gather_layout=3)):
        with pytest.raises(FusedPRError):
            fpr.Graph(10, s, t, plan=plan)
