"""Host-side behaviour of the library on the GPU: distinct graphs used from
distinct threads at once, cached hipGraphs reused across output and teleport
vectors, and the graph signature that keys tuned settings.  Results are
checked against the FP64 oracle's fixed point (L1 <= 1e-9)."""
import threading

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


def _ref(n, src, dst, p=None):
    og = oracle.csr(n, src, dst)
    x, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=5000, p=p)
    return x


def test_two_graphs_from_two_threads():
    fpr = _fpr()
    inputs = [(1 << 14, *gg.rmat(14, 16, seed=31)), (1 << 13, *gg.rmat(13, 8, seed=32))]
    refs = [_ref(n, s, t) for n, s, t in inputs]
    graphs = [fpr.Graph(n, s, t) for n, s, t in inputs]
    dev = torch.cuda.current_device()
    errors, results = [], [[] for _ in graphs]

    def work(i):
        try:
            torch.cuda.set_device(dev)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for rep in range(6):
                    mode = ("jacobi", "fused")[rep % 2]
                    prec = ("fp64", "fp32")[(rep // 2) % 2]
                    x, it, res, ok = graphs[i].solve(d=D, tol=1e-12, max_iter=1000, mode=mode, precision=prec,
                                                     stream=stream)
                    stream.synchronize()
                    results[i].append((mode, prec, ok, x.cpu().numpy()))
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(graphs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i, ref in enumerate(refs):
        assert len(results[i]) == 6
        for mode, prec, ok, x in results[i]:
            assert ok and l1(x, ref) <= 1e-9, (i, mode, prec, l1(x, ref))
    for g in graphs:
        g.close()


def test_new_output_and_teleport_vectors_reuse_the_captured_graph():
    fpr = _fpr()
    n = 1 << 12
    s, t = gg.rmat(12, 16, seed=33)
    ref = _ref(n, s, t)
    g = fpr.Graph(n, s, t)
    for mode in ("jacobi", "fused"):
        g.solve(d=D, tol=1e-12, max_iter=1000, mode=mode)
    base = g.stats()["graph_captures"]
    assert base >= 2
    for k in range(40):
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        mode = ("jacobi", "fused")[k % 2]
        x2, it, res, ok = g.solve(d=D, tol=1e-12, max_iter=1000, mode=mode, x=x)
        assert x2.data_ptr() == x.data_ptr()
        assert ok and l1(x.cpu().numpy(), ref) <= 1e-9, (k, mode)
    assert g.stats()["graph_captures"] == base
    # a new teleport vector on every call: same captured graphs again
    p_ref = None
    for k in range(6):
        p_h = gg.uniforms(40 + k, 9, n)
        p_h /= p_h.sum()
        p = torch.tensor(p_h, device="cuda")
        x, it, res, ok = g.solve(d=D, tol=1e-12, max_iter=1000, mode="jacobi", p=p)
        p_ref = _ref(n, s, t, p_h)
        assert ok and l1(x.cpu().numpy(), p_ref) <= 1e-9, k
    after_p = g.stats()["graph_captures"]
    # "p given" is another launch configuration: its own graphs, at most one
    # per power-of-two batch size (8, 4, 2, 1), whatever the number of vectors
    assert after_p <= base + 4
    g.close()


def test_graph_signature_tells_equal_sized_graphs_apart():
    fpr = _fpr()
    n = 1 << 11
    a = fpr.Graph(n, *gg.rmat(11, 8, seed=34))
    b = fpr.Graph(n, *gg.rmat(11, 8, seed=35))
    c = fpr.Graph(n, *gg.rmat(11, 8, seed=34))
    sa, sb, sc = (g.stats()["signature"] for g in (a, b, c))
    assert sa == sc and sa != sb
    for g in (a, b, c):
        g.close()


def test_pagerank_convenience_plans_every_form():
    fpr = _fpr()
    n = 1 << 12
    s, t = gg.rmat(12, 8, seed=36)
    ref = _ref(n, s, t)
    for mode in ("jacobi", "fused", "inplace", "edge_list", "fused_edge_list"):
        for prec in ("fp64", "fp32"):
            x, it = fpr.pagerank(n, s, t, tol=1e-12, mode=mode, precision=prec)
            assert l1(x.cpu().numpy(), ref) <= 1e-9, (mode, prec)


def test_gather_probe_times_and_validates():
    """pr_probe_gathers (measurement support): positive, ordered times for both
    precisions and both slot streams, and PR_EINVAL for bad arguments."""
    import ctypes
    from paper_2203_09284_amd import _lib as L
    fpr = _fpr()
    n = 1 << 14
    s, t = gg.rmat(14, 16, seed=33)
    g = fpr.Graph(n, s, t)
    try:
        for prec in ("fp64", "fp32"):
            for mode in ("graph", "uniform"):
                best, mean = g.probe_gathers(prec, mode, reps=3)
                assert 0.0 < best <= mean * (1 + 1e-9) < 1e6, (prec, mode, best, mean)
        with pytest.raises(ValueError):
            g.probe_gathers("fp16")
        lib = L.lib()
        out = ctypes.c_double(0.0)
        for prec, mode, reps in ((7, 0, 3), (L.PR_FP64, 2, 3), (L.PR_FP64, 0, 0), (L.PR_FP32, 1, 1001)):
            rc = lib.pr_probe_gathers(g._h, prec, mode, reps, ctypes.byref(out), None, None)
            assert rc == L.PR_EINVAL, (prec, mode, reps, rc)
        assert lib.pr_probe_gathers(g._h, L.PR_FP64, 0, 1, None, None, None) == L.PR_EINVAL
        # the graph still solves to the oracle's fixed point afterwards
        x, _, _, ok = g.solve(d=D, tol=1e-12, max_iter=1000, mode="fused")
        assert ok and l1(x.cpu().numpy(), _ref(n, s, t)) <= 1e-9
    finally:
        g.close()
