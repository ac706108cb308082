"""Caller-owned device memory at the C ABI: a graph bound into a torch tensor
(pr_graph_device_bytes / pr_graph_bind / pr_graph_free) and solves in a
torch workspace (pr_workspace_bytes / pr_solve_ws) give the same bits as the
library-owned graph and workspace, in every form, and the oracle's fixed
point (L1 <= 1e-9); the library allocates no device memory for a bound
graph; bad buffers are refused."""
import ctypes

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


@pytest.mark.timeout(300)
def test_bound_graph_gives_the_same_bits_in_every_form():
    fpr = _fpr()
    n = 1 << 14
    s, t = gg.rmat(14, 16, seed=61)
    og = oracle.csr(n, s, t)
    xr, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=5000, threads=8)
    plan = dict(with_cl=1, with_inplace=1)
    own = fpr.Graph(n, s, t, plan=plan)
    bound = fpr.Graph(n, s, t, plan=plan, device_memory="torch")
    assert bound.graph_memory is not None and bound.graph_memory.numel() >= bound.stats()["device_bytes"]
    for mode in ("jacobi", "fused", "edge_list", "fused_edge_list"):
        for prec in ("fp64", "fp32"):
            a = own.solve(d=D, tol=1e-12, mode=mode, precision=prec)
            b = bound.solve(d=D, tol=1e-12, mode=mode, precision=prec)
            assert a[1] == b[1] and torch.equal(a[0], b[0]), (mode, prec)
            assert l1(b[0].cpu().numpy(), xr) <= 1e-9
    x, it, res, ok = bound.solve(d=D, tol=1e-12, mode="inplace")
    assert ok and l1(x.cpu().numpy(), xr) <= 1e-9
    seeds = torch.tensor(gg.sample_distinct(n, 8, 61, 4), dtype=torch.int32, device="cuda")
    Xa, ia, _ = own.solve_batched(seeds, d=D, tol=1e-6, tile=8)
    Xb, ib, _ = bound.solve_batched(seeds, d=D, tol=1e-6, tile=8)
    assert torch.equal(Xa, Xb) and np.array_equal(ia, ib)
    own.close()
    mem = bound.graph_memory
    bound.close()
    assert mem.numel() > 0  # the caller's buffer outlives the graph


def test_bound_graph_takes_no_library_memory():
    fpr = _fpr()
    n = 1 << 17
    s, t = gg.rmat(17, 16, seed=62)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    own = fpr.Graph(n, s, t)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    own_bytes = own.stats()["device_bytes"]
    own.close()
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    bound = fpr.Graph(n, s, t, device_memory="torch")
    torch.cuda.synchronize()
    free3, _ = torch.cuda.mem_get_info()
    # the library-owned graph takes its arrays from the device; the bound one
    # only its torch tensor (allocated through torch's caching allocator)
    tensor_bytes = bound.graph_memory.numel()
    assert own_bytes > 8 << 20 and free0 - free1 >= own_bytes - (4 << 20)
    assert free2 - free3 <= tensor_bytes + (4 << 20)
    assert tensor_bytes >= own_bytes
    bound.close()


def test_solve_in_a_caller_workspace():
    fpr = _fpr()
    n = 1 << 13
    s, t = gg.rmat(13, 16, seed=63)
    og = oracle.csr(n, s, t)
    xr, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=5000, threads=8)
    g = fpr.Graph(n, s, t, plan=dict(with_inplace=1))
    for mode in ("jacobi", "fused", "inplace"):
        for prec in ("fp64", "fp32"):
            need = g.workspace_bytes(1e-12, mode=mode, precision=prec)
            assert need >= (16 if prec == "fp64" else 28) * n
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            a = g.solve(d=D, tol=1e-12, mode=mode, precision=prec)
            b = g.solve(d=D, tol=1e-12, mode=mode, precision=prec, workspace=ws)
            assert b[3] and l1(b[0].cpu().numpy(), xr) <= 1e-9, (mode, prec)
            if mode != "inplace":  # the in-place form is asynchronous: same fixed point, not the same bits
                assert a[1] == b[1] and torch.equal(a[0], b[0]), (mode, prec)
    from paper_2203_09284_amd._lib import FusedPRError
    need = g.workspace_bytes(1e-12)
    with pytest.raises(FusedPRError, match="needs"):
        g.solve(d=D, tol=1e-12, workspace=torch.empty(need - 256, dtype=torch.uint8, device="cuda"))
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(FusedPRError, match="aligned"):
        g.solve(d=D, tol=1e-12, workspace=big[8:])
    g.close()


def test_bind_refuses_bad_buffers():
    fpr = _fpr()
    from paper_2203_09284_amd import _lib as L
    from paper_2203_09284_amd.graph import build_csr
    lib = fpr.lib()
    n = 1 << 10
    s, t = gg.rmat(10, 8, seed=64)
    csr, _ = build_csr(n, s, t)
    po = L.PrPlanOpts()
    lib.pr_plan_opts_default(ctypes.byref(po))
    nb = ctypes.c_size_t(0)
    assert lib.pr_graph_device_bytes(ctypes.byref(csr), ctypes.byref(po), ctypes.byref(nb)) == 0
    h = ctypes.c_void_p()
    small = torch.empty(nb.value // 2, dtype=torch.uint8, device="cuda")
    assert lib.pr_graph_bind(ctypes.byref(csr), ctypes.byref(po), ctypes.c_void_p(small.data_ptr()), small.numel(),
                             ctypes.byref(h)) == L.PR_ENOMEM and not h.value
    host = np.zeros(nb.value + 256, np.uint8)
    assert lib.pr_graph_bind(ctypes.byref(csr), ctypes.byref(po), host.ctypes.data_as(ctypes.c_void_p), nb.value,
                             ctypes.byref(h)) == L.PR_EINVAL
    ok = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    assert lib.pr_graph_bind(ctypes.byref(csr), ctypes.byref(po), ctypes.c_void_p(ok.data_ptr() + 8), nb.value,
                             ctypes.byref(h)) == L.PR_EINVAL
    assert lib.pr_graph_bind(ctypes.byref(csr), ctypes.byref(po), ctypes.c_void_p(ok.data_ptr()), nb.value,
                             ctypes.byref(h)) == 0 and h.value
    lib.pr_graph_free(h)
    lib.pr_csr_free(ctypes.byref(csr))
