"""Python binding of the fusedpr C ABI: argument marshalling only.

Every step of the computation runs in libfusedpr.so (hipcc, gfx950).  PyTorch
provides device memory for the vectors (ranks, teleport vectors, gradients)
and the stream the calls are ordered on.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

MODES = {"jacobi": L.PR_JACOBI, "fused": L.PR_FUSED, "edge_list": L.PR_EDGE_LIST, "inplace": L.PR_INPLACE,
         "fused_edge_list": L.PR_FUSED_EDGE_LIST}
PRECISIONS = {"fp64": L.PR_FP64, "fp32": L.PR_FP32}
DANGLING = {"uniform": L.PR_DANGLING_UNIFORM, "leak": L.PR_DANGLING_LEAK}
NORMS = {"l1": L.PR_NORM_L1, "linf": L.PR_NORM_LINF}


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor | None, dtype, n: int | None, name: str):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class CanonicalCSR:
    """Host copy of the library's canonical graph (pr_build_csr)."""
    n: int
    m: int
    in_ptr: np.ndarray
    in_src: np.ndarray
    in_w: np.ndarray | None
    out_ptr: np.ndarray
    out_dst: np.ndarray
    out_w: np.ndarray | None
    out_to_in: np.ndarray
    out_deg: np.ndarray
    in_deg: np.ndarray
    edge_map: np.ndarray


def build_csr(n: int, src, dst, weights=None, keep: bool = True, library=None):
    """Run pr_build_csr on host arrays.  Returns (PrCsr owned by the library,
    CanonicalCSR numpy copy or None)."""
    lib = library or L.lib()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    if w is not None and w.shape != src.shape:
        raise ValueError("weights differ in length from the edge list")
    csr = L.PrCsr()
    rc = lib.pr_build_csr(n, len(src), src.ctypes.data_as(L.vp), dst.ctypes.data_as(L.vp),
                          None if w is None else w.ctypes.data_as(L.vp), ctypes.byref(csr))
    L.check(rc, library=lib)
    copy = None
    if keep:
        n_, m_ = csr.n, csr.m

        def arr(ptr, count, dt):
            if not ptr or count == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

        copy = CanonicalCSR(
            n=n_, m=m_,
            in_ptr=arr(csr.in_ptr, n_ + 1, np.int64), in_src=arr(csr.in_src, m_, np.int32),
            in_w=arr(csr.in_w, m_, np.float64) if csr.in_w else None,
            out_ptr=arr(csr.out_ptr, n_ + 1, np.int64), out_dst=arr(csr.out_dst, m_, np.int32),
            out_w=arr(csr.out_w, m_, np.float64) if csr.out_w else None,
            out_to_in=arr(csr.out_to_in, m_, np.int64), out_deg=arr(csr.out_deg, n_, np.int32),
            in_deg=arr(csr.in_deg, n_, np.int32), edge_map=arr(csr.edge_map, csr.m_input, np.int64))
    return csr, copy


class Graph:
    """A graph resident on the current GPU, with its execution plan."""

    def __init__(self, n: int, src, dst, weights=None, with_adjoint: bool = False,
                 plan: dict | None = None, keep_csr: bool = False, library: str = "",
                 device_memory: str = "library"):
        """library: "" for the product build, "naive" for the test variant whose
        FP32 sums are uncompensated.  device_memory: "library" (pr_graph_create
        allocates the graph's device arrays) or "torch" (pr_graph_bind places
        them in one torch uint8 tensor this object holds)."""
        lib = self._lib = L.lib(library)
        csr, copy = build_csr(n, src, dst, weights, keep=True, library=lib)
        self.csr = copy if keep_csr else None
        self.edge_map = torch.from_numpy(copy.edge_map) if weights is not None else None
        po = L.PrPlanOpts()
        lib.pr_plan_opts_default(ctypes.byref(po))
        for k, v in (plan or {}).items():
            setattr(po, k, int(v))
        po.with_adjoint = 1 if with_adjoint else 0
        handle = ctypes.c_void_p()
        self.graph_memory = None
        try:
            if device_memory == "torch":
                nbytes = ctypes.c_size_t(0)
                L.check(lib.pr_graph_device_bytes(ctypes.byref(csr), ctypes.byref(po), ctypes.byref(nbytes)),
                        library=lib)
                self.graph_memory = torch.empty(max(1, nbytes.value), dtype=torch.uint8,
                                                device=torch.device("cuda", torch.cuda.current_device()))
                rc = lib.pr_graph_bind(ctypes.byref(csr), ctypes.byref(po),
                                       ctypes.c_void_p(self.graph_memory.data_ptr()), nbytes.value,
                                       ctypes.byref(handle))
            elif device_memory == "library":
                rc = lib.pr_graph_create(ctypes.byref(csr), ctypes.byref(po), ctypes.byref(handle))
            else:
                raise ValueError("device_memory must be 'library' or 'torch'")
            L.check(rc, library=lib)
        finally:
            lib.pr_csr_free(ctypes.byref(csr))
        self._h = handle
        self.n = int(copy.n)
        self.m = int(copy.m)
        self.weighted = weights is not None
        self.with_adjoint = with_adjoint
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pr_graph_free(self._h)
            self._h = ctypes.c_void_p()
        self.graph_memory = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = L.PrGraphStats()
        L.check(self._lib.pr_graph_stats_get(self._h, ctypes.byref(s)), library=self._lib)
        return {k: getattr(s, k) for k, _ in L.PrGraphStats._fields_}

    # ------------------------------------------------------------- solve --
    def _opts(self, mode, precision, dangling, norm, warm, fused_scaled, sweeps_per_poll,
              use_hip_graph, refine_tol, fp32_tol, trace_buf):
        o = L.PrOpts()
        self._lib.pr_opts_default(ctypes.byref(o))
        o.mode = MODES[mode]
        o.precision = PRECISIONS[precision]
        o.dangling = DANGLING[dangling]
        o.norm = NORMS[norm]
        o.warm_start = 1 if warm else 0
        o.fused_scaled = 1 if fused_scaled else 0
        if sweeps_per_poll is not None:
            o.sweeps_per_poll = int(sweeps_per_poll)
        o.use_hip_graph = 1 if use_hip_graph else 0
        if refine_tol is not None:
            o.refine_tol = float(refine_tol)
        if fp32_tol is not None:
            o.fp32_tol = float(fp32_tol)
        if trace_buf is not None:
            o.trace = trace_buf.ctypes.data_as(L.c_f64p)
        return o

    def solve(self, d: float = 0.85, tol: float = 1e-8, max_iter: int = 1000, mode: str = "jacobi",
              precision: str = "fp64", p: torch.Tensor | None = None, x: torch.Tensor | None = None,
              warm_start: bool = False, dangling: str = "uniform", norm: str = "l1",
              fused_scaled: bool = True, sweeps_per_poll: int | None = None,
              use_hip_graph: bool = True, refine_tol: float | None = None,
              fp32_tol: float | None = None, trace: bool = False, stream=None, no_alloc: bool = False,
              workspace=None):
        """pr_solve; pr_solve_noalloc with no_alloc (the library allocates no
        device memory in the call); pr_solve_ws with a workspace (a torch
        uint8 CUDA tensor of at least workspace_bytes(...) bytes, or "torch" for
        a fresh one).  Returns (x, sweeps, residual, converged[, trace])."""
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        tr = np.zeros(max_iter) if trace else None
        o = self._opts(mode, precision, dangling, norm, warm_start, fused_scaled, sweeps_per_poll,
                       use_hip_graph, refine_tol, fp32_tol, tr)
        it = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        if workspace is not None:
            if isinstance(workspace, str):
                workspace = torch.empty(max(1, self.workspace_bytes(tol, o)), dtype=torch.uint8, device=self.device)
            if not workspace.is_cuda or workspace.dtype != torch.uint8:
                raise ValueError("workspace must be a uint8 CUDA tensor")
            rc = self._lib.pr_solve_ws(self._h, d, tol, max_iter, ctypes.byref(o),
                                       _dev_ptr(p, torch.float64, self.n, "p"), _dev_ptr(x, torch.float64, self.n, "x"),
                                       ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.byref(it),
                                       ctypes.byref(res), _stream_ptr(stream))
        else:
            entry = self._lib.pr_solve_noalloc if no_alloc else self._lib.pr_solve
            rc = entry(self._h, d, tol, max_iter, ctypes.byref(o), _dev_ptr(p, torch.float64, self.n, "p"),
                       _dev_ptr(x, torch.float64, self.n, "x"), ctypes.byref(it), ctypes.byref(res),
                       _stream_ptr(stream))
        L.check(rc, library=self._lib)
        out = (x, it.value, res.value, rc == L.PR_OK)
        if trace:
            return out + (tr[:it.value].copy(),)
        return out

    def workspace_bytes(self, tol: float = 1e-8, opts=None, mode: str = "jacobi", precision: str = "fp64",
                        refine_tol: float | None = None) -> int:
        """pr_workspace_bytes: device bytes pr_solve_ws needs for these options."""
        if opts is None:
            opts = self._opts(mode, precision, "uniform", "l1", False, True, None, True, refine_tol, None, None)
        nb = ctypes.c_size_t(0)
        L.check(self._lib.pr_workspace_bytes(self._h, tol, ctypes.byref(opts), ctypes.byref(nb)), library=self._lib)
        return nb.value

    def iterate(self, x: torch.Tensor, sweeps: int, d: float = 0.85, mode: str = "jacobi",
                p: torch.Tensor | None = None, dangling: str = "uniform", norm: str = "l1",
                fused_scaled: bool = True, use_hip_graph: bool = False, timed: bool = False,
                precision: str = "fp64", stream=None):
        """pr_iterate: exactly `sweeps` sweeps from the FP64 vector x, in place.  Returns
        the last residual, or (residual, device milliseconds of the sweeps) when timed."""
        o = self._opts(mode, precision, dangling, norm, True, fused_scaled, None, use_hip_graph, None,
                       None, None)
        res = ctypes.c_double(0.0)
        ms = ctypes.c_double(0.0)
        rc = self._lib.pr_iterate(self._h, d, ctypes.byref(o), _dev_ptr(p, torch.float64, self.n, "p"),
                                _dev_ptr(x, torch.float64, self.n, "x"), int(sweeps),
                                ctypes.byref(res), ctypes.byref(ms) if timed else None,
                                _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return (res.value, ms.value) if timed else res.value

    def profile_sweeps(self, sweeps: int, d: float = 0.85, mode: str = "jacobi", precision: str = "fp64",
                       fused_scaled: bool = True, stream=None):
        """pr_profile_sweeps from x = 1/n: average device milliseconds per sweep of
        the sweep kernel (all of its launches in that sweep) and of its finalize
        kernel, (sweep_ms, finalize_ms)."""
        o = self._opts(mode, precision, "uniform", "l1", True, fused_scaled, None, False, None, None, None)
        x = torch.full((self.n,), 1.0 / self.n, dtype=torch.float64, device=self.device)
        a = ctypes.c_double(0.0)
        b = ctypes.c_double(0.0)
        rc = self._lib.pr_profile_sweeps(self._h, d, ctypes.byref(o), _dev_ptr(x, torch.float64, self.n, "x"),
                                       int(sweeps), ctypes.byref(a), ctypes.byref(b), _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return a.value, b.value

    def probe_gathers(self, precision: str = "fp64", mode: str = "graph", reps: int = 5, stream=None):
        """pr_probe_gathers: device microseconds of the sweep's memory gathers
        alone (mode "graph": this plan's in-edge slots past the LDS copy;
        "uniform": as many uniformly random slots), (best, mean)."""
        modes = {"graph": 0, "uniform": 1}
        if precision not in PRECISIONS or mode not in modes:
            raise ValueError("precision must be one of %s and mode one of %s" % (sorted(PRECISIONS), sorted(modes)))
        best = ctypes.c_double(0.0)
        mean = ctypes.c_double(0.0)
        rc = self._lib.pr_probe_gathers(self._h, PRECISIONS[precision], modes[mode], int(reps), ctypes.byref(best),
                                        ctypes.byref(mean), _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return best.value, mean.value

    def certificate(self, x: torch.Tensor, d: float = 0.85, p: torch.Tensor | None = None,
                    stream=None) -> float:
        """||F(x) - x||_1, computed on the GPU; ||x - x*||_1 <= this / (1 - d)."""
        out = ctypes.c_double(0.0)
        rc = self._lib.pr_certificate(self._h, d, _dev_ptr(p, torch.float64, self.n, "p"),
                                    _dev_ptr(x, torch.float64, self.n, "x"), ctypes.byref(out),
                                    _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return out.value

    # ---------------------------------------------------------- batched --
    def solve_batched(self, seeds: torch.Tensor, d: float = 0.85, tol: float = 1e-6,
                      max_iter: int = 1000, tile: int = 0, shape: dict | None = None,
                      X: torch.Tensor | None = None, stream=None):
        """pr_solve_batched.  shape: {"tile", "items_per_grab", "wg_per_cu"}; or
        tile > 0 alone (default grab and workgroups); neither: autotuned.
        Returns (X [n, k] float32, iters[k], residuals[k])."""
        k = int(seeds.numel())
        if X is None:
            X = torch.empty((self.n, k), dtype=torch.float32, device=self.device)
        sh = None
        if shape is not None or tile:
            sh = L.PrBatchShape()
            self._lib.pr_batch_shape_default(ctypes.byref(sh))
            if tile:
                sh.tile = int(tile)
            for key, v in (shape or {}).items():
                setattr(sh, key, int(v))
        its = (ctypes.c_int * k)()
        res = (ctypes.c_double * k)()
        rc = self._lib.pr_solve_batched(self._h, d, tol, max_iter, k,
                                        _dev_ptr(seeds, torch.int32, k, "seeds"),
                                        ctypes.byref(sh) if sh is not None else None,
                                        _dev_ptr(X, torch.float32, self.n * k, "X"), its, res,
                                        _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return X, np.array(its[:], np.int64), np.array(res[:], np.float64)

    def autotune_batched(self, k: int, cache_path: str | None = None, stream=None) -> dict:
        """pr_autotune_batched: the fastest launch shape for k columns, as a dict."""
        sh = L.PrBatchShape()
        rc = self._lib.pr_autotune_batched(self._h, int(k), None if cache_path is None else cache_path.encode(),
                                           ctypes.byref(sh), _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return {"tile": sh.tile, "items_per_grab": sh.items_per_grab, "wg_per_cu": sh.wg_per_cu}

    # ---------------------------------------------------------- adjoint --
    def adjoint(self, x: torch.Tensor, dLdx: torch.Tensor, d: float = 0.85, tol: float = 1e-14,
                max_iter: int = 10_000, want_p: bool = True, want_w: bool = True, stream=None):
        """pr_adjoint.  Returns (lam, dL/dp or None, dL/dw in out-edge order or None, sweeps, residual)."""
        lam = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gp = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_p else None
        gw = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.device) if want_w else None
        it = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        rc = self._lib.pr_adjoint(self._h, d, _dev_ptr(x, torch.float64, self.n, "x"),
                                _dev_ptr(dLdx, torch.float64, self.n, "dLdx"), tol, max_iter,
                                _dev_ptr(lam, torch.float64, None, "lam"),
                                _dev_ptr(gp, torch.float64, None, "dLdp"),
                                _dev_ptr(gw, torch.float64, None, "dLdw"), ctypes.byref(it),
                                ctypes.byref(res), _stream_ptr(stream))
        L.check(rc, library=self._lib)
        return lam, gp, (gw[:self.m] if gw is not None else None), it.value, res.value
