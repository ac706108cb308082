#!/usr/bin/env python3
"""Benchmark of the PageRank hot path on one MI355X.

Headline workload: R-MAT scale 24 (2^24 vertices, edge factor 16, a=0.57,
b=c=0.19, seed 5, deduplicated, vertices relabelled in BFS order), d = 0.85,
stop at L1 < 1e-8.  A "step" is one full solve from x = 1/n to L1 < 1e-8 with
the loop-fused form (the paper's method) in FP64: init, every sweep (pull +
update + dangling / residual reductions + convergence test) and the host
polls.  `value` = edges traversed per second over those sweeps,
m' * sweeps / time, in GTEPS; inputs are resident in HBM before timing.

The same JSON line carries, on the same GPU:
  forms       at scale 24: plain FP64 Jacobi, fused FP64, FP32 Jacobi / fused
              with FP64 refinement to 1e-8, and the edge-centric
              contributionList form of Algorithm 1 (scatter, then contiguous row
              sums), each with the oracle's certificate on its error;
  roofline    of the dominant kernel, the fused FP64 sweep at scale 24 (the
              FP32 sweep's beside it), with the device time of the sweep's
              memory gathers alone beside it (gather_probe);
  cpu_baseline the FP64 CPU oracle timed on the host cores: one application of
              Eq. 1 over the same scale-24 edge list (one Jacobi sweep);
  rmat20      R-MAT scale 20 (permuted ids; its working set fits the Infinity
              Cache): the same forms against the oracle's fixed point, with the
              oracle's full solves on 1..16 host threads (Seq/Par-EC against
              Seq/Par-FusEd);
  batched     k = 64 one-hot personalized solves on R-MAT-20 (FP32, per-column
              tol 1e-6) against 64 sequential plain FP64 single-seed solves;
  er10k       directed Erdos-Renyi n=10,000, m=80,000, plain FP64, tol 1e-10;
  adjoint     weighted R-MAT scale 18: forward solve + adjoint + gradients;
  road8m      a road-network-shaped street grid (8.4 M vertices, degree ~2.8).

    python bench.py [--steps K] [--warmup W] [--quick]
    python bench.py --profile FORM [--workload rmat20|rmat24]   (kernel-only driver
        for rocprofv3: sweeps of one form, or one k = 64 batched solve with
        FORM = batched, or the sweep's gathers alone with FORM = probe-fp64|fp32,
        then a reference copy kernel)
    python bench.py --pmc-summary KEY FETCH_CSV WRITE_CSV DRIVER_LOG  (counter runs of
        that driver -> HBM bytes per sweep, into profiles/traffic.json)
    python bench.py --study [WORKLOAD ...]   (convergence study: thresholds 1e-6..1e-15,
        L1 and max-norm stop rules, fused vs Jacobi distance, residual traces)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GTEPS/iter + time-to-L1 1e-8 (fused/batched/fp32 vs plain fp64), % HBM peak")
HBM_PEAK_GBS = 8000.0
D = 0.85
# the kernels and the plan that shapes their launches
KERNEL_SOURCES = ("sweep.hip", "plan.hip", "device_common.h", "internal.h")
BATCHED_SOURCES = ("batched.hip", "plan.hip", "device_common.h", "internal.h")
PROBE_SOURCES = ("probe.hip", "plan.hip", "device_common.h", "internal.h")
COPY_BYTES = 256 << 20  # the reference copy kernel reads and writes this many bytes


def sig(v, digits=6):
    return float("%.*g" % (digits, v))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rounded(d):
    return {k: (sig(v) if isinstance(v, float) else v) for k, v in d.items()}


def workload(name):
    import graphgen as gg
    if name == "rmat20":
        w = gg.rmat20()
        w.update(tol=1e-8, desc="R-MAT scale 20, edge factor 16, a=.57 b=c=.19, seed 2, permuted ids")
    elif name == "er10k":
        w = gg.er_10k()
        w.update(tol=1e-10, desc="directed Erdos-Renyi n=10,000 m=80,000, seed 1")
    elif name == "rmat24":
        w = gg.rmat24_bfs()
        w.update(tol=1e-8, desc="R-MAT scale 24, edge factor 16, a=.57 b=c=.19, seed 5, BFS order")
    elif name == "road8m":
        w = gg.road8m()
        w.update(tol=1e-8, desc="2896 x 2896 street grid, segments kept 0.75, one-way 0.1, seed 6, "
                                "row-major ids")
    elif name in ("rmat21", "rmat22", "rmat23"):
        sc = int(name[4:])
        w = gg.rmat_permuted(sc, seed=sc)
        w.update(tol=1e-8, desc="R-MAT scale %d, edge factor 16, a=.57 b=c=.19, seed %d, permuted ids" % (sc, sc))
    elif name == "rmat18w":
        w = gg.rmat18_weighted()
        w.update(tol=1e-12, desc="weighted R-MAT scale 18, weights U[0.5,1.5], seed 4")
    else:
        raise SystemExit("unknown workload %s" % name)
    return w


def b_alg(n, m, s):
    """Algorithmic bytes of one sweep: stream the graph once (4 B per edge id,
    8 B per vertex offset), read and write every rank once (s B each), read the
    degree (4 B per vertex)."""
    return 4 * m + 8 * (n + 1) + 2 * s * n + 4 * n


def kernel_source_sha(files=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2203_09284_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(key, files=KERNEL_SOURCES):
    """HBM bytes per sweep (the sweep kernel's launches of one sweep) from the
    committed rocprofv3 counter runs (profiles/traffic.json), valid only while
    the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != kernel_source_sha(files):
        return None
    return rec.get("bytes_per_sweep")


def timed(torch, fn, steps, warmup):
    """Median device time (HIP events on torch's current stream, which the
    library joins on entry and exit) of `steps` calls after `warmup` calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times, out = [], None
    for _ in range(steps):
        e0.record()
        out = fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    return float(np.median(times)), out


def sweep_kernel_us(g, mode, precision="fp64", sweeps=50, reps=3):
    """Average device time per sweep of the sweep kernel (all of its launches in
    one sweep) and of its finalize kernel, in microseconds: HIP events recorded
    by the library on its own work stream around them (pr_profile_sweeps), best
    of `reps` runs."""
    best = None
    for _ in range(reps):
        ks, kf = g.profile_sweeps(sweeps, d=D, mode=mode, precision=precision)
        if best is None or ks < best[0]:
            best = (ks, kf)
    return best[0] * 1e3, best[1] * 1e3


def solve_legs(torch, g, m, tol, steps, warmup, names, x_ref=None, cert=None):
    """Time each form's solve to `tol`; state its error against the oracle:
    the L1 distance to the oracle's fixed point (x_ref), or the oracle's
    certificate ||F(x) - x||_1 / (1 - d), which bounds ||x - x*||_1 (cert)."""
    forms = {}
    for name in names:
        mode, prec = name.split("-")[:2]
        kw = dict(d=D, tol=tol, max_iter=1000, mode=mode, precision=prec)
        if name.endswith("unscaled"):
            kw["fused_scaled"] = False
        t_ms, (x, it, r, ok) = timed(torch, lambda: g.solve(**kw), steps, warmup)
        f = dict(ms=t_ms, sweeps=it, resid=r, converged=bool(ok), gteps=m * it / (t_ms * 1e-3) / 1e9)
        xh = x.cpu().numpy()
        if x_ref is not None:
            f["l1_vs_oracle"] = float(np.abs(xh - x_ref).sum())
        else:
            f["oracle_certificate"] = float(cert(xh))
        forms[name] = f
        log("%-20s %9.3f ms  sweeps=%3d  GTEPS=%8.2f  resid=%.2e" % (name, t_ms, it, f["gteps"], r))
    return forms


def roofline(achieved_gbs, traffic, kernel, bytes_sweep, us_sweep, launches, edge_bytes=None):
    """`achieved` and `traffic` are per sweep: the sweep kernel's launches of one
    sweep (one per Gauss-Seidel block in the fused form), timed together.
    `edge_bytes` is the pessimistic count that adds one value read per edge
    gather to the algorithmic bytes."""
    r = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "alg_bytes_per_sweep": bytes_sweep, "us_per_sweep": round(us_sweep, 2),
         "launches_per_sweep": launches}
    if edge_bytes is not None:
        r["edge_bytes_per_sweep"] = edge_bytes
        r["edge_gbs"] = round(edge_bytes / (us_sweep * 1e-6) / 1e9, 1)
    if traffic is not None:
        r["traffic_gbs"] = round(traffic / (us_sweep * 1e-6) / 1e9, 1)
    return r


def host_cpu():
    """CPU model string and the number of logical CPUs the host shows."""
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


# ----------------------------------------------------------------- legs --

def leg_batched(torch, fpr, oracle, og, g, n, m, steps):
    import graphgen as gg
    seeds_h = gg.ppr_seeds(n)
    seeds = torch.tensor(seeds_h, dtype=torch.int32, device="cuda")
    tune = g.autotune_batched(64)
    t_b, (X, its, res) = timed(torch, lambda: g.solve_batched(seeds, d=D, tol=1e-6), max(3, steps // 4), 1)
    log("batched k=64 shape=%s: %.2f ms, sweeps max %d" % (tune, t_b, its.max()))
    # the oracle's certificate of every column: ||F_j(x_j) - x_j||_1 / (1 - d)
    # with the one-hot teleport of seed j (Eq. 1), on the FP32 result cast up
    Xh = X.cpu().numpy().astype(np.float64)
    certs = []
    for j, s in enumerate(seeds_h):
        p = np.zeros(n)
        p[s] = 1.0
        certs.append(oracle.certificate(og, Xh[:, j], D, p))
    del Xh

    ps = torch.zeros((64, n), dtype=torch.float64, device="cuda")
    ps[torch.arange(64, device="cuda"), seeds.long()] = 1.0
    xs = torch.empty(n, dtype=torch.float64, device="cuda")

    def sequential():
        return [g.solve(d=D, tol=1e-6, max_iter=1000, mode="jacobi", p=ps[j], x=xs)[1] for j in range(64)]
    t_s, its_s = timed(torch, sequential, 1, 1)
    log("64 sequential FP64 Jacobi PPR solves: %.2f ms" % t_s)
    col = float(its.sum())
    # with all 64 columns in one launch, every sweep reads, per in-edge, the
    # source's 256-byte row (rate over the whole solve, init and output included)
    row_bytes = float(m) * 4 * 64 * int(its.max()) if tune["tile"] == 64 else None
    traffic = traffic_record("batched_rmat20", BATCHED_SOURCES) if n == (1 << 20) else None
    return rounded(dict(k=64, tol=1e-6, shape=tune, ms=t_b, max_sweeps=int(its.max()),
                        column_sweeps=int(col), column_gteps=m * col / (t_b * 1e-3) / 1e9,
                        row_read_gbs=row_bytes / (t_b * 1e-3) / 1e9 if row_bytes else None,
                        b_alg_per_sweep=b_alg(n, m, 4 * 64), traffic_per_sweep=traffic,
                        sequential_fp64_ms=t_s, sequential_sweeps=int(sum(its_s)),
                        speedup_vs_sequential_fp64=t_s / t_b,
                        oracle_certificate_max=max(certs), oracle_certificate_median=float(np.median(certs))))


def leg_er10k(torch, fpr, oracle, steps, warmup):
    w = workload("er10k")
    og = oracle.csr(w["n"], w["src"], w["dst"])
    xr, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=1000)
    g = fpr.Graph(w["n"], w["src"], w["dst"])
    forms = solve_legs(torch, g, g.m, 1e-10, steps, warmup, ["jacobi-fp64", "fused-fp64"], xr)
    g.close()
    return dict(workload="er10k", n=w["n"], m=og.m, tol=1e-10, forms={k: rounded(v) for k, v in forms.items()})


def leg_adjoint(torch, fpr, oracle, steps, warmup, threads):
    w = workload("rmat18w")
    n = w["n"]
    gvec = np.zeros(n)
    gvec[w["targets"]] = 1.0
    g = fpr.Graph(n, w["src"], w["dst"], w["w"], with_adjoint=True)
    gdev = torch.tensor(gvec, device="cuda")
    t_f, (x, it, _, _) = timed(torch, lambda: g.solve(d=D, tol=1e-12, max_iter=2000), steps, warmup)
    t_a, (lam, gp, gw, it2, _) = timed(torch, lambda: g.adjoint(x, gdev, d=D, tol=1e-12), steps, warmup)
    log("adjoint rmat18w: forward %.3f ms (%d sweeps), adjoint+grads %.3f ms (%d sweeps)" % (t_f, it, t_a, it2))
    og = oracle.csr(n, w["src"], w["dst"], w["w"])
    xr, _, _ = oracle.jacobi(og, D, tol=1e-15, max_iter=2000, threads=threads)
    lam_o, gp_o, gw_o, _, _ = oracle.adjoint(og, xr, gvec, D, tol=1e-14)
    rel = lambda a, b: float(np.abs(a.cpu().numpy() - b).sum() / np.abs(b).sum())
    out = dict(workload="rmat18w", n=n, m=g.m, tol=1e-12, forward_ms=t_f, forward_sweeps=it,
               forward_l1_vs_oracle=float(np.abs(x.cpu().numpy() - xr).sum()), adjoint_ms=t_a, adjoint_sweeps=it2, rel_l1_lambda=rel(lam, lam_o), rel_l1_dLdp=rel(gp, gp_o),
               rel_l1_dLdw=rel(gw, gw_o))
    g.close()
    return rounded(out)


def leg_road(torch, fpr, oracle, steps, warmup, threads):
    """Road-network-shaped graph (low degree, no hubs, long diameter): the
    regime where the paper reports its smallest gains."""
    w = workload("road8m")
    g = fpr.Graph(w["n"], w["src"], w["dst"], plan=dict(with_cl=1, with_inplace=1))
    n, m = g.n, g.m
    cert = lambda xh: oracle.residual_edges(n, w["src"], w["dst"], xh, D, threads=threads) / (1 - D)
    forms = solve_legs(torch, g, m, 1e-8, steps, warmup,
                       ["jacobi-fp64", "fused-fp64", "jacobi-fp32", "fused-fp32", "edge_list-fp64",
                        "fused_edge_list-fp64", "inplace-fp64", "inplace-fp32"], cert=cert)
    kern = {name: sweep_kernel_us(g, *name.split("-"), sweeps=20) for name in
            ("jacobi-fp64", "fused-fp64", "inplace-fp64")}
    st = g.stats()
    out = dict(workload="road8m", graph=w["desc"], n=n, m=m, tol=1e-8, gs_blocks=st["gs_blocks"],
               forms={k: rounded(v) for k, v in forms.items()},
               kernel_us={k: {"sweep": round(v[0], 2), "finalize": round(v[1], 2)} for k, v in kern.items()},
               alg_gbs_jacobi_fp64=sig(b_alg(n, m, 8) / (kern["jacobi-fp64"][0] * 1e-6) / 1e9))
    # the fastest form on this graph: the in-place sweep, against the same
    # algorithmic bytes (it reads the same per-vertex and per-edge arrays)
    b64 = b_alg(n, m, 8)
    ki = kern["inplace-fp64"][0]
    out["roofline_inplace_fp64"] = roofline(b64 / (ki * 1e-6) / 1e9, traffic_record("inplace_fp64_road8m"),
                                            "k_inplace<double>", b64, ki, 1)
    out["speedup_vs_jacobi_fp64"] = {k: sig(forms["jacobi-fp64"]["ms"] / f["ms"]) for k, f in forms.items()
                                     if k != "jacobi-fp64"}
    log("road8m: jacobi %.3f ms (%d), fused %.3f ms (%d), inplace %.3f ms (%d), sweep %.1f us" %
        (forms["jacobi-fp64"]["ms"], forms["jacobi-fp64"]["sweeps"], forms["fused-fp64"]["ms"],
         forms["fused-fp64"]["sweeps"], forms["inplace-fp64"]["ms"], forms["inplace-fp64"]["sweeps"],
         kern["jacobi-fp64"][0]))
    g.close()
    return out


def leg_scale(torch, fpr, oracle, name, steps, warmup, threads):
    """One of the intermediate R-MAT sizes the paper's synthetic set covers
    (scales 21-23, Section 6.2), permuted ids: time to L1 < 1e-8 of the four
    main forms, each with the oracle's certificate, and the sweep kernel's time
    per sweep."""
    import graphgen as gg
    w = workload(name)
    g = fpr.Graph(w["n"], w["src"], w["dst"])
    n, m = g.n, g.m
    src, dst = gg.dedup(n, w["src"], w["dst"])
    del w
    cert = lambda xh: oracle.residual_edges(n, src, dst, xh, D, threads=threads) / (1 - D)
    forms = solve_legs(torch, g, m, 1e-8, steps, warmup, ["jacobi-fp64", "fused-fp64", "jacobi-fp32", "fused-fp32"],
                       cert=cert)
    kern = {k: sweep_kernel_us(g, *k.split("-"), sweeps=20) for k in forms}
    out = dict(workload=name, n=n, m=m, tol=1e-8, gs_blocks=g.stats()["gs_blocks"],
               forms={k: rounded(v) for k, v in forms.items()},
               kernel_us={k: {"sweep": round(v[0], 2), "finalize": round(v[1], 2)} for k, v in kern.items()},
               alg_gbs={k: sig(b_alg(n, m, 8 if k.endswith("fp64") else 4) / (v[0] * 1e-6) / 1e9)
                        for k, v in kern.items()},
               speedup_vs_jacobi_fp64={k: sig(forms["jacobi-fp64"]["ms"] / f["ms"]) for k, f in forms.items()
                                       if k != "jacobi-fp64"})
    g.close()
    return out


def headline_rmat24(torch, fpr, oracle, steps, warmup, cores, cpu_baseline):
    """The headline: R-MAT scale 24 in BFS order, every form to L1 < 1e-8 with
    the oracle's certificate, the sweep kernels' device time, and the oracle's
    own sweep over the same edge list on the host cores."""
    t0 = time.perf_counter()
    w = workload("rmat24")
    n, src, dst = w["n"], w["src"], w["dst"]
    log("generated rmat24 in %.1fs" % (time.perf_counter() - t0))
    t0 = time.perf_counter()
    g = fpr.Graph(n, src, dst, plan=dict(with_cl=1, with_inplace=1))
    setup_s = time.perf_counter() - t0
    m = g.m
    st = g.stats()
    log("rmat24 on device: m'=%d blocks=%d setup %.1fs" % (m, st["gs_blocks"], setup_s))
    cert = lambda xh: oracle.residual_edges(n, src, dst, xh, D, threads=cores) / (1 - D)
    forms = solve_legs(torch, g, m, 1e-8, steps, warmup, ["jacobi-fp64", "fused-fp64", "jacobi-fp32", "fused-fp32"],
                       cert=cert)
    forms.update(solve_legs(torch, g, m, 1e-8, 3, 1, ["edge_list-fp32", "fused_edge_list-fp32", "inplace-fp64",
                                                      "inplace-fp32"], cert=cert))
    # the configuration's own stop rule for this graph: fused FP32 with
    # compensated sums to L1 < 1e-7, FP64 refinement sweeps at the end
    # (Jacobi FP64 to the same tolerance beside it)
    c5 = solve_legs(torch, g, m, 1e-7, steps, warmup, ["jacobi-fp64", "fused-fp32"], cert=cert)
    c5_out = dict(tol=1e-7, forms={k: rounded(v) for k, v in c5.items()},
                  fused_fp32_vs_jacobi_fp64=sig(c5["jacobi-fp64"]["ms"] / c5["fused-fp32"]["ms"]))
    kern = {name: sweep_kernel_us(g, *name.split("-"), sweeps=20) for name in
            ("fused-fp64", "jacobi-fp64", "fused-fp32", "jacobi-fp32", "inplace-fp32")}
    for name, (ks, kf) in kern.items():
        log("rmat24 %-12s sweep kernel %.1f us + finalize %.1f us per sweep" % (name, ks, kf))
    # the sweep's memory gathers alone (every in-edge's slot past the LDS copy,
    # nothing else), the floor of a sweep whose reads land on random lines; and
    # as many uniformly random slots, the device's rate for uncached lines
    floor = {p: g.probe_gathers(p, "graph")[0] for p in ("fp64", "fp32")}
    uni_us = g.probe_gathers("fp64", "uniform")[0]
    gather_probe = dict(fp64_us=round(floor["fp64"], 1), fp32_us=round(floor["fp32"], 1),
                        fp64_traffic=traffic_record("probe_fp64_rmat24", PROBE_SOURCES),
                        fp32_traffic=traffic_record("probe_fp32_rmat24", PROBE_SOURCES),
                        uniform_fp64_us=round(uni_us, 1), uniform_g_gathers_s=sig(m / (uni_us * 1e-6) / 1e9),
                        uniform_line_fill_tbs=sig(m * 128 / (uni_us * 1e-6) / 1e12))
    log("rmat24 gathers alone: FP64 %.1f us, FP32 %.1f us per sweep; %d uniform FP64 gathers %.1f us"
        % (floor["fp64"], floor["fp32"], m, uni_us))
    cpu = None
    if cpu_baseline:
        # the oracle as it stands, on a bounded sample of this workload: one
        # application of Eq. 1 over the whole edge list (one Jacobi sweep plus
        # its residual), from x = 1/n; median of 3 on all host threads, once on 1
        x0 = np.full(n, 1.0 / n)
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.residual_edges(n, src, dst, x0, D, threads=cores)
            runs.append(time.perf_counter() - t0)
        cpu_s = float(np.median(runs))
        t0 = time.perf_counter()
        oracle.residual_edges(n, src, dst, x0, D, threads=1)
        one_s = time.perf_counter() - t0
        cpu = dict(value=sig(m / cpu_s / 1e9), unit="GTEPS", cores=cores, kind="oracle",
                   sample="one Jacobi sweep of Eq. 1 (F(x) and ||F(x) - x||_1) over the same scale-24 edge "
                          "list, x = 1/n, FP64: median of 3 runs of %.2f s on %d threads; 1 thread: %.2f s"
                          % (cpu_s, cores, one_s),
                   single_thread_gteps=sig(m / one_s / 1e9))
        cpu["cpu_model"], cpu["nproc"] = host_cpu()
        log("cpu oracle sweep at rmat24: %.3f GTEPS on %d threads, %.3f on 1" %
            (cpu["value"], cores, cpu["single_thread_gteps"]))
    g.close()
    return dict(n=n, m=m, setup_s=setup_s, gs_blocks=st["gs_blocks"], forms=forms, kern=kern, cpu=cpu,
                tol_1e7=c5_out, gather_probe=gather_probe)


def leg_rmat20(torch, fpr, oracle, steps, warmup, cores, args):
    """R-MAT scale 20, permuted ids: every form against the oracle's fixed point,
    the sweep kernels, the batched personalized solve on the same graph, and the
    oracle's own full solves on the host (Seq/Par-EC against Seq/Par-FusEd)."""
    w = workload("rmat20")
    n, tol = w["n"], w["tol"]
    g = fpr.Graph(n, w["src"], w["dst"], plan=dict(with_cl=1, with_inplace=1))
    m = g.m
    st = g.stats()
    og = oracle.csr(n, w["src"], w["dst"])
    x_ref, _, _ = oracle.jacobi(og, D, tol=1e-13, max_iter=1000, threads=cores)
    forms = solve_legs(torch, g, m, tol, steps, warmup,
                       ["jacobi-fp64", "fused-fp64", "fused-fp64-unscaled", "jacobi-fp32", "fused-fp32",
                        "edge_list-fp64", "fused_edge_list-fp64", "inplace-fp64", "inplace-fp32"], x_ref)
    kern = {name: sweep_kernel_us(g, *name.split("-")) for name in
            ("fused-fp64", "jacobi-fp64", "fused-fp32", "jacobi-fp32", "edge_list-fp64")}
    for name, (ks, kf) in kern.items():
        log("rmat20 %-12s sweep kernel %.1f us + finalize %.1f us per sweep" % (name, ks, kf))
    b64 = b_alg(n, m, 8)
    kf = kern["fused-fp64"][0]
    out = dict(workload="rmat20", graph=w["desc"], n=n, m=m, tol=tol, gs_blocks=st["gs_blocks"],
               forms={k: rounded(f) for k, f in forms.items()},
               kernel_us={k: {"sweep": round(v[0], 2), "finalize": round(v[1], 2)} for k, v in kern.items()},
               speedup_vs_jacobi_fp64_time_to_tol={
                   k: sig(forms["jacobi-fp64"]["ms"] / f["ms"]) for k, f in forms.items() if k != "jacobi-fp64"},
               roofline=dict(roofline(b64 / (kf * 1e-6) / 1e9, traffic_record("fused_fp64_rmat20"),
                                      "k_sweep<double, fused>", b64, kf, st["gs_blocks"], b64 + 8 * m),
                             note="cache-resident: the FP64 working set (94 MB) fits the 256 MB Infinity Cache"))
    if not args.quick:
        try:
            out["batched"] = leg_batched(torch, fpr, oracle, og, g, n, m, args.steps)
        except Exception as e:  # reported, not fatal
            out["batched"] = dict(error=str(e)[:300])
            log("batched leg failed: %s" % e)
    g.close()
    if not args.no_cpu_baseline:
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, it_cpu, _ = oracle.jacobi(og, D, tol=tol, max_iter=1000, threads=cores)
            runs.append(time.perf_counter() - t0)
        cpu_s = float(np.median(runs))
        out["cpu_oracle_solve"] = dict(gteps=sig(og.m * it_cpu / cpu_s / 1e9), threads=cores, sweeps=it_cpu,
                                       s=sig(cpu_s, 4))
        if not args.quick:
            out["cpu_thread_scaling"] = host_scaling(oracle, og, tol, cores)
    return out


def host_scaling(oracle, og, tol, cores):
    """The paper's host comparison (Section 6.3, its thread-scaling figure) on
    this box: the oracle's Jacobi iteration (the baseline's numbers, Seq-EC /
    Par-EC) against its in-place Eq. 9 loop (Seq-FusEd / Par-FusEd, mass-scaled,
    asynchronous across threads), FP64, same graph and stop rule, for
    1..cores threads."""
    out = []
    counts = [k for k in (1, 2, 4, 8, 12, 16, 20) if k <= cores]
    for th in counts:
        t0 = time.perf_counter()
        _, it_ec, _ = oracle.jacobi(og, D, tol=tol, max_iter=1000, threads=th)
        t_ec = time.perf_counter() - t0
        t0 = time.perf_counter()
        if th == 1:
            _, it_f, _ = oracle.gauss_seidel(og, D, tol=tol, max_iter=1000, scaled=True)
        else:
            _, it_f, _ = oracle.gauss_seidel_threads(og, D, tol=tol, max_iter=1000, scaled=True, threads=th)
        t_f = time.perf_counter() - t0
        out.append(dict(threads=th, ec_s=sig(t_ec, 4), ec_sweeps=it_ec, fused_s=sig(t_f, 4), fused_sweeps=it_f,
                        fused_speedup_vs_ec=sig(t_ec / t_f, 4)))
        log("host %2d threads: EC %.3f s (%d sweeps), FusEd %.3f s (%d sweeps)" % (th, t_ec, it_ec, t_f, it_f))
    return out


def profile_driver(args):
    """Kernel-only run for rocprofv3: `sweeps` sweeps of one form, launched one
    by one, then five reference copies of COPY_BYTES (read + write) through
    torch's elementwise kernel, to calibrate the HBM byte counters."""
    import torch
    import paper_2203_09284_amd as fpr
    torch.cuda.set_device(0)
    w = workload(args.workload)
    if args.profile == "batched":
        import graphgen as gg
        g = fpr.Graph(w["n"], w["src"], w["dst"])
        seeds = torch.tensor(gg.ppr_seeds(g.n), dtype=torch.int32, device="cuda")
        # the library's default launch shape (tile 64, one item per grab, two
        # workgroups per CU), which is also the one the tuner picks at this size;
        # tuning here would put the tuner's trial launches into the trace
        X, its, _ = g.solve_batched(seeds, d=D, tol=1e-6, tile=64)
        shape = dict(tile=64)
        torch.cuda.synchronize()
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        # sweeps that did work (launches after every column froze exit at once)
        print(json.dumps({"profile": "batched", "workload": args.workload, "n": g.n, "m": g.m,
                          "sweeps": int(its.max()), "shape": shape,
                          "copy_bytes": COPY_BYTES, "columns": 64,
                          "b_alg": b_alg(g.n, g.m, 4 * 64),
                          "source_sha": kernel_source_sha(BATCHED_SOURCES)}), flush=True)
        g.close()
        return
    if args.profile.startswith("probe-"):
        # the sweep's memory gathers alone (pr_probe_gathers, this plan's slots):
        # one untimed and `sweeps` timed launches, each one sweep's gathers
        prec = args.profile.split("-")[1]
        g = fpr.Graph(w["n"], w["src"], w["dst"])
        best, mean = g.probe_gathers(prec, "graph", reps=args.profile_sweeps)
        torch.cuda.synchronize()
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"profile": args.profile, "workload": args.workload, "n": g.n, "m": g.m,
                          "sweeps": args.profile_sweeps + 1, "best_us": best, "mean_us": mean,
                          "copy_bytes": COPY_BYTES, "b_alg": b_alg(g.n, g.m, 8 if prec == "fp64" else 4),
                          "source_sha": kernel_source_sha(PROBE_SOURCES)}),
              flush=True)
        g.close()
        return
    mode, prec = args.profile.split("-")[:2]
    g = fpr.Graph(w["n"], w["src"], w["dst"], plan=dict(with_cl=1 if "edge_list" in mode else 0,
                                                        with_inplace=1 if mode == "inplace" else 0))
    x = torch.full((g.n,), 1.0 / g.n, dtype=torch.float64, device="cuda")
    g.iterate(x, args.profile_sweeps, d=D, mode=mode, precision=prec, use_hip_graph=False)
    torch.cuda.synchronize()
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"profile": args.profile, "workload": args.workload, "n": g.n, "m": g.m,
                      "sweeps": args.profile_sweeps, "copy_bytes": COPY_BYTES,
                      "b_alg": b_alg(g.n, g.m, 8 if prec == "fp64" else 4),
                      "source_sha": kernel_source_sha()}), flush=True)
    g.close()


def study(args):
    """Convergence study (the paper's threshold sweep, Section 6.3, on the
    synthetic stand-ins): for thresholds 1e-6 .. 1e-15, sweeps and time of the
    Jacobi pull under the L1 and max-norm stop rules (Eq. 3 uses the max-norm),
    of the fused form and of the edge-list form (L1), the L1 distance between
    the fused and the Jacobi results at the same threshold (the paper compares
    FusEd against the edge-centric baseline this way), the certificate bound of
    each, the per-sweep residuals of the 1e-15 solves, and the per-sweep L1 and
    max-norm errors against the fixed point (the paper's error curves)."""
    import torch
    import paper_2203_09284_amd as fpr
    torch.cuda.set_device(0)
    out = {"study": "convergence", "d": D, "workloads": {}}
    for name in args.study:
        w = workload(name)
        g = fpr.Graph(w["n"], w["src"], w["dst"], plan=dict(with_cl=1))
        rows = []
        for e in range(6, 16):
            tol = 10.0 ** (-e)
            row = {"tol": tol}
            xs = {}
            for form, mode, norm in (("jacobi", "jacobi", "l1"), ("jacobi_linf", "jacobi", "linf"),
                                     ("fused", "fused", "l1"), ("edge_list", "edge_list", "l1")):
                kw = dict(d=D, tol=tol, max_iter=2000, mode=mode, norm=norm)
                t_ms, (x, it, r, ok) = timed(torch, lambda: g.solve(**kw), 3, 1)
                row[form] = {"sweeps": it, "ms": sig(t_ms), "converged": bool(ok),
                             "certificate_bound": sig(g.certificate(x, d=D) / (1 - D))}
                xs[form] = x.clone()
            row["l1_fused_vs_jacobi"] = sig(float((xs["fused"] - xs["jacobi"]).abs().sum()))
            row["l1_edge_list_vs_jacobi"] = float((xs["edge_list"] - xs["jacobi"]).abs().sum())
            rows.append(row)
            log("%s tol %.0e: jacobi %d (linf %d), fused %d, edge_list %d sweeps; |fused - jacobi|_1 %.2e" %
                (name, tol, row["jacobi"]["sweeps"], row["jacobi_linf"]["sweeps"], row["fused"]["sweeps"],
                 row["edge_list"]["sweeps"], row["l1_fused_vs_jacobi"]))
        traces = {}
        for mode in ("jacobi", "fused"):
            _, it, _, _, tr = g.solve(d=D, tol=1e-15, max_iter=2000, mode=mode, trace=True)
            traces[mode] = [sig(float(v), 4) for v in tr]
        # error curves: the iterate after each sweep against the fixed point
        # solved to 1e-15, in L1 and max-norm (one sweep per call, from 1/n)
        xstar = g.solve(d=D, tol=1e-15, max_iter=2000, mode="jacobi")[0]
        errors = {}
        for mode in ("jacobi", "fused"):
            x = torch.full((g.n,), 1.0 / g.n, dtype=torch.float64, device="cuda")
            e1, einf = [], []
            for _ in range(len(traces[mode])):
                g.iterate(x, 1, d=D, mode=mode)
                diff = (x - xstar).abs()
                e1.append(sig(float(diff.sum()), 4))
                einf.append(sig(float(diff.max()), 4))
            errors[mode] = {"l1": e1, "linf": einf}
        out["workloads"][name] = {"n": g.n, "m": g.m, "rows": rows, "residual_trace_1e-15": traces,
                                  "error_trace": errors}
        g.close()
    print(json.dumps(out), flush=True)


def pmc_summary(args):
    """Turn two rocprofv3 --pmc runs of the --profile driver (FETCH_SIZE, then
    WRITE_SIZE; counter_collection CSVs) into the bytes one sweep moves through
    the sweep kernel (all of its launches in that sweep: one per Gauss-Seidel
    block in the fused form).  Each counter is scaled by bytes / reading of the
    reference copy kernel of the same run (torch.mul over COPY_BYTES, read +
    write).  Writes the record into profiles/traffic.json under KEY."""
    import csv
    key, fetch_csv, write_csv, driver_log = args.pmc_summary
    drv = json.loads([ln for ln in open(driver_log) if ln.startswith('{"profile"')][-1])
    kname = ("k_vsweep<" if drv["profile"] == "batched" else
             "k_inplace<" if drv["profile"].startswith("inplace") else
             "k_probe_gather<" if drv["profile"].startswith("probe") else "k_sweep<")

    def read(path, counter):
        sweep, copy = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0  # KiB per dispatch
            if kname in r["Kernel_Name"]:
                sweep.append(v)
            elif "MulFunctor" in r["Kernel_Name"]:
                copy.append(v)
        if not sweep or not copy:
            raise SystemExit("%s: no sweep or reference copy dispatches for %s" % (path, counter))
        return float(np.sum(sweep)) / drv["sweeps"], float(np.median(copy)), len(sweep)
    f_sweep, f_copy, n_f = read(fetch_csv, "FETCH_SIZE")
    w_sweep, w_copy, n_w = read(write_csv, "WRITE_SIZE")
    cb = drv["copy_bytes"]
    rd = f_sweep * cb / f_copy
    wr = w_sweep * cb / w_copy
    rec = {"bytes_per_sweep": int(round(rd + wr)), "read_bytes": int(round(rd)), "write_bytes": int(round(wr)),
           "fetch_scale": sig(cb / f_copy), "write_scale": sig(cb / w_copy),
           "fetch_raw_bytes_per_sweep": int(round(f_sweep)), "write_raw_bytes_per_sweep": int(round(w_sweep)),
           "launches_per_sweep": n_f // drv["sweeps"], "sweeps": drv["sweeps"], "b_alg": drv["b_alg"],
           "amplification": sig((rd + wr) / drv["b_alg"], 4), "n": drv["n"], "m": drv["m"],
           "source_sha": drv["source_sha"]}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    allrec = json.load(open(path)) if os.path.exists(path) else {}
    allrec[key] = rec
    with open(path, "w") as f:
        json.dump(allrec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps({key: rec}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline workload and R-MAT-20 forms only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default=None, metavar="LEGS",
                    help="comma-separated legs to run alone (rmat20,er10k,adjoint,road8m), without the "
                         "headline: a quick measurement, not the benchmark line")
    ap.add_argument("--profile", default=None,
                    help="{jacobi,fused,edge_list,inplace}-{fp64,fp32} | batched | probe-{fp64,fp32}")
    ap.add_argument("--profile-sweeps", type=int, default=20)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--scales", nargs="*", type=int, default=None, metavar="SCALE",
                    help="add the permuted R-MAT legs of these scales (21-23) to the line")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("KEY", "FETCH_CSV", "WRITE_CSV", "DRIVER_LOG"))
    ap.add_argument("--study", nargs="*", default=None, metavar="WORKLOAD",
                    help="convergence study over thresholds 1e-6..1e-15 (default: er10k rmat20)")
    args = ap.parse_args()
    if args.study is not None:
        args.study = args.study or ["er10k", "rmat20"]
        study(args)
        return
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_driver(args)
        return

    import torch
    import paper_2203_09284_amd as fpr
    import oracle

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU: the HIP library has no CPU path")
    torch.cuda.set_device(0)
    # host threads for the oracle legs: one GPU's process gets a share of 16
    # host CPUs, whatever the host shows (`nproc` is reported beside it)
    cores = min(os.cpu_count() or 1, 16)

    if args.only:
        table = {"rmat20": lambda: leg_rmat20(torch, fpr, oracle, args.steps, args.warmup, cores, args),
                 "er10k": lambda: leg_er10k(torch, fpr, oracle, args.steps, args.warmup),
                 "adjoint": lambda: leg_adjoint(torch, fpr, oracle, args.steps, args.warmup, cores),
                 "road8m": lambda: leg_road(torch, fpr, oracle, max(3, args.steps // 4), 1, cores)}
        print(json.dumps({name: table[name]() for name in args.only.split(",")}), flush=True)
        return

    h = headline_rmat24(torch, fpr, oracle, args.steps, args.warmup, cores, not args.no_cpu_baseline)
    n, m, forms, kern = h["n"], h["m"], h["forms"], h["kern"]

    extra = {}
    legs = [("rmat20", lambda: leg_rmat20(torch, fpr, oracle, args.steps, args.warmup, cores, args))]
    if not args.quick:
        legs += [("er10k", lambda: leg_er10k(torch, fpr, oracle, args.steps, args.warmup)),
                 ("adjoint", lambda: leg_adjoint(torch, fpr, oracle, args.steps, args.warmup, cores)),
                 ("road8m", lambda: leg_road(torch, fpr, oracle, max(3, args.steps // 4), 1, cores))]
    legs += [("rmat%d" % sc, (lambda sc=sc: leg_scale(torch, fpr, oracle, "rmat%d" % sc, max(3, args.steps // 4),
                                                      1, cores))) for sc in args.scales or []]
    for name, fn in legs:
        try:
            extra[name] = fn()
        except Exception as e:  # reported, not fatal: the headline stands on its own
            extra[name] = dict(error=str(e)[:300])
            log("%s leg failed: %s" % (name, e))
    if "batched" in extra.get("rmat20", {}):
        extra["batched"] = extra["rmat20"].pop("batched")

    head = forms["fused-fp64"]
    b64, b32 = b_alg(n, m, 8), b_alg(n, m, 4)
    k64, k32 = kern["fused-fp64"][0], kern["fused-fp32"][0]
    out = {
        "metric": METRIC,
        "value": round(head["gteps"], 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rmat24", "graph": w_desc("rmat24"), "n": n, "m": m, "d": D, "tol": 1e-8,
                   "form": "fused-fp64", "gs_blocks": h["gs_blocks"], "step": "one solve from 1/n to L1<tol"},
        "roofline": roofline(b64 / (k64 * 1e-6) / 1e9, traffic_record("fused_fp64_rmat24"), "k_sweep<double, fused>",
                             b64, k64, h["gs_blocks"], b64 + 8 * m),
        "roofline_fp32": roofline(b32 / (k32 * 1e-6) / 1e9, traffic_record("fused_fp32_rmat24"),
                                  "k_sweep<float, fused>", b32, k32, h["gs_blocks"], b32 + 4 * m),
        "cpu_baseline": h["cpu"],
        "gather_probe": h["gather_probe"],
        "forms": {k: rounded(f) for k, f in forms.items()},
        "kernel_us": {k: {"sweep": round(v[0], 2), "finalize": round(v[1], 2)} for k, v in kern.items()},
        "speedup_vs_jacobi_fp64_time_to_tol": {
            k: sig(forms["jacobi-fp64"]["ms"] / f["ms"]) for k, f in forms.items() if k != "jacobi-fp64"},
        "tol_1e-7": h["tol_1e7"],
        "setup_s": round(h["setup_s"], 2),
    }
    # the sweep against its own gathers' floor on this device
    out["roofline"]["gather_floor_us"] = h["gather_probe"]["fp64_us"]
    out["roofline"]["vs_gather_floor"] = round(h["gather_probe"]["fp64_us"] / k64, 3)
    out["roofline_fp32"]["gather_floor_us"] = h["gather_probe"]["fp32_us"]
    out["roofline_fp32"]["vs_gather_floor"] = round(h["gather_probe"]["fp32_us"] / k32, 3)
    out.update(extra)
    print(json.dumps(out), flush=True)


def w_desc(name):
    return {"rmat20": "R-MAT scale 20, edge factor 16, a=.57 b=c=.19, seed 2, permuted ids",
            "rmat24": "R-MAT scale 24, edge factor 16, a=.57 b=c=.19, seed 5, deduplicated, BFS order"}[name]


if __name__ == "__main__":
    main()
