"""The benchmark's host-side arithmetic (no GPU): the one-GPU guard, the
algorithmic bytes, the roofline fields, the counter-run summary (scaling by
the reference copy kernel) and the source-hash key of the recorded traffic."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes():
    # 4 B per edge id, 8 B per row offset, a rank read and written, a degree read
    assert bench.b_alg(10, 100, 8) == 4 * 100 + 8 * 11 + 2 * 8 * 10 + 4 * 10
    assert bench.b_alg(1 << 20, 16086543, 8) == 93706308


def test_roofline_fields():
    r = bench.roofline(1262.2, 237462286, "k", 93706308, 74.24, 2, edge_bytes=222398652)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - 1262.2 / 8000.0) < 1e-4
    assert abs(r["traffic_gbs"] - 237462286 / 74.24e-6 / 1e9) < 0.1
    assert abs(r["edge_gbs"] - 222398652 / 74.24e-6 / 1e9) < 0.1
    assert bench.roofline(1.0, None, "k", 1, 1.0, 1)["traffic"] is None


def _counter_csv(path, counter, sweep_kib, copy_kib):
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i, v in enumerate(sweep_kib):
        rows.append('%d,"void (anonymous namespace)::k_sweep<double, true, 0>(args)",%s,%r' % (i, counter, v))
    for i, v in enumerate(copy_kib):
        rows.append('%d,"void at::native::vectorized_elementwise_kernel<MulFunctor>",%s,%r' % (100 + i, counter, v))
    path.write_text("\n".join(rows) + "\n")


def test_counter_summary_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    cb = bench.COPY_BYTES
    # 4 dispatches (2 sweeps of 2 launches); the copy reads cb bytes and FETCH_SIZE shows half
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [1000.0, 1000.0, 3000.0, 3000.0], [cb / 2048.0] * 5)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [500.0, 500.0, 500.0, 500.0], [cb / 1024.0] * 5)
    drv = {"profile": "fused-fp64", "workload": "x", "n": 10, "m": 100, "sweeps": 2, "copy_bytes": cb,
           "b_alg": 1000, "source_sha": "abc"}
    (tmp_path / "d.log").write_text("noise\n" + json.dumps(drv) + "\n")

    class A:
        pmc_summary = ["key", str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "d.log")]
    bench.pmc_summary(A())
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))["key"]
    assert rec["launches_per_sweep"] == 2
    assert abs(rec["fetch_scale"] - 2.0) < 1e-6 and abs(rec["write_scale"] - 1.0) < 1e-6
    # per sweep: (1000 + 1000 + 3000 + 3000) KiB / 2 sweeps, times 2 for reads
    assert rec["read_bytes"] == 4000 * 1024 * 2
    assert rec["write_bytes"] == 1000 * 1024
    assert rec["bytes_per_sweep"] == rec["read_bytes"] + rec["write_bytes"]
    assert rec["source_sha"] == "abc"


def test_recorded_traffic_is_dropped_when_the_sources_change(monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = "fused_fp64_rmat20"
    assert key in rec
    monkeypatch.setattr(bench, "kernel_source_sha", lambda files=bench.KERNEL_SOURCES: rec[key]["source_sha"])
    assert bench.traffic_record(key) == rec[key]["bytes_per_sweep"]
    monkeypatch.setattr(bench, "kernel_source_sha", lambda files=bench.KERNEL_SOURCES: "0" * 16)
    assert bench.traffic_record(key) is None


def test_no_gpu_is_an_error_not_a_cpu_run():
    import pytest
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "needs a GPU" in r.stderr
    assert '"metric"' not in r.stdout


def test_host_thread_scaling_leg():
    import graphgen as gg
    import numpy as np
    import oracle
    s, t = gg.rmat(10, 8, seed=5)
    og = oracle.csr(1 << 10, s, t)
    rows = bench.host_scaling(oracle, og, 1e-10, 4)
    assert [r["threads"] for r in rows] == [1, 2, 4]
    _, it_ec, _ = oracle.jacobi(og, bench.D, tol=1e-10, max_iter=1000)
    _, it_f, _ = oracle.gauss_seidel(og, bench.D, tol=1e-10, max_iter=1000, scaled=True)
    assert rows[0]["ec_sweeps"] == it_ec and rows[0]["fused_sweeps"] == it_f
    # the edge-centric form is deterministic at any thread count; the fused one
    # is asynchronous across threads but still reaches the tolerance
    assert all(r["ec_sweeps"] == it_ec for r in rows)
    assert all(1 <= r["fused_sweeps"] < 1000 and np.isfinite(r["fused_speedup_vs_ec"]) for r in rows)


def test_committed_traffic_records_match_the_committed_sources():
    """Every counter record the benchmark reads was taken with the kernel
    sources as committed (a change to a kernel source without new counter
    runs would make the bench report null traffic)."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    used = {"fused_fp64_rmat24": bench.KERNEL_SOURCES, "fused_fp32_rmat24": bench.KERNEL_SOURCES,
            "fused_fp64_rmat20": bench.KERNEL_SOURCES, "inplace_fp64_road8m": bench.KERNEL_SOURCES,
            "batched_rmat20": bench.BATCHED_SOURCES, "probe_fp64_rmat24": bench.PROBE_SOURCES,
            "probe_fp32_rmat24": bench.PROBE_SOURCES}
    for key, files in used.items():
        assert key in rec, key
        assert rec[key]["source_sha"] == bench.kernel_source_sha(files), key
        assert bench.traffic_record(key, files) == rec[key]["bytes_per_sweep"], key
