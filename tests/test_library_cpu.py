"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/fusedpr.h declares, and its host CSR builder matches
the oracle's independent CSR bit for bit."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import graphgen as gg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fusedpr.h")


def _lib():
    from paper_2203_09284_amd import _lib as L
    return L, L.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pr_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pr_build_csr", "pr_solve", "pr_iterate", "pr_solve_batched", "pr_adjoint",
                     "pr_graph_create", "pr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(pr_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)
        assert n in L.SIGNATURES, "binding lacks %s" % n


def _compare_csr(n, src, dst, w=None):
    from paper_2203_09284_amd.graph import build_csr
    L, lib = _lib()
    csr, c = build_csr(n, src, dst, w)
    lib.pr_csr_free(ctypes.byref(csr))
    o = oracle.csr(n, src, dst, w)
    assert c.m == o.m
    assert np.array_equal(c.in_ptr, o.in_ptr)
    assert np.array_equal(c.in_src, o.in_src)
    assert np.array_equal(c.out_ptr, o.out_ptr)
    assert np.array_equal(c.out_dst, o.out_dst)
    assert np.array_equal(c.out_to_in, o.offset)
    assert np.array_equal(c.out_deg, o.out_deg)
    assert np.array_equal(c.in_deg, o.in_deg)
    assert np.array_equal(c.edge_map, o.edge_map)
    if w is not None:
        assert np.array_equal(c.in_w, o.in_w)  # bit-exact: same summation order
        assert np.array_equal(c.out_w, o.out_w)
    else:
        assert c.in_w is None and c.out_w is None


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_csr_bit_exact_small(seed):
    src, dst = gg.random_graph(60, 700, seed)
    _compare_csr(60, src, dst)
    _compare_csr(60, src, dst, gg.weights(len(src), seed))


def test_csr_bit_exact_er10k():
    d = gg.er_10k()
    _compare_csr(d["n"], d["src"], d["dst"])


def test_csr_bit_exact_rmat16_with_repeats():
    s, t = gg.rmat(16, 16, seed=2)
    _compare_csr(1 << 16, s, t)
    _compare_csr(1 << 16, s, t, gg.weights(len(s), 2))


def test_csr_edge_cases():
    _compare_csr(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    _compare_csr(5, np.array([1, 1, 1], np.int32), np.array([1, 1, 1], np.int32))  # only self-loops
    _compare_csr(3, np.array([0, 0, 0, 2], np.int32), np.array([1, 1, 1, 1], np.int32))
    _compare_csr(*((6,) + gg.complete(6)))


def test_csr_errors():
    from paper_2203_09284_amd.graph import build_csr
    from paper_2203_09284_amd._lib import FusedPRError
    with pytest.raises(FusedPRError, match="outside"):
        build_csr(4, np.array([0, 5], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(FusedPRError, match="outside"):
        build_csr(4, np.array([0, -1], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(FusedPRError, match="weight"):
        build_csr(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, np.nan]))
    with pytest.raises(FusedPRError, match="weight"):
        build_csr(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, 0.0]))
    with pytest.raises(FusedPRError):
        build_csr(0, np.zeros(0, np.int32), np.zeros(0, np.int32))


def test_error_message_is_thread_local_and_cleared():
    from paper_2203_09284_amd.graph import build_csr
    from paper_2203_09284_amd._lib import FusedPRError
    L, lib = _lib()
    with pytest.raises(FusedPRError):
        build_csr(4, np.array([0, 9], np.int32), np.array([1, 2], np.int32))
    assert b"outside" in lib.pr_last_error()
    csr, _ = build_csr(4, np.array([0], np.int32), np.array([1], np.int32))
    lib.pr_csr_free(ctypes.byref(csr))
    assert lib.pr_last_error() == b""


def _source_lines(folder, exts):
    for dirpath, _, files in os.walk(os.path.join(ROOT, folder)):
        if "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith(exts):
                path = os.path.join(dirpath, f)
                for ln in open(path, errors="replace"):
                    yield os.path.relpath(path, ROOT), ln


def test_product_and_oracle_share_no_code():
    # The library and its binding never import, include or load the oracle;
    # the oracle never reaches into the library; the input generators use neither.
    link = re.compile(r"^\s*(import|from|#\s*include)\b|CDLL|dlopen|\.so\b")
    for path, ln in _source_lines("paper_2203_09284_amd", (".py", ".hip", ".h", ".cpp")):
        assert not (link.search(ln) and "oracle" in ln), (path, ln)
    for folder in ("oracle", "graphgen"):
        for path, ln in _source_lines(folder, (".py", ".c", ".h")):
            if link.search(ln):
                assert "paper_2203_09284_amd" not in ln and "fusedpr" not in ln and "csrc" not in ln, (path, ln)
    for path, ln in _source_lines("graphgen", (".py",)):
        assert not (link.search(ln) and "oracle" in ln), (path, ln)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    from paper_2203_09284_amd import _lib as L
    monkeypatch.setattr(L, "_LIBS", {})
    monkeypatch.setattr(L, "VARIANTS", {"": str(tmp_path / "missing.so"), "naive": str(tmp_path / "gone.so")})
    with pytest.raises(ImportError, match="not built"):
        L.lib()
    with pytest.raises(ImportError, match="not built"):
        L.lib("naive")


def test_every_compute_entry_point_cites_the_paper():
    text = open(HEADER).read()
    cited = {}
    for m in re.finditer(r"(/\*.*?\*/)\s*(?:[a-z_0-9 ]+\*?\s*)(pr_[a-z_0-9]+)\s*\(", text, flags=re.S):
        cited[m.group(2)] = bool(re.search(r"Section \d|Eq\. ?\d|Algorithm \d|Fig\. ?\d", m.group(1)))
    for name in ("pr_build_csr", "pr_graph_create", "pr_solve", "pr_iterate", "pr_profile_sweeps",
                 "pr_certificate", "pr_solve_batched", "pr_autotune_batched", "pr_adjoint"):
        assert cited.get(name), name


def _csr_view(c):
    """A pr_csr whose arrays are the given numpy arrays (kept alive by the caller)."""
    from paper_2203_09284_amd import _lib as L
    p = lambda a, t: a.ctypes.data_as(t) if a is not None else None
    return L.PrCsr(n=c["n"], m=c["m"], in_ptr=p(c["in_ptr"], L.c_i64p), in_src=p(c["in_src"], L.c_i32p),
                   in_w=None, out_ptr=p(c["out_ptr"], L.c_i64p), out_dst=p(c["out_dst"], L.c_i32p), out_w=None,
                   out_to_in=p(c["out_to_in"], L.c_i64p), out_deg=p(c["out_deg"], L.c_i32p),
                   in_deg=p(c["in_deg"], L.c_i32p), m_input=0, edge_map=None)


def test_graph_create_refuses_a_malformed_csr():
    # the structural checks run before any device work, so they hold without a GPU
    from paper_2203_09284_amd.graph import build_csr
    L, lib = _lib()
    src, dst = gg.random_graph(50, 300, 7)
    csr, c = build_csr(50, src, dst)
    lib.pr_csr_free(ctypes.byref(csr))
    good = dict(n=c.n, m=c.m, in_ptr=c.in_ptr.copy(), in_src=c.in_src.copy(), out_ptr=c.out_ptr.copy(),
                out_dst=c.out_dst.copy(), out_to_in=c.out_to_in.copy(), out_deg=c.out_deg.copy(),
                in_deg=c.in_deg.copy())
    bad_cases = []
    b = dict(good, in_ptr=good["in_ptr"].copy())
    b["in_ptr"][5], b["in_ptr"][6] = b["in_ptr"][6] + 1, b["in_ptr"][5]
    bad_cases.append((b, "decreasing offsets"))
    b = dict(good, in_src=good["in_src"].copy())
    b["in_src"][3] = 50
    bad_cases.append((b, "outside"))
    b = dict(good, out_deg=good["out_deg"].copy())
    b["out_deg"][0] += 1
    bad_cases.append((b, "out_deg"))
    b = dict(good, out_ptr=good["out_ptr"].copy())
    b["out_ptr"][-1] -= 1
    bad_cases.append((b, "span"))
    b = dict(good, out_dst=None)
    bad_cases.append((b, "not a pr_build_csr result"))
    for arrays, msg in bad_cases:
        view = _csr_view(arrays)
        po = L.PrPlanOpts()
        lib.pr_plan_opts_default(ctypes.byref(po))
        h = ctypes.c_void_p()
        rc = lib.pr_graph_create(ctypes.byref(view), ctypes.byref(po), ctypes.byref(h))
        assert rc == L.PR_EINVAL and not h.value, msg
        assert msg.encode() in lib.pr_last_error(), (msg, lib.pr_last_error())
