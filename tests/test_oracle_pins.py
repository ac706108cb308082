"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses an independent
route (dense linear algebra, closed forms, brute-force sets, invariants of the
fixed point, Eq. 9 and Eq. 2 written as small pure-Python loops, finite
differences).  test_pins_catch_planted_mistakes plants known mistakes in the
oracle and shows that the pins fail on each.
"""
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import dense

D = 0.85
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def l1(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum())


# ------------------------------------------------------------------ CSR ----

def test_offsetlist_example_section3():
    """Section 3's worked example of contributionList / offsetList."""
    n, edges, facts = None, [], {"offset": {}}
    with open(os.path.join(GOLDEN, "offsetlist_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.replace(":", " ").split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "edge":
                edges.append((int(tok[1]), int(tok[2])))
            elif tok[0] == "offset":
                facts["offset"][int(tok[1])] = int(tok[2])
            elif tok[0] == "cl_slots_of_vertex":
                facts["slots"] = (int(tok[1]), [int(t) for t in tok[2:]])
            elif tok[0] == "cl_sources_of_vertex":
                facts["sources"] = (int(tok[1]), [int(t) for t in tok[2:]])
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    g = oracle.csr(n, src, dst)
    v, slots = facts["slots"]
    assert list(range(g.in_ptr[v], g.in_ptr[v + 1])) == slots
    v, srcs = facts["sources"]
    assert g.in_src[g.in_ptr[v]:g.in_ptr[v + 1]].tolist() == srcs
    for i, val in facts["offset"].items():
        assert g.offset[i] == val


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_csr_brute_force(seed):
    n = 40
    src, dst = gg.random_graph(n, 300, seed)
    w = gg.weights(len(src), seed)
    g = oracle.csr(n, src, dst, w)
    # brute force: distinct non-self-loop pairs, weights summed in input order
    pairs = {}
    for i, (s, t) in enumerate(zip(src.tolist(), dst.tolist())):
        if s != t:
            pairs[(s, t)] = pairs.get((s, t), 0.0) + float(w[i])
    assert g.m == len(pairs)
    for u in range(n):
        ins = sorted(s for (s, t) in pairs if t == u)
        assert g.in_src[g.in_ptr[u]:g.in_ptr[u + 1]].tolist() == ins
        outs = sorted(t for (s, t) in pairs if s == u)
        assert g.out_dst[g.out_ptr[u]:g.out_ptr[u + 1]].tolist() == outs
        assert g.out_deg[u] == len(outs) and g.in_deg[u] == len(ins)
        for e in range(g.out_ptr[u], g.out_ptr[u + 1]):
            assert g.out_w[e] == pairs[(u, int(g.out_dst[e]))]
    # offsetList is a bijection onto CL slots and maps each out-edge to the same pair
    assert sorted(g.offset.tolist()) == list(range(g.m))
    row_of_slot = np.repeat(np.arange(n), np.diff(g.in_ptr))
    for u in range(n):
        for e in range(g.out_ptr[u], g.out_ptr[u + 1]):
            slot = g.offset[e]
            assert g.in_src[slot] == u and row_of_slot[slot] == g.out_dst[e]
            assert g.in_w[slot] == g.out_w[e]
    # edge_map sends each input edge to its merged out position (or -1 for a self-loop)
    for i, (s, t) in enumerate(zip(src.tolist(), dst.tolist())):
        if s == t:
            assert g.edge_map[i] == -1
        else:
            e = g.edge_map[i]
            assert g.out_dst[e] == t and g.out_ptr[s] <= e < g.out_ptr[s + 1]


def test_sampled_in_lists_match_csr():
    n = 2000
    src, dst = gg.random_graph(n, 30000, 7)
    g = oracle.csr(n, src, dst)
    rows = np.array([0, 5, 17, 999, 1999], np.int32)
    lists = oracle.sample_in_lists(n, src, dst, rows)
    for r, lst in zip(rows, lists):
        assert lst.tolist() == g.in_src[g.in_ptr[r]:g.in_ptr[r + 1]].tolist()


# ----------------------------------------------------- fixed point pins ----

def _graphs():
    out = []
    src, dst = gg.random_graph(300, 1500, 11)  # repeats, self-loops, dangling vertices
    out.append(("random300", 300, src, dst, None, None))
    s, t = gg.rmat(10, 8, seed=12)
    out.append(("rmat10", 1024, s, t, None, None))
    src, dst = gg.random_graph(500, 2500, 13)
    out.append(("weighted500", 500, src, dst, gg.weights(len(src), 13), None))
    src, dst = gg.random_graph(400, 1200, 14)
    p = gg.uniforms(14, 9, 400)
    p /= p.sum()
    out.append(("personalized400", 400, src, dst, None, p))
    return out


@pytest.mark.parametrize("name,n,src,dst,w,p", _graphs(), ids=[g[0] for g in _graphs()])
def test_jacobi_matches_dense_solve(name, n, src, dst, w, p):
    g = oracle.csr(n, src, dst, w)
    x, it, r = oracle.jacobi(g, D, tol=1e-15, max_iter=2000, p=p)
    xd = dense.solve(n, src, dst, w, D, p)
    assert l1(x, xd) <= 1e-12
    assert it < 2000


@pytest.mark.parametrize("name,n,src,dst,w,p", _graphs(), ids=[g[0] for g in _graphs()])
def test_fused_matches_dense_solve(name, n, src, dst, w, p):
    g = oracle.csr(n, src, dst, w)
    x, it, r = oracle.gauss_seidel(g, D, tol=1e-15, max_iter=2000, p=p)
    xd = dense.solve(n, src, dst, w, D, p)
    assert l1(x, xd) <= 1e-12


def test_leak_mode_matches_dense_leak():
    n = 300
    src, dst = gg.random_graph(n, 900, 21)
    g = oracle.csr(n, src, dst)
    x, _, _ = oracle.jacobi(g, D, tol=1e-16, max_iter=3000, dangling="leak")
    assert l1(x, dense.solve(n, src, dst, None, D, None, "leak")) <= 1e-12
    xf, _, _ = oracle.gauss_seidel(g, D, tol=1e-16, max_iter=3000, dangling="leak")
    assert l1(xf, dense.solve(n, src, dst, None, D, None, "leak")) <= 1e-12


# ------------------------------------------------ edge-list residual ----

def _distinct_cases():
    """Duplicate-free edge lists (the edge-list residual needs each pair once):
    unweighted with dangling vertices, weighted, personalized."""
    out = []
    for name, n, src, dst, w, p in _graphs():
        s2, t2 = gg.dedup(n, src, dst)
        w2 = None if w is None else gg.weights(len(s2), 91)
        out.append((name, n, s2, t2, w2, p))
    return out


@pytest.mark.parametrize("threads", [1, 3])
@pytest.mark.parametrize("name,n,src,dst,w,p", _distinct_cases(), ids=[g[0] for g in _distinct_cases()])
def test_residual_edges_is_dense_F(name, n, src, dst, w, p, threads):
    """F(x) from the raw edge list equals (1-d) p + d P x with the dense P,
    for a random x and at the dense fixed point (where the residual vanishes)."""
    P = dense.transition(n, src, dst, w)
    pv = np.full(n, 1.0 / n) if p is None else p
    x = gg.uniforms(92, 1, n) + 0.1
    x /= x.sum()
    F = (1 - D) * pv + D * (P @ x)
    r, y = oracle.residual_edges(n, src, dst, x, D, p=p, w=w, threads=threads, want_F=True)
    assert np.max(np.abs(y - F)) <= 1e-15 * np.max(F) * n
    assert abs(r - float(np.abs(F - x).sum())) <= 1e-13
    xs = dense.solve(n, src, dst, w, D, p)
    assert oracle.residual_edges(n, src, dst, xs, D, p=p, w=w, threads=threads) <= 1e-14


def test_residual_edges_closed_forms():
    """Zero residual at the closed-form fixed points of a cycle and an in-star."""
    n = 50
    s, t = gg.cycle(n)
    assert oracle.residual_edges(n, s, t, np.full(n, 1.0 / n), D) <= 1e-16
    s, t = gg.in_star(n)
    assert oracle.residual_edges(n, s, t, _in_star(n), D) <= 1e-15


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 6])
def test_residual_edges_catch_planted_mistakes(mutation):
    """Each planted mistake moves F away from the dense fixed point's F."""
    name, n, src, dst, w, p = _distinct_cases()[3]  # personalized, dangling vertices
    assert (np.bincount(src, minlength=n) == 0).any()
    xs = dense.solve(n, src, dst, w, D, p)
    assert oracle.residual_edges(n, src, dst, xs, D, p=p, w=w) <= 1e-14
    try:
        oracle.set_mutation(mutation)
        assert oracle.residual_edges(n, src, dst, xs, D, p=p, w=w) > 1e-6
    finally:
        oracle.set_mutation(0)


CLOSED = []
for _n in (7, 50):
    CLOSED.append(("cycle", _n, gg.cycle(_n), lambda n: np.full(n, 1.0 / n)))
    CLOSED.append(("complete", _n, gg.complete(_n), lambda n: np.full(n, 1.0 / n)))
    CLOSED.append(("edgeless", _n, (np.zeros(0, np.int32), np.zeros(0, np.int32)),
                   lambda n: np.full(n, 1.0 / n)))


def _in_star(n):
    xh = (1 + (n - 1) * D) / (n + (n - 1) * D)
    xl = ((1 - D) + D * xh) / n
    return np.array([xh] + [xl] * (n - 1))


def _out_star(n):
    xh = 1.0 / (n + D)
    xl = (n + D - 1) / ((n + D) * (n - 1))
    return np.array([xh] + [xl] * (n - 1))


def _bi_star(n):
    xh = (D + (1 - D) / n) / (1 + D)
    xl = (1 - xh) / (n - 1)
    return np.array([xh] + [xl] * (n - 1))


for _n in (5, 64):
    CLOSED.append(("in_star", _n, gg.in_star(_n), _in_star))
    CLOSED.append(("out_star", _n, gg.out_star(_n), _out_star))
    CLOSED.append(("bi_star", _n, gg.bi_star(_n), _bi_star))


@pytest.mark.parametrize("name,n,edges,formula", CLOSED, ids=["%s%d" % (c[0], c[1]) for c in CLOSED])
def test_closed_forms(name, n, edges, formula):
    g = oracle.csr(n, edges[0], edges[1])
    want = formula(n)
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        x, _, _ = fn(g, D, tol=1e-16, max_iter=500)
        assert np.max(np.abs(x - want)) <= 1e-15 * max(1.0, n * want.max())


@pytest.mark.parametrize("n,seed", [(7, 0), (7, 3), (50, 49)])
def test_one_hot_teleport_on_a_cycle_closed_form(n, seed):
    # Eq. 1 with p = e_s on the directed cycle v -> v+1: x_u = (1-d)[u=s] + d x_{u-1},
    # so x_{s+k} = d^k x_s with x_s = (1-d) / (1 - d^n) (the personalized teleport
    # of batched PageRank; no vertex is dangling)
    g = oracle.csr(n, *gg.cycle(n))
    k = (np.arange(n) - seed) % n
    want = (1 - D) * D ** k / (1 - D ** n)
    p = np.zeros(n)
    p[seed] = 1.0
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        x, _, _ = fn(g, D, tol=1e-17, max_iter=2000, p=p)
        assert np.max(np.abs(x - want)) <= 1e-14 * want.max()


def test_cycle_converges_after_one_sweep():
    g = oracle.csr(10, *gg.cycle(10))
    x, it, r, tr, sums = oracle.jacobi(g, D, tol=1e-30, max_iter=3, trace=True)
    assert tr[0] == 0.0


@pytest.mark.parametrize("n", [6, 40])
def test_path_leak_closed_form(n):
    g = oracle.csr(n, *gg.path(n))
    want = np.array([(1 - D ** (i + 1)) / n for i in range(n)])
    x, _, _ = oracle.jacobi(g, D, tol=1e-18, max_iter=500, dangling="leak")
    assert np.max(np.abs(x - want)) <= 1e-15 * want.max()
    # Gauss-Seidel in topological order is forward substitution: exact after one sweep
    x1, _, _, tr = oracle.gauss_seidel(g, D, tol=0.0, max_iter=2, dangling="leak", trace=True)
    assert np.max(np.abs(x1 - want)) <= 1e-15 * want.max()
    assert tr[1] == 0.0


def test_dag_one_gauss_seidel_sweep_is_exact():
    n = 200
    src, dst = gg.random_dag(n, 1200, 31)
    g = oracle.csr(n, src, dst)
    x, _, _, tr = oracle.gauss_seidel(g, D, tol=0.0, max_iter=2, dangling="leak", trace=True)
    assert tr[1] == 0.0
    assert l1(x, dense.solve(n, src, dst, None, D, None, "leak")) <= 1e-13
    # Jacobi needs about the longest-path length in sweeps on the same graph
    _, itj, _ = oracle.jacobi(g, D, tol=1e-16, max_iter=1000, dangling="leak")
    assert itj > 2


def test_sum_is_one_after_every_jacobi_sweep():
    d = gg.er_10k()
    g = oracle.csr(d["n"], d["src"], d["dst"])
    x, it, r, tr, sums = oracle.jacobi(g, D, tol=1e-13, max_iter=300, trace=True)
    assert np.max(np.abs(sums - 1.0)) <= 1e-12
    assert abs(x.sum() - 1.0) <= 1e-12


def test_contraction_and_iteration_bound():
    d = gg.er_10k()
    g = oracle.csr(d["n"], d["src"], d["dst"])
    tol = 1e-10
    x, it, r, tr, _ = oracle.jacobi(g, D, tol=tol, max_iter=200, trace=True)
    floor = 1e-14
    for k in range(1, len(tr)):
        assert tr[k] <= D * tr[k - 1] * (1 + 1e-9) + floor
    # ||x_k - x_{k-1}||_1 <= 2 d^(k-1) for probability vectors
    assert it <= math.ceil(math.log(tol / 2) / math.log(D)) + 1
    assert r < tol
    # certificate: ||x - x*||_1 <= ||F(x) - x||_1 / (1 - d)
    xs = dense.solve(d["n"], d["src"], d["dst"], None, D) if d["n"] <= 2000 else None
    cert = oracle.certificate(g, x, D)
    assert cert <= D / (1 - D) * r * (1 + 1e-6) + 1e-14
    del xs


def test_certificate_bounds_true_error():
    n = 600
    src, dst = gg.random_graph(n, 3000, 41)
    g = oracle.csr(n, src, dst)
    xs = dense.solve(n, src, dst, None, D)
    for tol in (1e-3, 1e-6, 1e-9):
        x, _, _ = oracle.jacobi(g, D, tol=tol, max_iter=1000)
        assert l1(x, xs) <= oracle.certificate(g, x, D) * (1 + 1e-9) + 1e-15


def test_gauss_seidel_sweep_counts():
    """The paper's claim (Section 6.3) that the fused form needs fewer sweeps
    holds for its literal algorithms, which leak dangling mass; with the
    dangling mass redistributed, plain Gauss-Seidel drifts in total mass and
    needs more sweeps than Jacobi, and the mass-scaled variant needs fewer."""
    s, t = gg.rmat(14, 16, seed=2)
    g = oracle.csr(1 << 14, s, t)
    _, itj_leak, _ = oracle.jacobi(g, D, tol=1e-10, max_iter=1000, dangling="leak")
    _, itf_leak, _ = oracle.gauss_seidel(g, D, tol=1e-10, max_iter=1000, dangling="leak")
    assert itf_leak < itj_leak
    xj, itj, _ = oracle.jacobi(g, D, tol=1e-10, max_iter=1000)
    xf, itf, _ = oracle.gauss_seidel(g, D, tol=1e-10, max_iter=1000)
    xs, its, _ = oracle.gauss_seidel(g, D, tol=1e-10, max_iter=1000, scaled=True)
    assert its < itj < itf
    x_ref, _, _ = oracle.jacobi(g, D, tol=1e-15, max_iter=1000)
    for x in (xj, xf, xs):
        assert l1(x, x_ref) <= 1e-9


def test_mass_scaled_fused_matches_dense_solve():
    for name, n, src, dst, w, p in _graphs():
        g = oracle.csr(n, src, dst, w)
        x, it, r = oracle.gauss_seidel(g, D, tol=1e-15, max_iter=2000, p=p, scaled=True)
        assert l1(x, dense.solve(n, src, dst, w, D, p)) <= 1e-12, name


def _eq9_gauss_seidel(n, ins, outdeg, sweeps):
    """Eq. 9 written directly: vertex i reads x_j(k+1) for in-neighbours j < i
    and x_j(k) for j >= i (no dangling vertices in the graphs used here)."""
    x = [1.0 / n] * n
    for _ in range(sweeps):
        new = list(x)
        for i in range(n):
            s = 0.0
            for j in ins[i]:
                s += (new[j] if j < i else x[j]) / outdeg[j]
            new[i] = (1.0 - D) * (1.0 / n) + D * (s + 0.0)
        x = new
    return np.array(x)


def _eq2_jacobi(n, ins, outdeg, sweeps):
    x = [1.0 / n] * n
    for _ in range(sweeps):
        x = [(1.0 - D) * (1.0 / n) + D * (sum(x[j] / outdeg[j] for j in ins[i]) + 0.0)
             for i in range(n)]
    return np.array(x)


def test_gauss_seidel_oracle_is_eq9_and_jacobi_oracle_is_eq2():
    n = 60
    src, dst = gg.random_graph(n, 400, 51, self_loops=False)
    # add a cycle so no vertex is dangling (Eq. 9 / Eq. 2 have no dangling term)
    cs, ct = gg.cycle(n)
    src = np.concatenate([src, cs]).astype(np.int32)
    dst = np.concatenate([dst, ct]).astype(np.int32)
    g = oracle.csr(n, src, dst)
    assert (g.out_deg > 0).all()
    ins = [g.in_src[g.in_ptr[u]:g.in_ptr[u + 1]].tolist() for u in range(n)]
    for sweeps in (1, 2, 5):
        xf, _, _ = oracle.gauss_seidel(g, D, tol=0.0, max_iter=sweeps)
        assert np.array_equal(xf, _eq9_gauss_seidel(n, ins, g.out_deg.tolist(), sweeps))
        xj, _, _ = oracle.jacobi(g, D, tol=0.0, max_iter=sweeps)
        assert np.array_equal(xj, _eq2_jacobi(n, ins, g.out_deg.tolist(), sweeps))


def test_linf_norm_option():
    d = gg.er_10k()
    g = oracle.csr(d["n"], d["src"], d["dst"])
    x1, it1, r1 = oracle.jacobi(g, D, tol=1e-12, max_iter=500, norm="linf")
    assert r1 < 1e-12
    x2, it2, r2 = oracle.jacobi(g, D, tol=1e-12, max_iter=500, norm="l1")
    assert it1 <= it2  # max-norm <= L1 norm


def test_threads_do_not_change_result():
    s, t = gg.rmat(12, 16, seed=61)
    g = oracle.csr(1 << 12, s, t)
    x1, i1, r1 = oracle.jacobi(g, D, tol=1e-10, threads=1)
    x4, i4, r4 = oracle.jacobi(g, D, tol=1e-10, threads=4)
    assert np.array_equal(x1, x4) and i1 == i4 and r1 == r4


# --------------------------------------------------------------- adjoint ---

def _adjoint_case(seed=71, n=150, m=700):
    src, dst = gg.random_graph(n, m, seed)
    w = gg.weights(len(src), seed)
    p = np.full(n, 1.0 / n)
    targets = gg.sample_distinct(n, 20, seed)
    gvec = np.zeros(n)
    gvec[targets] = 1.0
    return n, src, dst, w, p, gvec


def test_adjoint_matches_dense_gradient():
    n, src, dst, w, p, gvec = _adjoint_case()
    g = oracle.csr(n, src, dst, w)
    x, _, _ = oracle.jacobi(g, D, tol=1e-15, max_iter=3000)
    lam, gp, gw, it, r = oracle.adjoint(g, x, gvec, D)
    lam_d = dense.adjoint(n, src, dst, w, D, gvec)
    assert l1(lam, lam_d) <= 1e-10 * np.abs(lam_d).sum()
    assert l1(gp, (1 - D) * lam_d) <= 1e-10 * np.abs(lam_d).sum()
    ref = dense.gradient_weights(n, src, dst, w, D, p, gvec)
    got = np.array([gw[e] for v in range(n) for e in range(g.out_ptr[v], g.out_ptr[v + 1])])
    want = np.array([ref[(v, int(g.out_dst[e]))] for v in range(n)
                     for e in range(g.out_ptr[v], g.out_ptr[v + 1])])
    assert l1(got, want) <= 1e-10 * np.abs(want).sum()


def test_adjoint_matches_finite_differences():
    n, src, dst, w, p, gvec = _adjoint_case(seed=72, n=80, m=400)
    g = oracle.csr(n, src, dst, w)
    x, _, _ = oracle.jacobi(g, D, tol=1e-15, max_iter=3000)
    lam, gp, gw, _, _ = oracle.adjoint(g, x, gvec, D)
    rng_edges = gg.sample_distinct(len(src), 12, 72, 5)
    for i in rng_edges.tolist():
        if src[i] == dst[i]:
            continue
        e = g.edge_map[i]
        fd = dense.gradient_fd_weight(n, src, dst, w, D, p, gvec, i)
        assert abs(gw[e] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gw).max())
    for u in gg.sample_distinct(n, 8, 72, 6).tolist():
        fd = dense.gradient_fd_p(n, src, dst, w, D, p, gvec, u)
        assert abs(gp[u] - fd) <= 1e-7 * max(abs(fd), 1.0)


def test_adjoint_duality_and_homogeneity():
    n, src, dst, w, p, gvec = _adjoint_case(seed=73, n=400, m=2400)
    g = oracle.csr(n, src, dst, w)
    x, _, _ = oracle.jacobi(g, D, tol=1e-15, max_iter=3000)
    lam, gp, gw, _, _ = oracle.adjoint(g, x, gvec, D)
    L = float(np.dot(gvec, x))
    assert abs(L - (1 - D) * float(np.dot(lam, p))) <= 1e-12 * abs(L)
    for v in range(n):
        a, b = g.out_ptr[v], g.out_ptr[v + 1]
        if b > a:
            s = float(np.dot(g.out_w[a:b], gw[a:b]))
            assert abs(s) <= 1e-12 * max(1.0, float(np.abs(g.out_w[a:b] * gw[a:b]).sum()))


# ------------------------------------------------------ planted mistakes ---

def _pins_pass():
    """A quick subset of the pins above, returning False on the first failure."""
    n, src, dst, w, p, gvec = _adjoint_case(seed=81, n=120, m=500)
    g = oracle.csr(n, src, dst, w)
    x, _, _ = oracle.jacobi(g, D, tol=1e-15, max_iter=3000)
    if l1(x, dense.solve(n, src, dst, w, D)) > 1e-12:
        return False
    rs, rt = gg.rmat(7, 4, seed=82)  # about half the vertices dangling
    gu = oracle.csr(128, rs, rt)
    assert (gu.out_deg == 0).sum() > 20
    xu, _, _ = oracle.jacobi(gu, D, tol=1e-15, max_iter=3000)
    if l1(xu, dense.solve(128, rs, rt, None, D)) > 1e-12:
        return False
    cs, ct = gg.cycle(9)
    pc = np.zeros(9)
    pc[4] = 1.0
    xc, _, _ = oracle.jacobi(oracle.csr(9, cs, ct), D, tol=1e-17, max_iter=2000, p=pc)
    if np.max(np.abs(xc - (1 - D) * D ** ((np.arange(9) - 4) % 9) / (1 - D ** 9))) > 1e-14:
        return False
    lam, gp, gw, _, _ = oracle.adjoint(g, x, gvec, D)
    for v in range(n):
        a, b = g.out_ptr[v], g.out_ptr[v + 1]
        if b > a and abs(float(np.dot(g.out_w[a:b], gw[a:b]))) > 1e-12:
            return False
    return True


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6])
def test_pins_catch_planted_mistakes(mutation):
    assert _pins_pass()
    try:
        oracle.set_mutation(mutation)
        assert not _pins_pass(), "pins missed planted mistake %d" % mutation
    finally:
        oracle.set_mutation(0)
    assert _pins_pass()


def test_par_fused_host_variant():
    """The host parallel fused variant (Section 6.3): one thread is exactly the
    mass-scaled sequential loop; several threads reach the Jacobi fixed point,
    which the dense solve pins."""
    n = 300
    s, t = gg.random_graph(n, 1800, 31)
    og = oracle.csr(n, s, t)
    x_dense = dense.solve(n, s, t, None, 0.85, None)
    xs, its, _ = oracle.gauss_seidel(og, 0.85, tol=1e-14, max_iter=2000, scaled=True)
    x1, it1, _ = oracle.gauss_seidel_threads(og, 0.85, tol=1e-14, max_iter=2000, scaled=True, threads=1)
    assert it1 == its and np.array_equal(x1, xs)
    for th in (2, 4, 8):
        for scaled in (True, False):
            x, it, r = oracle.gauss_seidel_threads(og, 0.85, tol=1e-14, max_iter=5000, scaled=scaled, threads=th)
            assert r < 1e-14
            assert np.abs(x - x_dense).sum() <= 1e-12
