"""Input generators: determinism, published SplitMix64 outputs, shape checks."""
import numpy as np

import graphgen as gg


def test_splitmix64_published_sequence():
    # SplitMix64 from state 0: the first three outputs of the reference generator
    assert gg.raw(0, 0) == 0xE220A8397B1DCDAF
    assert gg.raw(0, 1) == 0x6E789E6AA1B965F4
    assert gg.raw(0, 2) == 0x06C45D188009454F


def test_uniforms_deterministic_and_in_range():
    a = gg.uniforms(5, 1, 10000)
    b = gg.uniforms(5, 1, 10000)
    c = gg.uniforms(5, 2, 10000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() < 1.0
    assert abs(a.mean() - 0.5) < 0.02


def test_er_exact_distinct_no_self_loops():
    d = gg.er_10k()
    s, t = d["src"], d["dst"]
    assert len(s) == 80_000
    assert not np.any(s == t)
    keys = s.astype(np.int64) * d["n"] + t
    assert len(np.unique(keys)) == 80_000
    assert s.min() >= 0 and s.max() < d["n"] and t.min() >= 0 and t.max() < d["n"]
    d2 = gg.er_10k()
    assert np.array_equal(d2["src"], s) and np.array_equal(d2["dst"], t)


def test_rmat_quadrant_frequencies():
    scale = 12
    s, t = gg.rmat(scale, 16, seed=9, permute=False)
    m = len(s)
    # most significant bit pair follows the quadrant probabilities
    top_s, top_t = s >> (scale - 1), t >> (scale - 1)
    freq = np.array([np.mean((top_s == a) & (top_t == b)) for a, b in ((0, 0), (0, 1), (1, 0), (1, 1))])
    want = np.array([0.57, 0.19, 0.19, 0.05])
    sigma = np.sqrt(want * (1 - want) / m)
    assert np.all(np.abs(freq - want) < 5 * sigma)


def test_permutation_is_bijection_and_relabel():
    perm = gg.permutation(1000, 3)
    assert sorted(perm.tolist()) == list(range(1000))
    s, t = gg.rmat(10, 4, seed=3, permute=False)
    s2, t2 = gg.rmat(10, 4, seed=3, permute=True)
    p = gg.permutation(1024, 3)
    assert np.array_equal(s2, p[s]) and np.array_equal(t2, p[t])


def test_dedup_canonical():
    s, t = gg.random_graph(50, 2000, 4)
    ds, dt = gg.dedup(50, s, t)
    pairs = sorted({(a, b) for a, b in zip(s.tolist(), t.tolist()) if a != b})
    assert list(zip(ds.tolist(), dt.tolist())) == pairs


def test_bfs_labels_are_a_bfs_order():
    n = 1 << 10
    s, t = gg.rmat(10, 8, seed=5)
    s, t = gg.dedup(n, s, t)
    label = gg.bfs_labels(n, s, t)
    assert sorted(label.tolist()) == list(range(n))
    order = np.argsort(label)
    nbrs = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), t.tolist()):
        nbrs[a].add(b)
        nbrs[b].add(a)
    deg = np.array([len(x) for x in nbrs])
    # root is the vertex of largest total degree (smallest id on ties)
    tot = np.bincount(s, minlength=n) + np.bincount(t, minlength=n)
    assert order[0] == int(np.argmax(tot))
    # replay the BFS: each vertex's label is assigned when its first labelled
    # neighbour is expanded, in ascending neighbour id
    expect = [-1] * n
    nxt, queue, head, scan = 0, [], 0, 0
    root = int(order[0])
    while nxt < n:
        if root < 0:
            while expect[scan] >= 0:
                scan += 1
            root = scan
        expect[root] = nxt
        nxt += 1
        queue.append(root)
        root = -1
        while head < len(queue):
            v = queue[head]
            head += 1
            for u in sorted(nbrs[v]):
                if expect[u] < 0:
                    expect[u] = nxt
                    nxt += 1
                    queue.append(u)
    assert label.tolist() == expect
    assert deg.sum() > 0


def test_sample_distinct_and_weights():
    x = gg.sample_distinct(100, 100, 1)
    assert sorted(x.tolist()) == list(range(100))
    w = gg.weights(10000, 4)
    assert w.min() >= 0.5 and w.max() < 1.5
    seeds = gg.ppr_seeds(1 << 20)
    assert len(set(seeds.tolist())) == 64


def test_road_grid_shape():
    side = 40
    s, t = gg.road_grid(side, seed=6)
    n = side * side
    assert s.dtype == np.int32 and len(s) == len(t)
    # every edge joins grid neighbours
    rs, cs = np.divmod(s, side)
    rt, ct = np.divmod(t, side)
    assert np.all(np.abs(rs - rt) + np.abs(cs - ct) == 1)
    # no repeated edge, out-degree at most 4
    key = s.astype(np.int64) * n + t
    assert len(np.unique(key)) == len(key)
    assert np.bincount(s, minlength=n).max() <= 4
    # segments: 2 * side * (side - 1) candidates; kept ~0.75, one-way ~0.1 of kept
    und = np.unique(np.minimum(s, t).astype(np.int64) * n + np.maximum(s, t))
    cand = 2 * side * (side - 1)
    assert abs(len(und) / cand - 0.75) < 0.03
    one_way = 2 * len(und) - len(s)
    assert abs(one_way / len(und) - 0.1) < 0.03
    # deterministic; another seed differs
    s2, t2 = gg.road_grid(side, seed=6)
    assert np.array_equal(s, s2) and np.array_equal(t, t2)
    s3, _ = gg.road_grid(side, seed=7)
    assert not (len(s3) == len(s) and np.array_equal(s3, s))
