"""Pins of the oracle's neighbor-sampling loop (fig:api(b)) on CPU."""
import collections

import numpy as np
import pytest

import oracle
from paper_2009_09103_amd import inputs


@pytest.fixture(scope="module")
def tiny():
    rp, col = inputs.graph_for(inputs.TINY)
    offs, seeds = inputs.single_instance_seeds(rp, col, inputs.TINY["num_seeds"], inputs.TINY["seed_rng"])
    return rp, col, offs, seeds


def bfs_levels(rowptr, col, sources, depth):
    """Plain BFS (networkx) levels 0..depth-1 from a source set."""
    import networkx as nx
    n = len(rowptr) - 1
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    for u in range(n):
        for e in range(rowptr[u], rowptr[u + 1]):
            G.add_edge(u, int(col[e]))
    levels = [sorted(set(int(s) for s in sources))]
    seen = set(levels[0])
    for _ in range(depth - 1):
        nxt = set()
        for u in levels[-1]:
            for x in G.successors(u):
                if x not in seen:
                    nxt.add(x)
        seen |= nxt
        levels.append(sorted(nxt))
    return levels


def test_take_all_is_bfs(tiny):
    """NeighborSize >= pool (snowball sampling, Section II-A): each layer's
    frontier is exactly the BFS level and every out-edge of it is emitted, in
    (src, adjacency) order."""
    rp, col, offs, seeds = tiny
    src0 = seeds[:16]
    res = oracle.sample(rp, col, None, np.array([0, 16]), src0, [-1, -1, -1])
    levels = bfs_levels(rp, col, src0, 3)
    for l, lev in enumerate(levels):
        s, d = res.segment(l, 0)
        want_s = np.concatenate([np.full(rp[u + 1] - rp[u], u) for u in lev]) if lev else []
        want_d = np.concatenate([col[rp[u]:rp[u + 1]] for u in lev]) if lev else []
        np.testing.assert_array_equal(s, want_s)
        np.testing.assert_array_equal(d, want_d)


def check_invariants(rp, col, b_of, offs, seeds, fanouts, res):
    ni = len(offs) - 1
    L = len(fanouts)
    for i in range(ni):
        visited = set(int(x) for x in seeds[offs[i]:offs[i + 1]])
        frontier = sorted(visited)
        expanded = set()
        for l in range(L):
            s, d = res.segment(l, i)
            # sources appear in increasing order, each once per instance
            srcs = list(dict.fromkeys(s.tolist()))
            assert srcs == sorted(srcs)
            per = collections.defaultdict(list)
            for u, x in zip(s.tolist(), d.tolist()):
                per[u].append(x)
            for u in frontier:
                b = b_of(u)
                P = int((b > 0).sum())
                want = min(fanouts[l], P) if fanouts[l] >= 0 else P
                got = per.get(u, [])
                assert len(got) == want
                assert len(set(got)) == len(got)                  # without replacement
                nbrs = col[rp[u]:rp[u + 1]]
                idx = np.searchsorted(nbrs, got)
                assert np.all(nbrs[idx] == got)                   # edges of G
                assert np.all(b[idx] > 0)                         # zero bias never chosen
            assert set(per) <= set(frontier)
            assert not (set(frontier) & expanded)                 # expanded once
            expanded |= set(frontier)
            nxt = sorted(set(d.tolist()) - visited)
            visited |= set(nxt)
            frontier = nxt


def test_tiny_uniform_invariants(tiny):
    rp, col, offs, seeds = tiny
    res = oracle.sample(rp, col, None, offs, seeds, [10, 5], rng_seed=1)
    check_invariants(rp, col, lambda u: np.ones(rp[u + 1] - rp[u], dtype=np.int64), offs, seeds,
                     [10, 5], res)
    assert res.num_edges > 1000


def test_degree_bias_invariants_and_equivalence(tiny):
    """NEIGHBOR_DEGREE equals EDGE_WEIGHT with w = out-degree of the destination."""
    rp, col, offs, seeds = tiny
    deg = np.diff(rp)
    r1 = oracle.sample(rp, col, None, offs, seeds, [25, 10, 5], bias_kind=oracle.NEIGHBOR_DEGREE, rng_seed=2)
    ew = inputs.dst_outdeg_weights(rp, col)
    r2 = oracle.sample(rp, col, ew, offs, seeds, [25, 10, 5], bias_kind=oracle.EDGE_WEIGHT, rng_seed=2)
    np.testing.assert_array_equal(r1.src, r2.src)
    np.testing.assert_array_equal(r1.dst, r2.dst)
    np.testing.assert_array_equal(r1.offsets, r2.offsets)
    check_invariants(rp, col, lambda u: deg[col[rp[u]:rp[u + 1]]], offs, seeds, [25, 10, 5], r1)


def test_instances_are_independent_of_batch(tiny):
    """An instance's edges depend only on its id, seeds and fanouts: sampling
    it alone (same id) gives the same segment as inside a batch; threads and
    batch order change nothing."""
    rp, col, _, _ = tiny
    g = inputs.rng(5)
    pool = inputs.non_isolated(rp, col)
    sets = [inputs.distinct_seeds(g, pool, int(k)) for k in g.integers(1, 40, size=12)]
    offs = np.zeros(13, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in sets])
    seeds = np.concatenate(sets)
    fo = np.array([[10, 5, 0], [25, 10, 5]] * 6, dtype=np.int32)
    bk = np.array([0, 2] * 6, dtype=np.int32)
    ids = np.arange(100, 112, dtype=np.uint64)
    batch = oracle.sample(rp, col, None, offs, seeds, fo, rng_seed=9, instance_ids=ids, bias_kinds=bk,
                          nthreads=4)
    single_thread = oracle.sample(rp, col, None, offs, seeds, fo, rng_seed=9, instance_ids=ids,
                                  bias_kinds=bk, nthreads=1)
    np.testing.assert_array_equal(batch.dst, single_thread.dst)
    for i in (0, 5, 11):
        alone = oracle.sample(rp, col, None, np.array([0, len(sets[i])]), sets[i], fo[i],
                              rng_seed=9, instance_base=100 + i, bias_kind=int(bk[i]))
        for l in range(3):
            np.testing.assert_array_equal(batch.segment(l, i)[1], alone.segment(l, 0)[1])
            np.testing.assert_array_equal(batch.segment(l, i)[0], alone.segment(l, 0)[0])


def test_frontier_split_over_threads_equals_one_thread(tiny):
    """With fewer instances than threads the oracle splits each layer's
    frontier over the threads; edges, order and byte counts equal the
    one-thread run (one instance, two instances, forest fire)."""
    rp, col, offs, seeds = tiny
    deg = np.diff(rp).astype(np.uint32)
    ew = deg[col] + 1
    for ni, kw in ((1, {}), (2, {}), (1, dict(burn=int(0.7 * 2 ** 32)))):
        so = np.array([0, len(seeds)] if ni == 1 else [0, 100, len(seeds)], dtype=np.int64)
        for bias in (oracle.UNIFORM, oracle.EDGE_WEIGHT, oracle.NEIGHBOR_DEGREE):
            one = oracle.sample(rp, col, ew, so, seeds, [25, 10, 5], bias_kind=bias, rng_seed=3, nthreads=1, **kw)
            many = oracle.sample(rp, col, ew, so, seeds, [25, 10, 5], bias_kind=bias, rng_seed=3, nthreads=7, **kw)
            np.testing.assert_array_equal(one.src, many.src)
            np.testing.assert_array_equal(one.dst, many.dst)
            np.testing.assert_array_equal(one.offsets, many.offsets)
            assert (one.alg_bytes, one.expanded, one.fallbacks, one.draws) == \
                (many.alg_bytes, many.expanded, many.fallbacks, many.draws)
            assert one.num_edges > 500


def test_degenerate_cases():
    # 0 -> 1, 0 -> 2 (weight 0), 1 -> nothing; 3 isolated
    rp = np.array([0, 2, 2, 2, 2], dtype=np.int64)
    col = np.array([1, 2], dtype=np.int32)
    ew = np.array([4, 0], dtype=np.uint32)
    # no instances
    r = oracle.sample(rp, col, ew, np.array([0]), np.array([], dtype=np.int32), [3])
    assert r.num_edges == 0
    # empty seed set, duplicate seeds, sink seed, zero-weight neighbor
    offs = np.array([0, 0, 3, 4])
    seeds = np.array([0, 0, 1, 3], dtype=np.int32)
    r = oracle.sample(rp, col, ew, offs, seeds, [5, 5], bias_kind=oracle.EDGE_WEIGHT)
    assert r.segment(0, 0)[0].size == 0
    np.testing.assert_array_equal(r.segment(0, 1)[1], [1])   # only the positive-weight edge
    assert r.segment(0, 2)[0].size == 0
    assert r.num_edges == 1                                  # vertex 1 was a seed: not re-expanded
    # all-zero weights: nothing selected
    r = oracle.sample(rp, col, np.zeros(2, dtype=np.uint32), np.array([0, 1]), np.array([0], dtype=np.int32),
                      [1], bias_kind=oracle.EDGE_WEIGHT)
    assert r.num_edges == 0
    # a zero fanout ends the instance's layers
    r = oracle.sample(rp, col, None, np.array([0, 1]), np.array([0], dtype=np.int32), [1, 0, 1])
    assert r.num_edges == 1
    with pytest.raises(ValueError):
        oracle.sample(rp, col, None, np.array([0, 1]), np.array([4], dtype=np.int32), [1])
    with pytest.raises(ValueError):
        oracle.sample(rp, col, None, np.array([0, 1]), np.array([0], dtype=np.int32), [-2])


def test_paper_toy_graph_degree_bias():
    """On the reconstructed toy graph, v8's EdgeBias list under the degree bias
    is (3,6,2,2,2) and the biased selection from v8 follows Theorem 1."""
    rp, col = inputs.paper_toy_graph()
    assert col[rp[8]:rp[9]].tolist() == [5, 7, 9, 10, 11]
    assert np.diff(rp)[[5, 7, 9, 10, 11]].tolist() == [3, 6, 2, 2, 2]
    n = 30000
    res = oracle.sample(rp, col, None, np.arange(n + 1), np.full(n, 8, dtype=np.int32), [1],
                        bias_kind=oracle.NEIGHBOR_DEGREE, rng_seed=3)
    freq = {x: c / n for x, c in zip(*np.unique(res.dst, return_counts=True))}
    for x, b in zip([5, 7, 9, 10, 11], [3, 6, 2, 2, 2]):
        assert abs(freq[x] - b / 15) < 0.01
