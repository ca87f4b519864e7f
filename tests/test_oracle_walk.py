"""Pins of the oracle's random walks (Section II-A) on CPU.

The exact distribution of the walker's position after t steps is computed here
from the transition matrix (first-order walks) or from the second-order
edge-state chain (node2vec), with numpy, and compared by chi-square with the
positions of many independent walkers.
"""
import collections

import networkx as nx
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2009_09103_amd import inputs

NW = 60_000


def small_graph(seed=3, n=10, m=22, directed=False):
    G = nx.gnm_random_graph(n, m, seed=seed, directed=directed)
    edges = list(G.edges())
    if not directed:
        edges += [(v, u) for u, v in edges]
    return inputs.csr_from_edges(n, edges)


def first_order_matrix(rp, col, b):
    n = len(rp) - 1
    P = np.zeros((n + 1, n + 1))          # state n = stopped
    for v in range(n):
        w = b[rp[v]:rp[v + 1]].astype(np.float64)
        if w.sum() == 0:
            P[v, n] = 1.0
        else:
            for x, wx in zip(col[rp[v]:rp[v + 1]], w):
                P[v, x] += wx / w.sum()
    P[n, n] = 1.0
    return P


def compare(counts, probs):
    nz = probs > 0
    assert np.all(counts[~nz] == 0)
    if nz.sum() > 1:
        assert stats.chisquare(counts[nz], probs[nz] / probs[nz].sum() * counts.sum()).pvalue > 1e-4


@pytest.mark.parametrize("kind", ["uniform", "edge_weight", "neighbor_degree"])
def test_first_order_t_step_law(kind):
    rp, col = small_graph(seed=4, n=9, m=20, directed=True)    # directed: sinks possible
    n = len(rp) - 1
    g = np.random.Generator(np.random.PCG64(1))
    if kind == "uniform":
        bk, ew, b = oracle.UNIFORM, None, np.ones(len(col))
    elif kind == "edge_weight":
        ew = g.integers(0, 9, size=len(col)).astype(np.uint32)
        bk, b = oracle.EDGE_WEIGHT, ew
    else:
        bk, ew, b = oracle.NEIGHBOR_DEGREE, None, np.diff(rp)[col]
    start = int(np.argmax(np.diff(rp)))
    T = 4
    paths, steps, _ = oracle.walk(rp, col, ew, np.full(NW, start, dtype=np.int32), T, bias_kind=bk,
                                  rng_seed=11)
    P = first_order_matrix(rp, col, b)
    p = np.zeros(n + 1)
    p[start] = 1
    for t in range(1, T + 1):
        p = p @ P
        pos = paths[:, t]
        counts = np.bincount(np.where(pos < 0, n, pos), minlength=n + 1)
        compare(counts, p)
    # padding: -1 only after the walk stopped, steps = number of valid moves
    valid = (paths[:, 1:] >= 0)
    assert np.all(valid.sum(axis=1) == steps)
    assert np.all(np.diff(valid.astype(int), axis=1) <= 0)


def test_unbiased_stationary_degree_proportional():
    """Connected, non-bipartite, undirected: visit frequencies of a simple
    random walk converge to deg(v) / 2|E|."""
    G = nx.connected_watts_strogatz_graph(30, 4, 0.3, seed=2)
    assert nx.is_connected(G) and not nx.is_bipartite(G)
    edges = list(G.edges()) + [(v, u) for u, v in G.edges()]
    rp, col = inputs.csr_from_edges(30, edges)
    paths, _, _ = oracle.walk(rp, col, None, np.zeros(2000, dtype=np.int32), 400, rng_seed=5)
    visits = np.bincount(paths[:, 100:].ravel(), minlength=30).astype(np.float64)
    freq = visits / visits.sum()
    deg = np.diff(rp).astype(np.float64)
    assert 0.5 * np.abs(freq - deg / deg.sum()).sum() < 0.02


def node2vec_exact(rp, col, start, T, wr, wc, wo):
    """Exact distribution of the position after 1..T steps of node2vec."""
    n = len(rp) - 1
    nb = [set(col[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
    lists = [col[rp[v]:rp[v + 1]].tolist() for v in range(n)]
    out = []
    # step 1 is unbiased
    state = collections.defaultdict(float)
    for x in lists[start]:
        state[(start, x)] += 1.0 / len(lists[start])
    for t in range(1, T + 1):
        if t > 1:
            nxt = collections.defaultdict(float)
            for (tp, v), pr in state.items():
                w = np.array([wr if x == tp else (wc if x in nb[tp] else wo) for x in lists[v]],
                             dtype=np.float64)
                for x, wx in zip(lists[v], w):
                    nxt[(v, x)] += pr * wx / w.sum()
            state = nxt
        p = np.zeros(n)
        for (_, v), pr in state.items():
            p[v] += pr
        out.append(p)
    return out


@pytest.mark.parametrize("weights", [(1, 2, 4), (4, 1, 2), (3, 3, 3)])
def test_node2vec_t_step_law(weights):
    rp, col = small_graph(seed=7, n=9, m=18)
    start = 0
    T = 4
    paths, _, _ = oracle.walk(rp, col, None, np.full(NW, start, dtype=np.int32), T,
                              bias_kind=oracle.NODE2VEC, node2vec=weights, rng_seed=21)
    exact = node2vec_exact(rp, col, start, T, *weights)
    for t in range(1, T + 1):
        compare(np.bincount(paths[:, t], minlength=len(rp) - 1), exact[t - 1])


def test_node2vec_equal_weights_is_uniform_walk():
    """node2vec with w_return = w_common = w_outward equals the unbiased walk
    (weight-scale invariance), bit for bit."""
    rp, col = inputs.rmat_csr(10, 8192, 5, symmetrize=True)
    starts = inputs.walker_starts(rp, col, 500, 1)
    a, _, _ = oracle.walk(rp, col, None, starts, 20, bias_kind=oracle.NODE2VEC, node2vec=(5, 5, 5))
    b, _, _ = oracle.walk(rp, col, None, starts, 20, bias_kind=oracle.UNIFORM)
    np.testing.assert_array_equal(a, b)


def test_walk_draw_layout():
    """Each step uses counter (walker id, step, vertex, 0): recomputed here with
    the independent Philox and numpy's searchsorted."""
    from tests.helpers import torch_philox
    rp, col = inputs.rmat_csr(9, 4096, 8)
    ew = inputs.dst_outdeg_weights(rp, col) + 1
    starts = inputs.walker_starts(rp, col, 6, 2)
    paths, _, _ = oracle.walk(rp, col, ew, starts, 5, bias_kind=oracle.EDGE_WEIGHT, rng_seed=123,
                              walker_base=1000)
    for w in range(6):
        v = int(starts[w])
        for s in range(5):
            if rp[v + 1] == rp[v]:
                assert paths[w, s + 1] == -1
                break
            S = np.concatenate([[0], np.cumsum(ew[rp[v]:rp[v + 1]].astype(np.uint64))])
            r = torch_philox.draw(123, [1000 + w, s, v, 0], int(S[-1]))
            m = int(np.searchsorted(S[:-1], r, side="right")) - 1
            v = int(col[rp[v] + m])
            assert paths[w, s + 1] == v


def test_walk_threads_and_subsets_agree():
    rp, col = inputs.rmat_csr(11, 20000, 9, symmetrize=True)
    starts = inputs.walker_starts(rp, col, 3000, 3)
    full, _, _ = oracle.walk(rp, col, None, starts, 15, bias_kind=oracle.NODE2VEC, node2vec=(1, 2, 4),
                             rng_seed=4, nthreads=4)
    one, _, _ = oracle.walk(rp, col, None, starts, 15, bias_kind=oracle.NODE2VEC, node2vec=(1, 2, 4),
                            rng_seed=4, nthreads=1)
    np.testing.assert_array_equal(full, one)
    idx = np.arange(5, 3000, 97)
    sub, _, _ = oracle.walk(rp, col, None, starts[idx], 15, bias_kind=oracle.NODE2VEC,
                            node2vec=(1, 2, 4), rng_seed=4, walker_ids=idx.astype(np.uint64))
    np.testing.assert_array_equal(sub, full[idx])


@pytest.mark.parametrize("alpha,beta", [(0.25, 0.0), (0.0, 0.125), (0.25, 0.125)])
def test_restart_jump_t_step_law(alpha, beta):
    """Random walk with restart / with jump: each step moves to the start
    with probability alpha, to a uniform vertex with probability beta, and
    otherwise takes the biased step (or stops at a dead end); the exact t-step
    law is the matrix power of that chain."""
    rp, col = small_graph(seed=4, n=9, m=20, directed=True)    # sinks possible
    n = len(rp) - 1
    ew = np.random.Generator(np.random.PCG64(2)).integers(0, 9, size=len(col)).astype(np.uint32)
    start = int(np.argmax(np.diff(rp)))
    T = 4
    ra, ja = int(alpha * 2 ** 32), int(beta * 2 ** 32)
    paths, steps, _ = oracle.walk(rp, col, ew, np.full(NW, start, dtype=np.int32), T,
                                  bias_kind=oracle.EDGE_WEIGHT, rng_seed=13, restart=ra, jump=ja)
    P = first_order_matrix(rp, col, ew)
    Q = (1 - alpha - beta) * P
    Q[:n, start] += alpha
    Q[:n, :n] += beta / n
    Q[n, :] = 0
    Q[n, n] = 1.0
    p = np.zeros(n + 1)
    p[start] = 1
    for t in range(1, T + 1):
        p = p @ Q
        pos = paths[:, t]
        compare(np.bincount(np.where(pos < 0, n, pos), minlength=n + 1), p)
    valid = (paths[:, 1:] >= 0)
    assert np.all(valid.sum(axis=1) == steps)


@pytest.mark.parametrize("kind", ["edge_weight", "node2vec"])
def test_restart_jump_draw_layout(kind):
    """The move draw uses counter (walker id, step, vertex, 2) over [0, 2^32)
    and the jump target (walker id, step, vertex, 3) over [0, n); after a
    move the previous vertex is forgotten (node2vec's next step is unbiased).
    Recomputed with the independent Philox."""
    from tests.helpers import torch_philox
    rp, col = inputs.rmat_csr(9, 4096, 8, symmetrize=True)
    n = len(rp) - 1
    ew = inputs.dst_outdeg_weights(rp, col) + 1
    starts = inputs.walker_starts(rp, col, 5, 4)
    ra, ja = 1 << 30, 1 << 29
    if kind == "edge_weight":
        paths, _, _ = oracle.walk(rp, col, ew, starts, 12, bias_kind=oracle.EDGE_WEIGHT, rng_seed=77,
                                  walker_base=900, restart=ra, jump=ja)
    else:
        paths, _, _ = oracle.walk(rp, col, None, starts, 12, bias_kind=oracle.NODE2VEC, rng_seed=77,
                                  walker_base=900, restart=ra, jump=ja, node2vec=(1, 2, 4))
    moves = 0
    for w in range(5):
        v, t = int(starts[w]), -1
        for s in range(12):
            x = torch_philox.draw(77, [900 + w, s, v, 2], 2 ** 32)
            if x < ra + ja:
                nxt = int(starts[w]) if x < ra else torch_philox.draw(77, [900 + w, s, v, 3], n)
                assert paths[w, s + 1] == nxt
                v, t = nxt, -1
                moves += 1
                continue
            nb = col[rp[v]:rp[v + 1]]
            if len(nb) == 0:
                assert paths[w, s + 1] == -1
                break
            if kind == "edge_weight":
                b = ew[rp[v]:rp[v + 1]].astype(np.uint64)
            elif t < 0:
                b = np.ones(len(nb), dtype=np.uint64)
            else:
                nt = set(col[rp[t]:rp[t + 1]].tolist())
                b = np.array([1 if x2 == t else (2 if x2 in nt else 4) for x2 in nb.tolist()], dtype=np.uint64)
            S = np.concatenate([[0], np.cumsum(b)])
            r = torch_philox.draw(77, [900 + w, s, v, 0], int(S[-1]))
            m = int(np.searchsorted(S[:-1], r, side="right")) - 1
            t, v = v, int(nb[m])
            assert paths[w, s + 1] == v
    assert moves > 3


def mh_matrix(rp, col):
    """Metropolis-Hastings transition matrix: propose a uniform neighbor u of
    v, move with probability min(1, deg(v)/deg(u)), else stay; state n =
    stopped (no neighbor)."""
    n = len(rp) - 1
    deg = np.diff(rp).astype(np.float64)
    P = np.zeros((n + 1, n + 1))
    for v in range(n):
        if deg[v] == 0:
            P[v, n] = 1.0
            continue
        for u in col[rp[v]:rp[v + 1]]:
            a = min(1.0, deg[v] / deg[u]) if deg[u] > 0 else 1.0
            P[v, u] += a / deg[v]
            P[v, v] += (1 - a) / deg[v]
    P[n, n] = 1.0
    return P


def test_metropolis_hastings_t_step_law():
    """Exact t-step law of the Metropolis-Hastings walk (uniform proposals,
    acceptance min(1, deg(v)/deg(u)), a rejection stays), on a directed
    graph with sinks and on an undirected one."""
    for directed in (True, False):
        rp, col = small_graph(seed=6, n=9, m=19, directed=directed)
        n = len(rp) - 1
        start = int(np.argmin(np.where(np.diff(rp) > 0, np.diff(rp), 99)))
        T = 4
        paths, steps, _ = oracle.walk(rp, col, None, np.full(NW, start, dtype=np.int32), T,
                                      bias_kind=oracle.METROPOLIS, rng_seed=17)
        P = mh_matrix(rp, col)
        p = np.zeros(n + 1)
        p[start] = 1
        for t in range(1, T + 1):
            p = p @ P
            pos = paths[:, t]
            compare(np.bincount(np.where(pos < 0, n, pos), minlength=n + 1), p)
        assert np.all((paths[:, 1:] >= 0).sum(axis=1) == steps)


def test_metropolis_hastings_stationary_uniform():
    """On a connected undirected graph with unequal degrees the walk's visit
    frequencies converge to the uniform distribution over vertices (not to
    deg(v)/2|E| as for the simple walk)."""
    G = nx.connected_watts_strogatz_graph(30, 4, 0.5, seed=8)
    G.add_edges_from([(0, j) for j in range(2, 20)])
    assert nx.is_connected(G)
    edges = list(G.edges()) + [(v, u) for u, v in G.edges()]
    rp, col = inputs.csr_from_edges(30, edges)
    deg = np.diff(rp)
    assert deg.max() > 4 * deg.min()
    paths, _, _ = oracle.walk(rp, col, None, np.zeros(2000, dtype=np.int32), 600, bias_kind=oracle.METROPOLIS,
                              rng_seed=7)
    visits = np.bincount(paths[:, 150:].ravel(), minlength=30).astype(np.float64)
    freq = visits / visits.sum()
    assert 0.5 * np.abs(freq - 1.0 / 30).sum() < 0.03
    assert 0.5 * np.abs(freq - deg / deg.sum()).sum() > 0.1


def test_metropolis_hastings_draw_layout():
    """Proposal with counter (walker id, step, v, 0) over [0, deg v),
    acceptance word with counter (walker id, step, v, 4) over [0, 2^32):
    replayed with the independent Philox."""
    from tests.helpers import torch_philox
    rp, col = inputs.rmat_csr(9, 4096, 12, symmetrize=True)
    starts = inputs.walker_starts(rp, col, 6, 3)
    deg = np.diff(rp)
    paths, _, _ = oracle.walk(rp, col, None, starts, 6, bias_kind=oracle.METROPOLIS, rng_seed=321,
                              walker_base=50)
    stays = 0
    for w in range(6):
        v = int(starts[w])
        for s in range(6):
            m = torch_philox.draw(321, [50 + w, s, v, 0], int(deg[v]))
            u = int(col[rp[v] + m])
            x = torch_philox.draw(321, [50 + w, s, v, 4], 2 ** 32)
            if x * int(deg[u]) >= int(deg[v]) << 32:
                u = v
                stays += 1
            assert paths[w, s + 1] == u
            v = u
    assert stays > 0
