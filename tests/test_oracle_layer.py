"""Pins of the oracle's layer sampling (Section II-A: a constant number of
neighbors selected for the whole frontier in each round) on CPU.

The law of the first and second layer is computed from the definition (one
pick over the concatenated neighbor lists of the frontier, weight = EdgeBias
of the position) and compared by chi-square; the counter layout is replayed
with the independent Philox; invariants are checked on R-MAT."""
import collections
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2009_09103_amd import inputs

NI = 30_000


def toy():
    # 0: {1, 2, 3}, 1: {0, 4}, 2: {0, 3}, 3: {4}, 4: {} (a sink), 5: {0, 1, 2, 3, 4}
    edges = [(0, 1), (0, 2), (0, 3), (1, 0), (1, 4), (2, 0), (2, 3), (3, 4), (5, 0), (5, 1), (5, 2), (5, 3),
             (5, 4)]
    return inputs.csr_from_edges(6, edges)


def pick_law(rp, col, frontier, bias):
    """{(v, x): probability} of one pick from the concatenated lists."""
    w = {}
    for v in frontier:
        for e in range(int(rp[v]), int(rp[v + 1])):
            x = int(col[e])
            w[(v, x)] = bias(v, x)
    W = sum(w.values())
    return {k: Fraction(b, W) for k, b in w.items() if b > 0} if W else {}


def chi2(counts, law, n):
    keys = sorted(set(counts) | set(law))
    c = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    p = np.array([float(law.get(k, 0)) for k in keys])
    assert np.all(c[p == 0] == 0), "an impossible edge was picked"
    nz = p > 0
    if nz.sum() > 1:
        assert stats.chisquare(c[nz], p[nz] / p[nz].sum() * n).pvalue > 1e-4


def run(rp, col, seeds, fanouts, bias_kind=oracle.UNIFORM, ni=NI, seed=5):
    offs = np.arange(ni + 1, dtype=np.int64) * len(seeds)
    return oracle.layer_sample(rp, col, None, offs, np.tile(np.asarray(seeds, dtype=np.int32), ni), fanouts,
                               bias_kind=bias_kind, rng_seed=seed)


@pytest.mark.parametrize("kind", [oracle.UNIFORM, oracle.NEIGHBOR_DEGREE])
def test_first_and_second_layer_law(kind):
    rp, col = toy()
    deg = np.diff(rp)
    bias = (lambda v, x: 1) if kind == oracle.UNIFORM else (lambda v, x: int(deg[x]))
    src, dst, counts = run(rp, col, [0, 2], [1, 1], kind)
    law1 = pick_law(rp, col, [0, 2], bias)
    chi2(collections.Counter(zip(src[:, 0, 0].tolist(), dst[:, 0, 0].tolist())), law1, NI)
    # second layer: the frontier is the first pick's neighbor unless visited
    law2 = collections.defaultdict(Fraction)
    stop = Fraction(0)
    for (v, x), p in law1.items():
        if x in (0, 2):
            stop += p
            continue
        for key, q in pick_law(rp, col, [x], bias).items():
            law2[key] += p * q
        if not pick_law(rp, col, [x], bias):
            stop += p
    ok = counts[:, 1] == 1
    assert abs((~ok).mean() - float(stop)) < 0.01
    chi2(collections.Counter(zip(src[ok, 1, 0].tolist(), dst[ok, 1, 0].tolist())), law2, int(ok.sum()))


def test_draw_layout():
    """A single slot draws r over the pool prefix with counter (instance id,
    layer, 0xFFFFFFFF, 0): replayed with the independent Philox."""
    from tests.helpers import torch_philox
    rp, col = inputs.rmat_csr(10, 9000, 4)
    ew = inputs.dst_outdeg_weights(rp, col) + 1
    g = np.random.Generator(np.random.PCG64(2))
    pool = inputs.non_isolated(rp, col)
    for i in range(5):
        seeds = np.sort(g.choice(pool, size=int(g.integers(1, 20)), replace=False)).astype(np.int32)
        src, dst, counts = oracle.layer_sample(rp, col, ew, [0, len(seeds)], seeds, [1, 1, 1],
                                               bias_kind=oracle.EDGE_WEIGHT, rng_seed=77, instance_base=300 + i)
        front, vis = list(seeds), set(seeds.tolist())
        for l in range(3):
            own = [v for v in front for _ in range(int(rp[v + 1] - rp[v]))]
            nbr = [int(col[e]) for v in front for e in range(int(rp[v]), int(rp[v + 1]))]
            w = [int(ew[e]) for v in front for e in range(int(rp[v]), int(rp[v + 1]))]
            if not w:
                assert counts[0, l] == 0
                break
            S = np.concatenate([[0], np.cumsum(np.asarray(w, dtype=np.uint64))])
            r = torch_philox.draw(77, [300 + i, l, 0xFFFFFFFF, 0], int(S[-1]))
            m = int(np.searchsorted(S[:-1], r, side="right")) - 1
            assert (src[0, l, 0], dst[0, l, 0]) == (own[m], nbr[m])
            front = [] if nbr[m] in vis else [nbr[m]]
            vis.add(nbr[m])


def test_invariants_rmat():
    """Picks are distinct pool positions (edges, as lists hold no repeats) of
    frontier vertices; counts = min(k, P); each next frontier is the distinct
    unvisited picks, so it holds at most k vertices; a fanout above the pool
    takes every positive edge of the frontier in pool order."""
    rp, col = inputs.rmat_csr(12, 40000, 7)
    deg = np.diff(rp)
    offs0, seeds0 = inputs.batched_instances(rp, col, 12, 3)[:2]
    sets = [np.unique(seeds0[a:b]) for a, b in zip(offs0[:-1], offs0[1:])]
    seeds = np.concatenate(sets).astype(np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    fo = [20, 64, 7]
    src, dst, counts = oracle.layer_sample(rp, col, None, offs, seeds, fo, bias_kind=oracle.NEIGHBOR_DEGREE,
                                           rng_seed=4)
    edges = set(zip(np.repeat(np.arange(len(deg)), deg).tolist(), col.tolist()))
    for i in range(12):
        front = seeds[offs[i]:offs[i + 1]].tolist()
        vis = set(front)
        for l, k in enumerate(fo):
            c = counts[i, l]
            P = sum(int(np.sum(deg[col[rp[v]:rp[v + 1]]] > 0)) for v in front)
            assert c == min(k, P)
            pairs = list(zip(src[i, l, :c].tolist(), dst[i, l, :c].tolist()))
            assert len(set(pairs)) == c and all(p in edges and p[0] in front for p in pairs)
            assert np.all(src[i, l, c:] == -1)
            if k >= P:
                want = [(v, int(x)) for v in front for x in col[rp[v]:rp[v + 1]] if deg[x] > 0]
                assert pairs == want
            nxt = sorted({x for _, x in pairs} - vis)
            vis |= set(nxt)
            front = nxt


def test_bad_input():
    rp, col = toy()
    with pytest.raises(ValueError):
        oracle.layer_sample(rp, col, None, [0, 2], np.array([2, 0], dtype=np.int32), [3])   # unsorted
    with pytest.raises(ValueError):
        oracle.layer_sample(rp, col, None, [0, 1], np.array([0], dtype=np.int32), [65])     # fanout > 64
