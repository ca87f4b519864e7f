"""Pins of the oracle's multi-dimensional random walk (frontier sampling,
Section II-A; VertexBias select of fig:api(b)) on CPU.

The exact law of the first and second sampled edge is computed here from the
definition (pool vertex chosen with probability proportional to its degree,
then a uniform neighbor, and the chosen slot replaced by that neighbor) and
compared by chi-square with many independent instances; the counter layout is
recomputed with the independent Philox; invariants are checked on R-MAT.
"""
import collections
from fractions import Fraction

import numpy as np
from scipy import stats

import oracle
from paper_2009_09103_amd import inputs

NI = 40_000


def toy():
    # 0: {1, 2, 3}, 1: {0}, 2: {0, 3}, 3: {4}, 4: {} (a sink), 5: {0, 1, 2, 3, 4}
    edges = [(0, 1), (0, 2), (0, 3), (1, 0), (2, 0), (2, 3), (3, 4), (5, 0), (5, 1), (5, 2), (5, 3), (5, 4)]
    return inputs.csr_from_edges(6, edges)


def step_law(rp, pool):
    """{(v, u): probability} of one step from the pool, from the definition
    (exact fractions); empty if every pool vertex is a sink."""
    deg = {v: int(rp[v + 1] - rp[v]) for v in set(pool)}
    W = sum(deg[v] for v in pool)
    out = collections.defaultdict(Fraction)
    if W == 0:
        return out
    for v in pool:
        for u in range(int(rp[v]), int(rp[v + 1])):
            out[(v, u)] += Fraction(deg[v], W) * Fraction(1, deg[v])
    return out


def compare(counts, probs):
    keys = sorted(set(counts) | set(probs))
    c = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    p = np.array([float(probs.get(k, 0)) for k in keys])
    assert np.all(c[p == 0] == 0), "an impossible edge was sampled"
    nz = p > 0
    assert stats.chisquare(c[nz], p[nz] / p[nz].sum() * c.sum()).pvalue > 1e-4


def run(rp, col, pool, budget, base=0, ni=NI):
    po = np.arange(ni + 1, dtype=np.int64) * len(pool)
    pl = np.tile(np.asarray(pool, dtype=np.int32), ni)
    return oracle.mdrw(rp, col, po, pl, budget, rng_seed=7, instance_base=base)


def test_first_edge_law():
    """P(first edge = (v, u)) = (copies of v in the pool) / W for each
    neighbor u of v, W = total pool degree; sinks are never chosen."""
    rp, col = toy()
    pool = [0, 2, 2, 4, 5]
    src, dst, _ = run(rp, col, pool, 1)
    counts = collections.Counter(zip(src[:, 0].tolist(), dst[:, 0].tolist()))
    law = {(v, int(col[e])): p for (v, e), p in step_law(rp, pool).items()}
    compare(counts, law)


def test_second_edge_law():
    """The second edge follows the law of the pool after the first update
    (chosen slot replaced by the sampled neighbor), mixed over the first step."""
    rp, col = toy()
    pool = [0, 2, 3]
    src, dst, _ = run(rp, col, pool, 2)
    law = collections.defaultdict(Fraction)
    deg = lambda v: int(rp[v + 1] - rp[v])
    W = sum(deg(v) for v in pool)
    for j, v in enumerate(pool):
        for e in range(int(rp[v]), int(rp[v + 1])):
            pr = Fraction(deg(v), W) * Fraction(1, deg(v))
            newpool = pool[:j] + [int(col[e])] + pool[j + 1:]
            for (v2, e2), q in step_law(rp, newpool).items():
                law[(v2, int(col[e2]))] += pr * q
    ok = src[:, 1] >= 0
    counts = collections.Counter(zip(src[ok, 1].tolist(), dst[ok, 1].tolist()))
    stopped = Fraction(1) - sum(law.values())
    assert abs((~ok).mean() - float(stopped)) < 0.01
    compare(counts, law)


def test_draw_layout():
    """Step s draws the pool slot with counter (instance id, s, 0xFFFFFFFF, 0)
    over the degree prefix and the neighbor with (instance id, s, v, 1):
    recomputed here with the independent Philox and numpy."""
    from tests.helpers import torch_philox
    rp, col = inputs.rmat_csr(9, 4096, 8)
    deg = np.diff(rp)
    g = np.random.Generator(np.random.PCG64(3))
    pools = [g.integers(0, len(rp) - 1, size=k).astype(np.int32) for k in (1, 5, 17)]
    po = np.concatenate([[0], np.cumsum([len(p) for p in pools])])
    src, dst, steps = oracle.mdrw(rp, col, po, np.concatenate(pools), 6, rng_seed=99, instance_base=500)
    for i, pool in enumerate(pools):
        fp = pool.astype(np.int64).copy()
        for s in range(6):
            b = deg[fp].astype(np.uint64)
            S = np.concatenate([[0], np.cumsum(b)])
            if S[-1] == 0:
                assert src[i, s] == -1 and steps[i] == s
                break
            r = torch_philox.draw(99, [500 + i, s, 0xFFFFFFFF, 0], int(S[-1]))
            j = int(np.searchsorted(S[:-1], r, side="right")) - 1
            v = int(fp[j])
            m = torch_philox.draw(99, [500 + i, s, v, 1], int(deg[v]))
            u = int(col[rp[v] + m])
            assert (src[i, s], dst[i, s]) == (v, u)
            fp[j] = u


def test_invariants_rmat():
    """Every sampled edge is a graph edge whose source is in the current pool
    multiset; the pool changes by exactly that source leaving and the target
    entering; a one-vertex pool is a simple random walk; an ended instance
    writes -1."""
    rp, col = inputs.rmat_csr(12, 40000, 4)
    n = len(rp) - 1
    edges = set(zip(np.repeat(np.arange(n), np.diff(rp)).tolist(), col.tolist()))
    g = np.random.Generator(np.random.PCG64(5))
    pools = [g.integers(0, n, size=k).astype(np.int32) for k in (1, 2, 64, 300)]
    po = np.concatenate([[0], np.cumsum([len(p) for p in pools])])
    src, dst, steps = oracle.mdrw(rp, col, po, np.concatenate(pools), 400, rng_seed=3)
    for i, pool in enumerate(pools):
        ms = collections.Counter(pool.tolist())
        for s in range(int(steps[i])):
            v, u = int(src[i, s]), int(dst[i, s])
            assert ms[v] > 0 and (v, u) in edges
            ms[v] -= 1
            ms[u] += 1
        assert np.all(src[i, steps[i]:] == -1) and np.all(dst[i, steps[i]:] == -1)
    walk = steps[0]
    assert np.all(src[0, 1:walk] == dst[0, :walk - 1])


def test_dead_pool_and_empty():
    rp, col = toy()
    src, dst, steps = oracle.mdrw(rp, col, np.array([0, 2, 2]), np.array([4, 4], dtype=np.int32), 3)
    assert steps.tolist() == [0, 0] and np.all(src == -1) and np.all(dst == -1)
    src, dst, steps = oracle.mdrw(rp, col, np.array([0, 1]), np.array([1], dtype=np.int32), 0)
    assert src.shape == (1, 0) and steps.tolist() == [0]
