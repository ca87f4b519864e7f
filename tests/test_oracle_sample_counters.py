"""Pin of the counter wiring of the oracle's sampling loop (fig:api(b)).

The selection of one list is pinned elsewhere against its definition; this
file pins what the loop feeds it: every draw of instance i, layer l at
frontier vertex v uses the Philox counter (instance id mod 2^32, l, v,
slot | round << 16), the direct draws round 0xFFFF, and forest fire's trials
(instance id, l, v, 0xFFFE << 16 | j / 4), word j mod 4 (Section II-A,
Section IV-B, Theorem 1). The loop is rewritten here from the definition in
plain Python: distinct seeds as F_0 and visited set, every vertex of F_l in
increasing order selects min(k, P) distinct neighbors (all positive ones when
k >= P), F_{l+1} = picked neighbors not yet visited. Draws come from PyTorch's
Philox4x32-10 header (tests/helpers/torch_philox), not from the oracle, so a
swapped counter word anywhere in the oracle's loop changes its edges and fails
the comparison.
"""
import numpy as np
import pytest

import oracle
from paper_2009_09103_amd import inputs
from tests.helpers import torch_philox

DIRECT = 0xFFFF
BURN = 0xFFFE
MASK32 = 0xFFFFFFFF


class Blocks:
    """Philox blocks of the independent reference, fetched in batches."""

    def __init__(self, rng_seed):
        self.key = [rng_seed & MASK32, rng_seed >> 32]
        self.cache = {}

    def fetch(self, ctrs):
        need = sorted(set(c for c in ctrs if c not in self.cache))
        if need:
            out = torch_philox.blocks([self.key] * len(need), need)
            for c, x in zip(need, out):
                self.cache[c] = [int(w) for w in x]

    def draw(self, ctr, W):
        x = self.cache[ctr]
        return ((x[0] | (x[1] << 32)) * W) >> 64

    def word(self, ctr, q):
        return self.cache[ctr][q]


def biases(rp, col, ew, kind, v):
    b, e = int(rp[v]), int(rp[v + 1])
    if kind == oracle.UNIFORM:
        return [1] * (e - b)
    if kind == oracle.EDGE_WEIGHT:
        return [int(w) for w in ew[b:e]]
    return [int(rp[x + 1] - rp[x]) for x in col[b:e]]


def burn_count(bl, c0, l, v, burn, cap):
    g = 0
    while g < cap:
        if bl.word((c0, l, v, (BURN << 16) | (g // 4)), g % 4) >= burn:
            return g
        g += 1
    return g


def select(bl, b, k, rounds, c0, l, v):
    """min(k, P) distinct positions: rounds in slot order (a slot keeps its
    pick unless it is already held), then direct draws in slot order over the
    prefix rebuilt without the held positions."""
    P = sum(1 for x in b if x > 0)
    if k < 0 or k >= P:
        return [i for i, x in enumerate(b) if x > 0]
    S = np.cumsum(np.asarray(b, dtype=np.uint64))
    W = int(S[-1])
    held, pos, open_ = set(), [None] * k, list(range(k))
    for a in range(rounds):
        nxt = []
        for j in open_:
            m = int(np.searchsorted(S, bl.draw((c0, l, v, j | (a << 16)), W), side="right"))
            if m in held:
                nxt.append(j)
            else:
                held.add(m)
                pos[j] = m
        open_ = nxt
    for j in open_:
        bp = np.asarray(b, dtype=np.uint64).copy()
        bp[sorted(held)] = 0
        Sp = np.cumsum(bp)
        m = int(np.searchsorted(Sp, bl.draw((c0, l, v, j | (DIRECT << 16)), int(Sp[-1])), side="right"))
        held.add(m)
        pos[j] = m
    return pos


def sample_from_definition(rp, col, ew, offs, seeds, fanouts, kinds, ids, rng_seed, rounds, burn):
    ni = len(offs) - 1
    L = fanouts.shape[1]
    bl = Blocks(rng_seed)
    seg = {}
    state = []
    for i in range(ni):
        f0 = sorted(set(int(s) for s in seeds[offs[i]:offs[i + 1]]))
        state.append((f0, set(f0)))
    for l in range(L):
        # every counter this layer can use, fetched in one batch
        ctrs = []
        for i in range(ni):
            c0 = ids[i] & MASK32
            k = int(fanouts[i, l])
            if any(fanouts[i, q] == 0 for q in range(l + 1)):
                continue
            kb = k if k > 0 else (64 if burn else 0)
            for v in state[i][0]:
                if burn:
                    ctrs += [(c0, l, v, (BURN << 16) | q) for q in range((kb + 3) // 4 + 1)]
                for j in range(kb):
                    ctrs += [(c0, l, v, j | (a << 16)) for a in range(rounds)]
                    ctrs.append((c0, l, v, j | (DIRECT << 16)))
        bl.fetch(ctrs)
        for i in range(ni):
            frontier, visited = state[i]
            c0 = ids[i] & MASK32
            if any(fanouts[i, q] == 0 for q in range(l + 1)):
                seg[(l, i)] = ([], [])
                continue
            src, dst = [], []
            for v in frontier:
                k = int(fanouts[i, l])
                if burn:
                    k = burn_count(bl, c0, l, v, burn, 64 if k < 0 else k)
                b = biases(rp, col, ew, int(kinds[i]), v)
                if not b or sum(b) == 0 or k == 0:
                    continue
                for m in select(bl, b, k, rounds, c0, l, v):
                    src.append(v)
                    dst.append(int(col[rp[v] + m]))
            seg[(l, i)] = (src, dst)
            nxt = sorted(set(x for x in dst if x not in visited))
            state[i] = (nxt, visited | set(nxt))
    return seg


@pytest.fixture(scope="module")
def graph():
    rp, col = inputs.rmat_csr(9, 4096, 77)
    ew = inputs.dst_outdeg_weights(rp, col).copy()
    ew[::3] = 0                      # zero weights are never selected
    ew[1::7] = 1000                  # a few heavy ones force collisions
    return rp, col, ew


def run_case(graph, ids, base, kinds, fanouts, seed_counts, rng_seed, rounds, burn, gen_seed, min_edges=100):
    rp, col, ew = graph
    pool = inputs.non_isolated(rp, col)
    g = inputs.rng(gen_seed)
    seeds = [g.choice(pool, size=c, replace=True).astype(np.int32) for c in seed_counts]  # duplicates merge
    offs = np.zeros(len(seeds) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in seeds])
    seeds = np.concatenate(seeds)
    fanouts = np.asarray(fanouts, dtype=np.int32)
    kinds = np.asarray(kinds, dtype=np.int32)
    res = oracle.sample(rp, col, ew, offs, seeds, fanouts, rng_seed=rng_seed, instance_base=base,
                        instance_ids=ids, bias_kinds=kinds, rounds=rounds, burn=burn)
    id_list = [int(x) for x in ids] if ids is not None else [base + i for i in range(len(kinds))]
    want = sample_from_definition(rp, col, ew, offs, seeds, fanouts, kinds, id_list, rng_seed, rounds, burn)
    drawn = 0
    for (l, i), (s, d) in want.items():
        got_s, got_d = res.segment(l, i)
        assert got_s.tolist() == s, "layer %d instance %d sources differ" % (l, i)
        assert got_d.tolist() == d, "layer %d instance %d neighbors differ" % (l, i)
        drawn += len(d)
    assert drawn == res.num_edges and drawn >= min_edges
    return res


@pytest.mark.parametrize("rounds", [8, 2, 0])
def test_sample_counter_wiring(graph, rounds):
    """Explicit instance ids (one above 2^32: counter word 0 is the id mod
    2^32), three bias kinds, per-instance fanout rows with a stop and a
    take-all layer; default rounds, two rounds, and direct draws only."""
    ids = np.array([7, (1 << 32) + 5, 123456, 3], dtype=np.uint64)
    run_case(graph, ids, 0, [0, 1, 2, 2], [[4, 3, 2], [6, 2, 0], [3, -1, 2], [9, 4, 3]],
             [12, 9, 15, 6], rng_seed=(9 << 32) | 11, rounds=rounds, burn=0, gen_seed=rounds + 1)


def test_sample_counter_wiring_instance_base(graph):
    """No explicit ids: instance i has id instance_base + i."""
    run_case(graph, None, (1 << 32) - 2, [2, 0, 1], [[5, 3], [5, 3], [2, 8]], [10, 14, 8], rng_seed=4,
             rounds=8, burn=0, gen_seed=40)


@pytest.mark.parametrize("burn", [int(0.7 * 2 ** 32), int(0.9 * 2 ** 32)])
def test_forest_fire_counter_wiring(graph, burn):
    """Forest fire: each vertex's NeighborSize from its own trials, capped by
    the fanout (64 for -1), then the same selection."""
    ids = np.array([11, 2 ** 40 + 1, 5], dtype=np.uint64)
    run_case(graph, ids, 0, [0, 2, 1], [[4, 3, 3], [-1, 2, 2], [10, 10, 10]], [40, 30, 50], rng_seed=21,
             rounds=8, burn=burn, gen_seed=burn % 97, min_edges=150)
