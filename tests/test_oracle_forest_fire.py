"""Pins of the oracle's forest fire sampling (Section II-A: neighbor sampling
whose NeighborSize per vertex comes from a burning probability) on CPU.

The burn count is checked against the capped geometric law by chi-square,
its counter layout is replayed with the independent Philox, and the two
ends of the burning probability reduce to plain neighbor sampling and to no
sampling at all."""
import numpy as np
from scipy import stats

import oracle
from paper_2009_09103_amd import inputs

P70 = int(0.7 * 2 ** 32)


def star_graph(hubs, degree):
    """hubs vertices, each with `degree` out-neighbors among the leaves."""
    n = hubs + degree
    edges = [(h, hubs + j) for h in range(hubs) for j in range(degree)]
    return inputs.csr_from_edges(n, edges)


def test_burn_count_law():
    """P(G = j) = (1 - p) p^j for j < cap and P(G = cap) = p^cap: edges per
    instance when every hub has more neighbors than the cap, unbiased."""
    cap, ni = 12, 30_000
    rp, col = star_graph(1, 40)
    offs = np.arange(ni + 1, dtype=np.int64)
    seeds = np.zeros(ni, dtype=np.int32)
    res = oracle.sample(rp, col, None, offs, seeds, [cap], rng_seed=5, burn=P70)
    counts = np.diff(res.offsets)
    p = P70 / 2 ** 32
    law = np.array([(1 - p) * p ** j for j in range(cap)] + [p ** cap])
    obs = np.bincount(counts, minlength=cap + 1)
    assert obs.sum() == ni and len(obs) == cap + 1
    assert stats.chisquare(obs, law * ni).pvalue > 1e-4
    assert abs(counts.mean() - sum(j * law[j] for j in range(cap + 1))) < 0.05


def test_burn_counter_layout():
    """Trial j uses word j mod 4 of the block with counter (instance id,
    layer, vertex, 0xFFFE << 16 | j / 4): replayed with the independent
    Philox for many (vertex, layer) pairs and burning thresholds."""
    from tests.helpers import torch_philox
    g = np.random.Generator(np.random.PCG64(4))
    cases, keys, ctrs = [], [], []
    for _ in range(300):
        c0, c1, c2 = (int(x) for x in g.integers(0, 2 ** 32, size=3))
        # thresholds spread over the range, and near 1 so that long runs occur
        burn = int(g.integers(0, 2 ** 32)) if g.random() < 0.5 else 2 ** 32 - int(g.integers(1, 2 ** 29))
        cap = int(g.integers(1, 30))
        seed = int(g.integers(0, 2 ** 63))
        cases.append((seed, c0, c1, c2, burn, cap, len(ctrs)))
        for blk in range((cap + 3) // 4):
            keys.append([seed & 0xFFFFFFFF, seed >> 32])
            ctrs.append([c0, c1, c2, (0xFFFE << 16) | blk])
    words = torch_philox.blocks(keys, ctrs)
    longest = 0
    for seed, c0, c1, c2, burn, cap, first in cases:
        want = 0
        while want < cap and int(words[first + want // 4][want % 4]) < burn:
            want += 1
        longest = max(longest, want)
        assert oracle.burn_count(seed, c0, c1, c2, burn, cap) == want
    assert longest >= 8


def test_burning_ends():
    """burn = 2^32 - 1 burns cap neighbors of every vertex (here: the same
    edges as plain neighbor sampling with that fanout); burn = 1 almost never
    burns (a trial succeeds only on a zero word)."""
    rp, col = inputs.rmat_csr(11, 20000, 6)
    offs, seeds = inputs.single_instance_seeds(rp, col, 300, 8)
    for bias in (oracle.UNIFORM, oracle.NEIGHBOR_DEGREE):
        full = oracle.sample(rp, col, None, offs, seeds, [6, 3], bias_kind=bias, rng_seed=3, burn=2 ** 32 - 1)
        plain = oracle.sample(rp, col, None, offs, seeds, [6, 3], bias_kind=bias, rng_seed=3)
        np.testing.assert_array_equal(full.offsets, plain.offsets)
        np.testing.assert_array_equal(full.dst, plain.dst)
    none = oracle.sample(rp, col, None, offs, seeds, [6, 3], rng_seed=3, burn=1)
    assert none.num_edges == 0
    # fanout -1 with burning: capped at 64
    rpS, colS = star_graph(1, 100)
    offs1 = np.arange(2001, dtype=np.int64)
    res = oracle.sample(rpS, colS, None, offs1, np.zeros(2000, dtype=np.int32), [-1], rng_seed=9,
                        burn=2 ** 32 - 1)
    assert np.all(np.diff(res.offsets) == 64)
