"""Pins of the oracle's selection arithmetic (CPU only).

Each test checks the oracle against something other than itself: numbers the
paper prints, exact big-integer arithmetic, an independent Philox
implementation, brute-force enumeration, or library routines.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests.helpers import torch_philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")
U64 = (1 << 64) - 1


# --------------------------------------------------------------------- Philox
def test_philox_matches_independent_implementation():
    """Philox4x32-10 (Salmon et al. SC'11) agrees word for word with PyTorch's
    at::philox_engine, called through its header, on random keys/counters and
    on edge counters (zeros, all-ones)."""
    g = np.random.Generator(np.random.PCG64(7))
    keys = g.integers(0, 1 << 32, size=(400, 2), dtype=np.uint64)
    ctrs = g.integers(0, 1 << 32, size=(400, 4), dtype=np.uint64)
    keys[0] = 0; ctrs[0] = 0
    keys[1] = 0xFFFFFFFF; ctrs[1] = 0xFFFFFFFF
    keys[2] = [1, 0]; ctrs[2] = [0, 0, 0, 1]
    ref = torch_philox.blocks(keys, ctrs)
    got = np.array([oracle.philox(k, c) for k, c in zip(keys, ctrs)], dtype=np.uint32)
    np.testing.assert_array_equal(got, ref)


def test_philox_bit_balance_and_byte_chisquare():
    """Output words of consecutive counters: every one of the 128 bits is set
    about half the time, and byte values are uniform (chi-square)."""
    from scipy import stats
    n = 20000
    words = np.array([oracle.philox([0x1234, 0x5678], [i, 0, 7, 0]) for i in range(n)],
                     dtype=np.uint32)
    bits = np.unpackbits(words.view(np.uint8).reshape(n, 16), axis=1)
    frac = bits.mean(axis=0)
    # binomial(n, 1/2): sd = 0.5/sqrt(n) ~ 0.0035; 5 sd bound over 128 bits
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
    counts = np.bincount(words.view(np.uint8).ravel(), minlength=256)
    p = stats.chisquare(counts).pvalue
    assert p > 1e-4


def test_draw_layout_matches_reference_block():
    """draw(seed, c0..c3, W) = floor((x0 + 2^32 x1) * W / 2^64) with the key
    (seed lo, seed hi), computed here from the independent block function and
    Python integers."""
    g = np.random.Generator(np.random.PCG64(11))
    for t in range(40):
        seed = int(g.integers(0, 1 << 63)) * 2 + int(g.integers(0, 2))
        ctr = [int(x) for x in g.integers(0, 1 << 32, size=4)]
        W = int(g.integers(1, 1 << 62)) if t % 2 else int(g.integers(1, 1000))
        assert oracle.draw(seed, *ctr, W) == torch_philox.draw(seed, ctr, W)


# ------------------------------------------------------------ range reduction
def test_range_reduction_exact_128bit():
    g = np.random.Generator(np.random.PCG64(3))
    cases = [(0, 1), (U64, 1), (U64, (1 << 63) - 1), (U64, 15), (1 << 63, 9), (12345, 1 << 40)]
    for _ in range(2000):
        cases.append((int(g.integers(0, 1 << 63)) * 2 + 1, int(g.integers(1, 1 << 63))))
    for u, W in cases:
        assert oracle.range_reduce(u, W) == (u * W) >> 64


def test_range_reduction_powers_of_two_take_top_bits():
    g = np.random.Generator(np.random.PCG64(4))
    for _ in range(200):
        u = int(g.integers(0, 1 << 63)) * 2 + int(g.integers(0, 2))
        j = int(g.integers(0, 63))
        assert oracle.range_reduce(u, 1 << j) == u >> (64 - j)


def test_range_reduction_preimages_balanced_small_analogue():
    """floor(u*W/2^b) gives each value floor or ceil of 2^b/W preimages: the
    same map on b = 16 bits, enumerated for every W <= 300 (the property the
    64-bit map inherits; the oracle's 64-bit map is checked exactly above)."""
    b = 16
    u = np.arange(1 << b, dtype=np.int64)
    for W in range(1, 301):
        c = np.bincount((u * W) >> b, minlength=W)
        lo, hi = (1 << b) // W, -(-(1 << b) // W)
        assert c.min() >= lo and c.max() <= hi and c.sum() == 1 << b


# ------------------------------------------------------- inverse transform
def test_paper_worked_example():
    """fig:example(b): b = (3,6,2,2,2) gives S = {0,3,9,11,13,15},
    F = S/15, and r = 0.5 selects v7 (the second candidate)."""
    ex = json.load(open(GOLDEN))
    its = ex["its"]
    S = oracle.prefix(its["biases"])
    assert S.tolist() == its["S"]
    np.testing.assert_allclose(S / S[-1], its["F"], atol=0.005)
    r = int(its["r"] * int(S[-1]))                  # floor(0.5 * 15) = 7
    assert its["names"][oracle.its(S, r)] == its["selected"]


def test_paper_updated_sampling_example_via_skip_map():
    """fig:brs(b)/(c): with v7 pre-selected the updated prefix is
    {0,3,5,7,9}; r = 0.58 selects v10. The skip map reaches v10 on the
    original prefix without rebuilding it (Theorem 2's inverse)."""
    ex = json.load(open(GOLDEN))
    names, b = ex["its"]["names"], ex["its"]["biases"]
    up = ex["updated_sampling"]
    pre = names.index(up["preselected"])
    rest = [x for i, x in enumerate(b) if i != pre]
    S_up = oracle.prefix(rest)
    assert S_up.tolist() == up["S_updated"]
    np.testing.assert_allclose(S_up / S_up[-1], up["F_updated"], atol=0.005)
    r = int(up["r"] * int(S_up[-1]))                # floor(0.58 * 9) = 5
    S = oracle.prefix(b)
    pos = oracle.its(S, oracle.skip_map(S, b, [pre], r))
    assert names[pos] == up["selected"] == ex["bipartite_region_search"]["selected"]
    # the fractional bipartite-region numbers land in the same region
    brs = ex["bipartite_region_search"]
    assert names[oracle.its(S, int(brs["r_shifted"] * 15))] == brs["selected"]


def _random_weights(g, d, zero_frac=0.3, hi=20):
    b = g.integers(0, hi, size=d).astype(np.uint32)
    b[g.random(d) < zero_frac] = 0
    return b


def test_its_preimage_counts_equal_biases():
    """Exhaustively over r in [0, W): #{r : its(r) = i} = b_i, including zero
    biases (never selected) and leading/trailing zeros."""
    g = np.random.Generator(np.random.PCG64(5))
    lists = [np.array([3, 6, 2, 2, 2]), np.array([0, 0, 5]), np.array([5, 0, 0]),
             np.array([0, 1, 0, 1, 0]), np.array([7])]
    lists += [_random_weights(g, int(g.integers(1, 12))) for _ in range(60)]
    for b in lists:
        b = b.astype(np.uint32)
        if b.sum() == 0:
            continue
        S = oracle.prefix(b)
        W = int(S[-1])
        hits = np.zeros(len(b), dtype=np.int64)
        for r in range(W):
            hits[oracle.its(S, r)] += 1
        np.testing.assert_array_equal(hits, b.astype(np.int64))


def test_its_matches_library_search():
    """its(S, r) equals numpy.searchsorted(S[:d], r, 'right') - 1 on large lists."""
    g = np.random.Generator(np.random.PCG64(6))
    for _ in range(30):
        b = _random_weights(g, int(g.integers(1, 3000)), hi=1 << 31)
        if b.sum() == 0:
            continue
        S = oracle.prefix(b)
        for r in g.integers(0, int(S[-1]), size=20, dtype=np.uint64):
            assert oracle.its(S, int(r)) == int(np.searchsorted(S[:-1], r, side="right")) - 1


def test_prefix_is_exact_for_large_weights():
    b = np.full(1000, 0xFFFFFFFF, dtype=np.uint32)
    S = oracle.prefix(b)
    assert int(S[-1]) == 1000 * 0xFFFFFFFF
    assert [int(x) for x in S[:4]] == [0, 0xFFFFFFFF, 2 * 0xFFFFFFFF, 3 * 0xFFFFFFFF]


# ----------------------------------------------------------------- skip map
def test_skip_map_equals_search_on_rebuilt_list():
    """For every r in [0, W - removed): its(skip_map(r)) on the original prefix
    selects the same candidate as inverse transform search over the list
    rebuilt without the pre-selected candidates (updated sampling, fig:brs(b))."""
    g = np.random.Generator(np.random.PCG64(8))
    for _ in range(120):
        d = int(g.integers(2, 12))
        b = _random_weights(g, d, zero_frac=0.2)
        pos = np.nonzero(b)[0]
        if len(pos) < 2:
            continue
        na = int(g.integers(1, len(pos)))
        acc = np.sort(g.choice(pos, size=na, replace=False))
        keep = np.array([i for i in range(d) if i not in set(acc.tolist())])
        S = oracle.prefix(b)
        S_rest = oracle.prefix(b[keep])
        for r in range(int(S_rest[-1])):
            want = keep[oracle.its(S_rest, r)]
            got = oracle.its(S, oracle.skip_map(S, b, acc, r))
            assert got == want


def test_theorem2_integer_form():
    """Eq. eq:brs in integers: with candidate s removed, the updated prefix is
    S'_k = S_k for k <= s and S_k - b_s for k > s."""
    g = np.random.Generator(np.random.PCG64(9))
    for _ in range(50):
        b = _random_weights(g, int(g.integers(2, 15)), zero_frac=0.1)
        s = int(g.integers(0, len(b)))
        S = oracle.prefix(b).astype(np.int64)
        Sp = oracle.prefix(np.delete(b, s)).astype(np.int64)
        for k in range(len(Sp)):
            want = S[k] if k <= s else S[k + 1] - b[s]
            assert Sp[k] == want


# ------------------------------------------------------------------- select
@pytest.mark.parametrize("rounds", [0, 1, 8])
def test_select_invariants(rounds):
    g = np.random.Generator(np.random.PCG64(10 + rounds))
    for t in range(300):
        d = int(g.integers(0, 40))
        b = _random_weights(g, d, zero_frac=0.25, hi=1000)
        if t % 7 == 0 and d:
            b[int(g.integers(0, d))] = 1 << 30           # one dominant bias
        P = int((b > 0).sum())
        k = int(g.integers(1, 30))
        pos = oracle.select(b, k, 99, t, 1, 2, rounds=rounds)
        if b.sum() == 0:
            assert len(pos) == 0
            continue
        assert len(pos) == min(k, P)
        assert len(set(pos.tolist())) == len(pos)
        assert np.all(b[pos] > 0)
        if k >= P:
            np.testing.assert_array_equal(pos, np.nonzero(b)[0])


def test_select_k1_is_single_its_draw():
    """k = 1 (and no collision possible): the slot is its(S, r) of the round-0
    draw with counter (c0, c1, c2, 0), r from the independent Philox."""
    g = np.random.Generator(np.random.PCG64(12))
    for t in range(30):
        b = _random_weights(g, int(g.integers(2, 50)), zero_frac=0.1, hi=100)
        if (b > 0).sum() < 2:
            continue
        S = oracle.prefix(b)
        r = torch_philox.draw(5, [t, 3, 17, 0], int(S[-1]))
        want = int(np.searchsorted(S[:-1], r, side="right")) - 1
        assert oracle.select(b, 1, 5, t, 3, 17).tolist() == [want]


def test_select_weight_scale_invariance():
    """Multiplying every bias by an integer c leaves every selection unchanged
    (c*S_i <= floor(c*y) iff S_i <= floor(y)), so UNIFORM equals any constant
    weight."""
    g = np.random.Generator(np.random.PCG64(13))
    for t in range(150):
        d = int(g.integers(1, 40))
        b = _random_weights(g, d, zero_frac=0.2, hi=50)
        c = int(g.integers(2, 1000))
        k = int(g.integers(1, 12))
        a1 = oracle.select(b, k, 3, t, 0, 9)
        a2 = oracle.select((b.astype(np.uint64) * c).astype(np.uint32), k, 3, t, 0, 9)
        np.testing.assert_array_equal(a1, a2)
        ones = np.ones(d, dtype=np.uint32)
        np.testing.assert_array_equal(oracle.select(ones, k, 3, t, 0, 9),
                                      oracle.select(ones * 7, k, 3, t, 0, 9))


def test_skewed_list_reaches_direct_draw():
    b = np.array([1 << 30] + [1] * 9, dtype=np.uint32)
    total_fb = 0
    for t in range(50):
        pos, fb = oracle.select(b, 5, 1, t, 0, 0, with_fallback=True)
        assert len(set(pos.tolist())) == 5 and 0 in pos
        total_fb += fb
    assert total_fb > 0


def _select_from_definition(b, k, seed, c0, c1, c2, rounds=8):
    """Selection written from its definition, with the independent Philox:
    rounds where slots are taken in slot order and a slot keeps its candidate
    unless it is already held, then direct draws in slot order, each an
    inverse transform search of the prefix rebuilt with held biases removed
    (the updated-sampling law that the skip map inverts)."""
    b = np.asarray(b, dtype=np.uint64)
    P = int((b > 0).sum())
    if k >= P:
        return [i for i in range(len(b)) if b[i] > 0]
    S = np.cumsum(b)
    W = int(S[-1])
    held, pos, open_ = set(), [None] * k, list(range(k))
    for a in range(rounds):
        nxt = []
        for j in open_:
            m = int(np.searchsorted(S, torch_philox.draw(seed, [c0, c1, c2, j | (a << 16)], W), side="right"))
            if m in held:
                nxt.append(j)
            else:
                held.add(m)
                pos[j] = m
        open_ = nxt
    for j in open_:
        bp = b.copy()
        bp[list(held)] = 0
        Sp = np.cumsum(bp)
        m = int(np.searchsorted(Sp, torch_philox.draw(seed, [c0, c1, c2, j | (0xFFFF << 16)], int(Sp[-1])),
                                side="right"))
        held.add(m)
        pos[j] = m
    return pos


def test_select_equals_definition_with_rebuilt_prefix():
    """The whole selection, including many direct draws (skewed lists with k
    close to P), equals the definition above bit for bit."""
    g = np.random.Generator(np.random.PCG64(14))
    fallbacks = 0
    for t in range(160):
        d = int(g.integers(2, 60))
        b = _random_weights(g, d, zero_frac=0.2, hi=50)
        if t % 2 == 0:
            b[g.integers(0, d, size=3)] = int(g.integers(1000, 1 << 20))
        P = int((b > 0).sum())
        if P == 0:
            continue
        k = int(g.integers(1, min(P + 2, 64) + 1))
        pos, fb = oracle.select(b, k, 21, t, 4, 8, with_fallback=True)
        assert pos.tolist() == _select_from_definition(b, k, 21, t, 4, 8)
        fallbacks += fb
    assert fallbacks > 80
