"""GPU parity of neighbor sampling: the HIP path through the C-ABI against the
CPU oracle, element by element (bit-exact: all integer work)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2009_09103_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csaw():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_09103_amd import csaw as c
    return c


def assert_same(res, ref):
    offs = res.offsets.cpu().numpy()
    np.testing.assert_array_equal(offs, ref.offsets)
    np.testing.assert_array_equal(res.src.cpu().numpy(), ref.src)
    np.testing.assert_array_equal(res.dst.cpu().numpy(), ref.dst)


def run_both(csaw, g, rp, col, ew, offs, seeds, fanouts, bias, rng_seed, instance_base=0):
    say("sample n=%d m=%d ni=%d seeds=%d fanouts=%s bias=%s seed=%d" % (
        len(rp) - 1, len(col), len(offs) - 1, len(seeds), np.asarray(fanouts).tolist()[:4], bias, rng_seed))
    res = g.sample(offs, seeds, fanouts, bias, rng_seed=rng_seed, instance_base=instance_base)
    if isinstance(bias, (list, np.ndarray)):
        ref = oracle.sample(rp, col, ew, offs, seeds, fanouts, bias_kinds=np.asarray(bias, dtype=np.int32),
                            rng_seed=rng_seed, instance_base=instance_base)
    else:
        ref = oracle.sample(rp, col, ew, offs, seeds, fanouts, bias_kind=bias, rng_seed=rng_seed,
                            instance_base=instance_base)
    assert_same(res, ref)
    return res, ref


def test_tiny_uniform(csaw):
    """R-MAT 12, 256 seeds, fanouts [10, 5], unbiased, Philox seed 1."""
    rp, col = inputs.graph_for(inputs.TINY)
    offs, seeds = inputs.single_instance_seeds(rp, col, 256, inputs.TINY["seed_rng"])
    g = csaw.Graph(rp, col)
    res, ref = run_both(csaw, g, rp, col, None, offs, seeds, [10, 5], csaw.UNIFORM, 1)
    assert res.num_edges > 1000


@pytest.mark.parametrize("rng_seed", [1, 2])
def test_degree_biased_rmat16(csaw, rng_seed):
    """Degree bias on R-MAT 16: hubs above the LDS window (coarse search),
    skewed weights (direct draws)."""
    rp, col = inputs.rmat_csr(16, 16 << 16, 16)
    assert np.diff(rp).max() > 1024
    offs, seeds = inputs.single_instance_seeds(rp, col, 2048, 33)
    g = csaw.Graph(rp, col)
    res, ref = run_both(csaw, g, rp, col, None, offs, seeds, [25, 10, 5], csaw.NEIGHBOR_DEGREE, rng_seed)
    assert ref.fallbacks > 0


def test_edge_weight_with_zero_weights(csaw):
    rp, col = inputs.rmat_csr(14, 16 << 14, 14)
    g0 = inputs.rng(1)
    ew = g0.integers(0, 50, size=len(col)).astype(np.uint32)
    ew[g0.random(len(col)) < 0.3] = 0
    offs, seeds = inputs.single_instance_seeds(rp, col, 1500, 5)
    g = csaw.Graph(rp, col, ew)
    run_both(csaw, g, rp, col, ew, offs, seeds, [10, 5, 3], csaw.EDGE_WEIGHT, 7)
    run_both(csaw, g, rp, col, ew, offs, seeds, [-1, 3], csaw.EDGE_WEIGHT, 8)   # take all positive


def test_batched_instances_mixed_bias(csaw):
    """Many instances with their own fanout rows and bias kinds, non-zero
    instance base; each instance's segment equals sampling it alone."""
    rp, col = inputs.rmat_csr(14, 16 << 14, 15)
    offs, seeds, fanouts, bias = inputs.batched_instances(rp, col, 96, 3, lo=1, hi=300, median=40)
    g = csaw.Graph(rp, col)
    res, ref = run_both(csaw, g, rp, col, None, offs, seeds, fanouts, bias, 11, instance_base=5000)
    ni = len(offs) - 1
    o = res.offsets.cpu().numpy()
    for i in (0, 1, 50):
        alone = g.sample(offs[i:i + 2] - offs[i], seeds[offs[i]:offs[i + 1]], fanouts[i], int(bias[i]),
                         rng_seed=11, instance_base=5000 + i)
        ao = alone.offsets.cpu().numpy()
        for l in range(fanouts.shape[1]):
            a, b = o[l * ni + i], o[l * ni + i + 1]
            np.testing.assert_array_equal(res.dst[a:b].cpu().numpy(), alone.dst[ao[l]:ao[l + 1]].cpu().numpy())


def test_wide_build_instance_boundaries(csaw):
    """Bitmaps above 2^20 words are built 16 words per thread; with 4,100
    words per instance (n = 2^17 + 100) a thread's words straddle instance
    boundaries. 300 instances, mixed fanout rows and bias kinds."""
    rp0, col = inputs.rmat_csr(17, 8 << 17, 23)
    rp = np.concatenate([rp0, np.full(100, rp0[-1], dtype=rp0.dtype)])  # 100 isolated vertices
    n = len(rp) - 1
    nwp = ((n + 31) // 32 + 3) // 4 * 4
    assert nwp % 16 != 0 and 300 * nwp > (1 << 20)
    offs, seeds, fanouts, bias = inputs.batched_instances(rp, col, 300, 9, lo=1, hi=40, median=8)
    g = csaw.Graph(rp, col)
    run_both(csaw, g, rp, col, None, offs, seeds, fanouts, bias, 5, instance_base=77)


def test_take_all_uniform_is_bfs(csaw):
    rp, col = inputs.graph_for(inputs.TINY)
    offs, seeds = inputs.single_instance_seeds(rp, col, 8, 2)
    g = csaw.Graph(rp, col)
    run_both(csaw, g, rp, col, None, offs, seeds, [-1, -1, -1], csaw.UNIFORM, 1)


def test_giant_hub(csaw):
    """One vertex with 200,000 weighted neighbors (coarse chunks of several
    64-wide pieces) and the largest drawn fanout, many instances."""
    d = 200_000
    rp = np.array([0, d] + [d] * d, dtype=np.int64)
    col = np.arange(1, d + 1, dtype=np.int32)
    g0 = inputs.rng(9)
    ew = g0.integers(0, 1000, size=d).astype(np.uint32)
    ew[:5] = 1 << 28                                     # a few dominant biases
    ni = 40
    offs = np.arange(ni + 1, dtype=np.int64)
    seeds = np.zeros(ni, dtype=np.int32)
    g = csaw.Graph(rp, col, ew)
    run_both(csaw, g, rp, col, ew, offs, seeds, [64], csaw.EDGE_WEIGHT, 3)
    run_both(csaw, g, rp, col, None, offs, seeds, [64], csaw.UNIFORM, 4)


def test_longest_lists_and_scratch_growth(csaw):
    """Lists of 1.2M weights (more chunks than the coarse table holds, so it
    covers four chunks per entry) in 8 instances, read from the graph's chunk
    prefix table; a second call must return the same edges."""
    d = 1_200_000
    rp = np.array([0, d] + [d] * d, dtype=np.int64)
    col = np.arange(1, d + 1, dtype=np.int32)
    g0 = inputs.rng(21)
    ew = g0.integers(0, 5000, size=d).astype(np.uint32)
    ew[g0.random(d) < 0.3] = 0
    ew[g0.choice(d, 7, replace=False)] = 1 << 26
    ni = 8
    offs = np.arange(ni + 1, dtype=np.int64)
    seeds = np.zeros(ni, dtype=np.int32)
    g = csaw.Graph(rp, col, ew)
    res, ref = run_both(csaw, g, rp, col, ew, offs, seeds, [25], csaw.EDGE_WEIGHT, 13)
    again = g.sample(offs, seeds, [25], csaw.EDGE_WEIGHT, rng_seed=13)
    np.testing.assert_array_equal(again.dst.cpu().numpy(), ref.dst)


def test_small_lists_and_collisions(csaw):
    """Lists barely longer than the fanout force long collision chains."""
    rng = inputs.rng(4)
    n = 3000
    edges = set()
    for u in range(n):
        for x in rng.choice(n, size=int(rng.integers(0, 40)), replace=False):
            if x != u:
                edges.add((u, int(x)))
    rp, col = inputs.csr_from_edges(n, edges)
    ew = (rng.integers(1, 5, size=len(col)) ** 6).astype(np.uint32)
    offs, seeds = inputs.single_instance_seeds(rp, col, 600, 8)
    g = csaw.Graph(rp, col, ew)
    for k in (1, 7, 30, 64):
        run_both(csaw, g, rp, col, ew, offs, seeds, [k, k], csaw.EDGE_WEIGHT, 100 + k)
        run_both(csaw, g, rp, col, ew, offs, seeds, [k], csaw.UNIFORM, 200 + k)


def test_edge_cases(csaw):
    rp = np.array([0, 2, 2, 2, 2], dtype=np.int64)
    col = np.array([1, 2], dtype=np.int32)
    ew = np.array([4, 0], dtype=np.uint32)
    g = csaw.Graph(rp, col, ew)
    say("edge cases")
    # no instances, no layers
    r = g.sample(np.array([0]), np.array([], dtype=np.int32), [3])
    assert r.num_edges == 0
    r = g.sample(np.array([0, 1]), np.array([0], dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert r.num_edges == 0
    # empty instance, duplicate seeds, sink seed, zero-weight neighbor
    offs = np.array([0, 0, 3, 4])
    seeds = np.array([0, 0, 1, 3], dtype=np.int32)
    res = g.sample(offs, seeds, [5, 5], csaw.EDGE_WEIGHT)
    ref = oracle.sample(rp, col, ew, offs, seeds, [5, 5], bias_kind=oracle.EDGE_WEIGHT)
    assert_same(res, ref)
    # zero fanout stops the instance
    res = g.sample(np.array([0, 1]), np.array([0], dtype=np.int32), [1, 0, 1])
    ref = oracle.sample(rp, col, None, np.array([0, 1]), np.array([0], dtype=np.int32), [1, 0, 1])
    assert_same(res, ref)
    # capacity too small: OUT_OF_MEMORY, total still reported
    with pytest.raises(csaw.CsawError) as ei:
        g.sample(np.array([0, 1]), np.array([0], dtype=np.int32), [-1], capacity=1)
    assert ei.value.status == 2
    # seed outside [0, n)
    with pytest.raises(csaw.CsawError) as ei:
        g.sample(np.array([0, 1]), np.array([7], dtype=np.int32), [1])
    assert ei.value.status == 1
    # drawn fanout above the limit
    big = csaw.Graph(np.array([0, 100] + [100] * 100, dtype=np.int64), np.arange(1, 101, dtype=np.int32))
    with pytest.raises(csaw.CsawError) as ei:
        big.sample(np.array([0, 1]), np.array([0], dtype=np.int32), [65])
    assert ei.value.status == 6
    # the workspace is clean afterwards: a normal call still matches
    res = g.sample(offs, seeds, [5, 5], csaw.EDGE_WEIGHT)
    ref = oracle.sample(rp, col, ew, offs, seeds, [5, 5], bias_kind=oracle.EDGE_WEIGHT)
    assert_same(res, ref)


def test_repeat_calls_identical(csaw):
    """Same arguments, same bits: the reused workspace leaves no state behind."""
    rp, col = inputs.rmat_csr(14, 16 << 14, 14)
    offs, seeds = inputs.single_instance_seeds(rp, col, 1000, 5)
    g = csaw.Graph(rp, col)
    say("repeat calls")
    a = g.sample(offs, seeds, [25, 10, 5], csaw.NEIGHBOR_DEGREE, rng_seed=3)
    b = g.sample(offs, seeds, [25, 10, 5], csaw.NEIGHBOR_DEGREE, rng_seed=3)
    assert np.array_equal(a.dst.cpu().numpy(), b.dst.cpu().numpy())
    assert np.array_equal(a.offsets.cpu().numpy(), b.offsets.cpu().numpy())


def test_degree_biased_rmat22_full(csaw):
    """The degree-biased workload at full size (R-MAT 22, 8,192 seeds,
    fanouts [25, 10, 5]) in the benchmark's launch configuration, whole
    output compared with the oracle."""
    rec = inputs.DEGREE_BIASED
    say("full degree-biased R-MAT 22: generating graph")
    rp, col = inputs.graph_for(rec)
    offs, seeds = inputs.single_instance_seeds(rp, col, rec["num_seeds"], rec["seed_rng"])
    g = csaw.Graph(rp, col)
    for s in rec["rng_seeds"][:1]:
        run_both(csaw, g, rp, col, None, offs, seeds, rec["fanouts"], csaw.NEIGHBOR_DEGREE, s)


def test_route_boundaries(csaw):
    """Weighted lists at the lengths where the kernels hand over (wavefront
    kernel / long-list path with a group-level table / with a chunk-level
    table): 512, 513, 8192, 8193, plus short ones, with zero weights and
    dominant weights; two short lists (64, 300) have a total weight above
    2^32 and take the long-list path. Many instances, fanouts up to 64."""
    degs = [16, 64, 300, 512, 513, 1024, 1025, 8192, 8193, 20000]
    hubs = len(degs)
    n = hubs + max(degs)
    rng = inputs.rng(17)
    edges = []
    for h, d in enumerate(degs):
        for x in rng.choice(np.arange(hubs, n), size=d, replace=False):
            edges.append((h, int(x)))
    rp, col = inputs.csr_from_edges(n, edges)
    ew = rng.integers(0, 300, size=len(col)).astype(np.uint32)
    ew[rng.random(len(col)) < 0.2] = 0
    ew[rng.random(len(col)) < 0.002] = 1 << 24
    for h in (1, 2):   # the lists of length 64 and 300: total weight >= 2^32
        a, b = rp[h], rp[h + 1]
        ew[a:b] = rng.integers(1 << 27, 1 << 32, size=b - a, dtype=np.uint64).astype(np.uint32)
        ew[a:b][rng.random(b - a) < 0.2] = 0
        assert int(ew[a:b].astype(np.uint64).sum()) >= 1 << 32
    g = csaw.Graph(rp, col, ew)
    ni = 4 * hubs
    offs = np.arange(ni + 1, dtype=np.int64)
    seeds = np.tile(np.arange(hubs, dtype=np.int32), 4)
    for k in (1, 25, 64):
        run_both(csaw, g, rp, col, ew, offs, seeds, [k], csaw.EDGE_WEIGHT, 50 + k, instance_base=7)


def test_replayed_launch_sequence_matches_eager(csaw):
    """Calls are replayed from a captured launch sequence when possible; with
    kernel profiling on they run eagerly. Both give the same bits, also when
    table contents change under the same shapes."""
    rp, col = inputs.rmat_csr(14, 16 << 14, 19)
    offs, seeds = inputs.single_instance_seeds(rp, col, 700, 21)
    g = csaw.Graph(rp, col)
    say("graph replay vs eager")
    outs = []
    for prof in (False, True, False, False):
        csaw.profile_enable(prof)
        r = g.sample(offs, seeds, [25, 10], csaw.NEIGHBOR_DEGREE, rng_seed=5)
        outs.append((r.dst.cpu().numpy().copy(), r.offsets.cpu().numpy().copy()))
    csaw.profile_enable(False)
    csaw.profile_reset()
    for d, o in outs[1:]:
        np.testing.assert_array_equal(d, outs[0][0])
        np.testing.assert_array_equal(o, outs[0][1])
    # same shapes, different seeds and bias kind: must not reuse stale values
    offs2, seeds2 = inputs.single_instance_seeds(rp, col, 700, 22)
    res = g.sample(offs2, seeds2, [25, 10], csaw.UNIFORM, rng_seed=5)
    ref = oracle.sample(rp, col, None, offs2, seeds2, [25, 10], bias_kind=oracle.UNIFORM, rng_seed=5)
    assert_same(res, ref)


def test_replay_key_covers_bias_kind(csaw):
    """A uniform call and a degree-biased call with the same shapes, seeds
    and output buffers: the biased call needs the long-list kernels that the
    uniform launch sequence does not contain, so it must not replay it."""
    import torch
    rp, col = inputs.rmat_csr(15, 16 << 15, 31)
    assert np.diff(rp).max() > 1024
    offs, seeds = inputs.single_instance_seeds(rp, col, 300, 8)
    g = csaw.Graph(rp, col)
    seeds_dev = torch.from_numpy(seeds).cuda()
    cap = max(g.sample_bound(offs, [25, 10], csaw.UNIFORM), g.sample_bound(offs, [25, 10], csaw.NEIGHBOR_DEGREE))
    out = (torch.empty(cap, dtype=torch.int32, device="cuda"), torch.empty(cap, dtype=torch.int32, device="cuda"),
           torch.empty(3, dtype=torch.int64, device="cuda"))
    say("replay key: uniform then degree-biased, same buffers")
    for bias in (csaw.UNIFORM, csaw.NEIGHBOR_DEGREE, csaw.UNIFORM, csaw.NEIGHBOR_DEGREE):
        res = g.sample(offs, seeds_dev, [25, 10], bias, rng_seed=6, out=out)
        ref = oracle.sample(rp, col, None, offs, seeds, [25, 10], bias_kind=bias, rng_seed=6)
        assert_same(res, ref)


def test_replay_key_covers_bias_tables(csaw):
    """On a weighted graph the edge-weight tables exist from the start and the
    out-degree tables only from their first use. An EDGE_WEIGHT call, then a
    NEIGHBOR_DEGREE call with the same shapes and buffers (both take the
    long-list path), then EDGE_WEIGHT again: none may replay another's
    launch sequence, whose kernel arguments name other bias tables."""
    import torch
    rp, col = inputs.rmat_csr(15, 16 << 15, 33)
    assert np.diff(rp).max() > 1024
    ew = inputs.dst_outdeg_weights(rp, col)
    ew = (ew * 3 + 1).astype(np.uint32)     # not proportional to the degree bias
    offs, seeds = inputs.single_instance_seeds(rp, col, 300, 9)
    g = csaw.Graph(rp, col, ew)
    seeds_dev = torch.from_numpy(seeds).cuda()
    cap = max(g.sample_bound(offs, [25, 10], b) for b in (csaw.EDGE_WEIGHT, csaw.NEIGHBOR_DEGREE))
    out = (torch.empty(cap, dtype=torch.int32, device="cuda"), torch.empty(cap, dtype=torch.int32, device="cuda"),
           torch.empty(3, dtype=torch.int64, device="cuda"))
    say("replay key: edge weight, degree, edge weight, same buffers")
    for bias in (csaw.EDGE_WEIGHT, csaw.NEIGHBOR_DEGREE, csaw.EDGE_WEIGHT, csaw.NEIGHBOR_DEGREE):
        res = g.sample(offs, seeds_dev, [25, 10], bias, rng_seed=6, out=out)
        ref = oracle.sample(rp, col, ew, offs, seeds, [25, 10], bias_kind=bias, rng_seed=6)
        assert_same(res, ref)


def test_visited_picks_leave_no_trace(csaw):
    """Dense graph (cliques of 40): most picks of the second layer are
    already visited. The next bitmap must come back all-zero, so the calls
    that follow (other seeds, other sizes) still match the oracle."""
    n, clique = 4000, 40
    edges = []
    for c0 in range(0, n, clique):
        for u in range(c0, c0 + clique):
            for v in range(c0, c0 + clique):
                if u != v:
                    edges.append((u, v))
    rp, col = inputs.csr_from_edges(n, edges)
    g = csaw.Graph(rp, col)
    say("visited picks, repeated calls")
    for seed_rng, ns, fan in ((1, 300, [20, 20, 20]), (2, 50, [30, 5]), (3, 800, [10, 10, 10])):
        offs, seeds = inputs.single_instance_seeds(rp, col, ns, seed_rng)
        run_both(csaw, g, rp, col, None, offs, seeds, fan, csaw.UNIFORM, seed_rng)


def test_replay_after_staging_growth(csaw):
    """A replayed launch sequence must not outlive the buffers it names: a
    large call grows the workspace's staging buffers between two small calls
    of the same shape, and the second small call still matches the oracle."""
    rp, col = inputs.rmat_csr(13, 16 << 13, 41)
    g = csaw.Graph(rp, col)
    offs, seeds = inputs.single_instance_seeds(rp, col, 50, 3)
    say("replay after staging growth")
    a = g.sample(offs, seeds, [10, 5], csaw.UNIFORM, rng_seed=2)
    big_offs, big_seeds, big_fan, big_bias = inputs.batched_instances(rp, col, 2000, 5, lo=1, hi=20, median=4)
    g.sample(big_offs, big_seeds, big_fan, big_bias, rng_seed=2)
    b = g.sample(offs, seeds, [10, 5], csaw.UNIFORM, rng_seed=2)
    ref = oracle.sample(rp, col, None, offs, seeds, [10, 5], bias_kind=oracle.UNIFORM, rng_seed=2)
    assert_same(a, ref)
    assert_same(b, ref)


TUNINGS = [(0, 0), (16, 0), (0, 32), (8, 32), (16, 32), (1, 1), (4, 20)]


def small_list_graph(n, degrees, seed):
    rng = inputs.rng(seed)
    edges = set()
    for u in range(n):
        d = int(rng.choice(degrees))
        for x in rng.choice(n, size=d, replace=False):
            if x != u:
                edges.add((u, int(x)))
    return inputs.csr_from_edges(n, edges)


def test_subwave_buckets_every_setting(csaw):
    """Sub-wave groups of 16 and 32 lanes against the oracle under every
    bucket setting: unbiased, edge-weight (with zero weights) and out-degree
    bias, take-all lists, draws of up to 32 slots, lists one longer than the
    fanout (slots still open after the rounds go back to the full wavefront)."""
    rp, col = small_list_graph(5000, [0, 1, 3, 9, 15, 16, 17, 20, 31, 32, 33, 40, 70], 31)
    rng = inputs.rng(32)
    ew = rng.integers(0, 4, size=len(col)).astype(np.uint32) ** 5
    offs, seeds = inputs.batched_instances(rp, col, 40, 33)[:2]
    g = csaw.Graph(rp, col, ew)
    bias = [0, 1, 2] * 14
    try:
        for t in TUNINGS:
            g.set_tuning(*t)
            assert g.get_tuning() == t
            say("tuning %s" % (t,))
            for fo in ([15, 5], [16, 31], [32, 3, 2], [8, -1]):
                run_both(csaw, g, rp, col, ew, offs, seeds, fo, bias[:40], 7 + fo[0])
    finally:
        g.set_tuning(16, 32)


def test_subwave_fallback_after_rounds(csaw):
    """Unbiased draws of k from k + 1 or k + 2 candidates leave slots open
    after the rounds in many groups; those entries are redone by the full
    wavefront and must match the oracle exactly."""
    for k in (15, 16, 31, 32):
        rp, col = small_list_graph(3000, [k + 1, k + 2], 40 + k)
        offs, seeds = inputs.single_instance_seeds(rp, col, 1500, 41)
        g = csaw.Graph(rp, col)
        run_both(csaw, g, rp, col, None, offs, seeds, [k, k], csaw.UNIFORM, 3 + k)
        g.set_tuning(0, 0)
        run_both(csaw, g, rp, col, None, offs, seeds, [k, k], csaw.UNIFORM, 3 + k)


def test_autotune_keeps_results(csaw):
    """The autotuner returns the call's exact result and leaves a valid
    setting on the graph."""
    rp, col = inputs.rmat_csr(14, 16 << 14, 5)
    offs, seeds, fan, bias = inputs.batched_instances(rp, col, 64, 9)
    g = csaw.Graph(rp, col)
    say("autotune on R-MAT 14, 64 instances")
    res, t = g.autotune_sample(offs, seeds, fan, bias, rng_seed=4, reps=2)
    assert t in [(0, 0), (8, 0), (16, 0), (0, 32), (8, 32), (16, 32)] and g.get_tuning() == t
    ref = oracle.sample(rp, col, None, offs, seeds, fan, bias_kinds=bias, rng_seed=4)
    assert_same(res, ref)
    with pytest.raises(csaw.CsawError):
        g.set_tuning(17, 0)
    with pytest.raises(csaw.CsawError):
        g.set_tuning(0, 33)
    assert g.get_tuning() == t


def test_long_lists_without_hubs(csaw):
    """The long-list path when the longest list is between 513 and 1024
    weights (one chunk), and for short lists whose total weight is 2^32 or
    more, with both weight arrays (edge weights and out-degrees) in one call."""
    rng = inputs.rng(23)
    degs = [3, 20, 200, 511, 512, 513, 600, 1000, 1024]
    hubs = len(degs)
    n = hubs + 1200
    edges = []
    for h, d in enumerate(degs):
        for x in rng.choice(np.arange(hubs, n), size=d, replace=False):
            edges.append((h, int(x)))
    for u in range(hubs, n):
        for x in rng.choice(n, size=int(rng.integers(0, 6)), replace=False):
            if x != u:
                edges.append((u, int(x)))
    rp, col = inputs.csr_from_edges(n, sorted(set(edges)))
    assert 512 < np.diff(rp).max() <= 1024
    ew = rng.integers(0, 50, size=len(col)).astype(np.uint32)
    for h in (1, 2):   # lists of 20 and 200 with a total weight above 2^32
        a, b = rp[h], rp[h + 1]
        ew[a:b] = rng.integers(1 << 28, 1 << 32, size=b - a, dtype=np.uint64).astype(np.uint32)
        assert int(ew[a:b].astype(np.uint64).sum()) >= 1 << 32
    g = csaw.Graph(rp, col, ew)
    ni = 3 * hubs
    offs = np.arange(ni + 1, dtype=np.int64)
    seeds = np.tile(np.arange(hubs, dtype=np.int32), 3)
    bias = [1, 2] * (ni // 2) + [1] * (ni % 2)
    for k in (2, 10, 64):
        run_both(csaw, g, rp, col, ew, offs, seeds, [k, 3], bias, 70 + k)


@pytest.mark.parametrize("rounds", [-1, 1, 2, 8, 0])
def test_rounds_and_direct_only(csaw, rounds):
    """The number of repeated-sampling rounds before the direct draws is a
    call argument: no rounds at all (every slot by direct draw from the
    updated prefix), 1, 2, 8 or the default; each against the oracle with the
    same rounds, on every route (sub-wave groups, wavefront, long lists)."""
    rp, col = small_list_graph(4000, [0, 2, 5, 12, 16, 30, 60, 200, 700, 1500], 51)
    rng = inputs.rng(52)
    ew = rng.integers(0, 9, size=len(col)).astype(np.uint32) ** 4
    offs, seeds = inputs.batched_instances(rp, col, 24, 53)[:2]
    g = csaw.Graph(rp, col, ew)
    orc_rounds = {-1: 0, 0: 8}.get(rounds, rounds)
    bias = [0, 1, 2] * 8
    say("rounds %d (oracle %d)" % (rounds, orc_rounds))
    res = g.sample(offs, seeds, [10, 25], bias, rng_seed=61, rounds=rounds)
    ref = oracle.sample(rp, col, ew, offs, seeds, [10, 25], bias_kinds=np.asarray(bias, dtype=np.int32),
                        rng_seed=61, rounds=orc_rounds)
    assert_same(res, ref)
    if rounds == -1:
        assert ref.draws == ref.fallbacks > 0
    with pytest.raises(csaw.CsawError):
        g.sample(offs, seeds, [10], 0, rounds=9)
    with pytest.raises(csaw.CsawError):
        g.sample(offs, seeds, [10], 0, rounds=-2)


@pytest.mark.parametrize("burn", [int(0.7 * 2 ** 32), 2 ** 31, 2 ** 32 - 1, 1])
def test_forest_fire(csaw, burn):
    """Forest fire sampling: each frontier vertex's NeighborSize is its burn
    count capped by the fanout (64 for -1), on every route (sub-wave groups,
    wavefront, long lists), all bias kinds, against the oracle."""
    rp, col = small_list_graph(4000, [0, 1, 3, 8, 20, 40, 90, 300, 900, 2000], 81)
    rng = inputs.rng(82)
    ew = rng.integers(0, 7, size=len(col)).astype(np.uint32) ** 3
    offs, seeds = inputs.batched_instances(rp, col, 30, 83)[:2]
    g = csaw.Graph(rp, col, ew)
    bias = [0, 1, 2] * 10
    for fo in ([10, 5], [40, -1, 3]):
        say("forest fire burn=%d fanouts=%s" % (burn, fo))
        res = g.sample(offs, seeds, fo, bias, rng_seed=91, burn=burn)
        ref = oracle.sample(rp, col, ew, offs, seeds, fo, bias_kinds=np.asarray(bias, dtype=np.int32),
                            rng_seed=91, burn=burn)
        assert_same(res, ref)
    if burn == 1:
        assert ref.num_edges == 0


def test_caller_allocator(csaw):
    """Workspace memory from a caller's allocator (torch's caching allocator
    here): same edges as the oracle, and every buffer handed out is returned
    when the graph is destroyed."""
    import torch
    calls = {"alloc": 0, "free": 0}

    def alloc(n):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n)

    def free(p):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    rp, col = inputs.rmat_csr(13, 16 << 13, 44)
    offs, seeds, fan, bias = inputs.batched_instances(rp, col, 20, 45)
    csaw.set_allocator(alloc, free)
    try:
        g = csaw.Graph(rp, col)
        say("sample with a caller allocator")
        res = g.sample(offs, seeds, fan, bias, rng_seed=8)
        ref = oracle.sample(rp, col, None, offs, seeds, fan, bias_kinds=bias, rng_seed=8)
        assert_same(res, ref)
        torch.cuda.synchronize()
        g.close()
        assert calls["alloc"] >= 2 and calls["free"] == calls["alloc"]
    finally:
        csaw.set_allocator(None, None)


@pytest.mark.parametrize("rng_seed", [3, 4])
def test_sparse_frontier_build(csaw, rng_seed):
    """Instance bitmaps of more than 2^23 words (1,100 instances of a 2^18-vertex
    graph) take the sparse frontier build: claims record dirty words in a
    summary bitmap, which is compacted into an ordered dirty-word list. Empty
    seed sets (also first and last), instances that stop early and long gaps
    of instances without frontier entries give the segment offsets every
    case; whole outputs against the oracle, and the next call on the same
    workspace is exact too (summary and bitmaps left clean)."""
    rp, col = inputs.rmat_csr(18, 16 << 18, 181)
    ew = inputs.dst_outdeg_weights(rp, col)
    g = csaw.Graph(rp, col, ew)
    gen = inputs.rng(rng_seed)
    ni = 1100
    pool = inputs.non_isolated(rp, col)
    counts = gen.integers(0, 40, size=ni)
    counts[0] = counts[-1] = 0
    counts[300:420] = 0
    seeds = [inputs.distinct_seeds(gen, pool, int(c)) for c in counts]
    offs = np.zeros(ni + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(x) for x in seeds])
    rows = np.array([[10, 5, 3], [25, 0, 0], [5, 5, 5], [-1, 2, 0]], dtype=np.int32)
    fan = rows[gen.integers(0, len(rows), size=ni)]
    bias = gen.integers(0, 3, size=ni).astype(np.int32)
    seeds = np.concatenate(seeds).astype(np.int32)
    assert ni * ((len(rp) - 1 + 31) // 32) > (1 << 23)
    run_both(csaw, g, rp, col, ew, offs, seeds, fan, bias, rng_seed, instance_base=77)
    run_both(csaw, g, rp, col, ew, offs, seeds, fan, bias, rng_seed + 10)


def light_run_hub(heavy, runs, run_len):
    """Vertex 0 adjacent to runs * (run_len + 1) leaves: per run one weight
    `heavy` then run_len weights of 1 (the leaves point back to vertex 0)."""
    d = runs * (run_len + 1)
    rp = np.concatenate([[0, d], np.arange(d + 1, 2 * d + 1)]).astype(np.int64)
    col = np.concatenate([np.arange(1, d + 1), np.zeros(d)]).astype(np.int32)
    ew = np.ones(2 * d, dtype=np.uint32)
    ew[0:d:run_len + 1] = heavy
    return rp, col, ew


@pytest.mark.parametrize("case", ["giant_hub", "rmat16_degree", "direct_only", "wide", "light_runs"])
def test_long_lists_through_the_walk_guide(csaw, case):
    """Weighted long lists draw through the walk guide once a weighted walk
    has built it for their weight array (two dependent loads a draw), and
    through the chunk tables before that or with the guide off: the same
    edges every time, equal to the oracle. Cases: a 200,000-neighbor hub with
    a few dominant weights; degree bias on R-MAT 16; no repeated-sampling
    rounds (every slot by the direct draw, whose held-candidate sums need
    each pick's exclusive prefix and weight); weights near 2^32 (totals of
    64 bits); runs of unit weights inside guide buckets (brackets longer
    than a probe)."""
    rounds = 0
    if case == "giant_hub":
        d = 200_000
        rp = np.array([0, d] + [d] * d, dtype=np.int64)
        col = np.arange(1, d + 1, dtype=np.int32)
        ew = inputs.rng(9).integers(0, 1000, size=d).astype(np.uint32)
        ew[:5] = 1 << 28
        offs, seeds, fan, bias = np.arange(41, dtype=np.int64), np.zeros(40, dtype=np.int32), [64], 1
    elif case in ("rmat16_degree", "direct_only"):
        rp, col = inputs.rmat_csr(16, 16 << 16, 61)
        ew = None
        offs, seeds = inputs.single_instance_seeds(rp, col, 3000, 62)
        fan, bias = [25, 10], 2
        rounds = -1 if case == "direct_only" else 0
    elif case == "wide":
        rp, col = inputs.rmat_csr(15, 16 << 15, 63)
        ew = inputs.rng(64).integers((1 << 32) - 1000, 1 << 32, size=len(col), dtype=np.uint64).astype(np.uint32)
        offs, seeds = inputs.single_instance_seeds(rp, col, 2000, 65)
        fan, bias = [25, 10], 1
    else:
        rp, col, ew = light_run_hub(207_000, 8, 100)
        offs, seeds, fan, bias = np.arange(65, dtype=np.int64), np.zeros(64, dtype=np.int32), [40], 1
    assert np.diff(rp).max() > 512
    orc_rounds = {-1: 0, 0: 8}.get(rounds, rounds)
    ref = oracle.sample(rp, col, ew, offs, seeds, fan, bias_kind=bias, rng_seed=71, rounds=orc_rounds)
    g = csaw.Graph(rp, col, ew)
    say("long lists %s: chunk tables" % case)
    assert_same(g.sample(offs, seeds, fan, bias, rng_seed=71, rounds=rounds), ref)
    g.walk(np.array([int(seeds[0])], dtype=np.int32), 1, bias, rng_seed=1)  # builds the guide
    say("long lists %s: walk guide" % case)
    assert_same(g.sample(offs, seeds, fan, bias, rng_seed=71, rounds=rounds), ref)
    g.set_walk_guides(False)
    say("long lists %s: guide off" % case)
    assert_same(g.sample(offs, seeds, fan, bias, rng_seed=71, rounds=rounds), ref)
