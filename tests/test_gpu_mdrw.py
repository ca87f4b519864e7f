"""GPU parity of the multi-dimensional random walk (frontier sampling): the
HIP kernel through the C-ABI against the CPU oracle, bit for bit."""
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


def run_both(csaw, g, rp, col, pools, budget, rng_seed=1, base=0):
    po = np.concatenate([[0], np.cumsum([len(p) for p in pools])]).astype(np.int64)
    pool = np.concatenate(pools).astype(np.int32) if len(pools) else np.zeros(0, np.int32)
    say("mdrw n=%d ni=%d pools=%s budget=%d seed=%d" % (len(rp) - 1, len(pools), [len(p) for p in pools][:6],
                                                        budget, rng_seed))
    src, dst, steps, total = g.mdrw(po, pool, budget, rng_seed=rng_seed, instance_base=base)
    rs, rd, rst = oracle.mdrw(rp, col, po, pool, budget, rng_seed=rng_seed, instance_base=base)
    np.testing.assert_array_equal(src.cpu().numpy(), rs)
    np.testing.assert_array_equal(dst.cpu().numpy(), rd)
    np.testing.assert_array_equal(steps.cpu().numpy(), rst)
    assert total == int(rst.sum())
    return rs, rst


def test_pool_sizes_and_budgets(csaw):
    """Pools of 1 (a simple walk) to the largest supported size, budgets
    around the 64-step output batches, degree-zero pool vertices."""
    rp, col = inputs.rmat_csr(14, 16 << 14, 21)
    g = csaw.Graph(rp, col)
    n = len(rp) - 1
    gen = np.random.Generator(np.random.PCG64(8))
    sizes = [1, 2, 63, 64, 65, 200, 1000, 2047, 2048]
    pools = [gen.integers(0, n, size=k).astype(np.int32) for k in sizes]
    for budget in (0, 1, 63, 64, 65, 300):
        run_both(csaw, g, rp, col, pools, budget, rng_seed=budget + 1, base=40)


def test_paper_scale_instances(csaw):
    """2,000 instances with pools of 2,000 vertices (the paper's frontier
    size) on R-MAT 18, 1,703 edges each; instances are independent, so the
    oracle checks the first 150 of them."""
    rp, col = inputs.rmat_csr(18, 16 << 18, 22)
    g = csaw.Graph(rp, col)
    pool_vertices = inputs.non_isolated(rp, col)
    gen = np.random.Generator(np.random.PCG64(9))
    pools = [pool_vertices[gen.integers(0, len(pool_vertices), size=2000)] for _ in range(2000)]
    po = np.concatenate([[0], np.cumsum([len(p) for p in pools])]).astype(np.int64)
    say("mdrw paper scale: 2000 instances x pool 2000 x 1703 steps")
    src, dst, steps, total = g.mdrw(po, np.concatenate(pools), 1703, rng_seed=3)
    k = 150
    rs, rd, rst = oracle.mdrw(rp, col, po[:k + 1], np.concatenate(pools[:k]), 1703, rng_seed=3)
    np.testing.assert_array_equal(src[:k].cpu().numpy(), rs)
    np.testing.assert_array_equal(dst[:k].cpu().numpy(), rd)
    assert steps.cpu().numpy().min() == 1703 and total == 2000 * 1703


def test_dead_pools_and_edge_cases(csaw):
    rp, col = inputs.graph_for(inputs.TINY)
    deg = np.diff(rp)
    sinks = np.nonzero(deg == 0)[0].astype(np.int32)
    assert len(sinks) >= 3
    g = csaw.Graph(rp, col)
    live = np.nonzero(deg > 0)[0].astype(np.int32)
    # an all-sink pool ends at once; an empty pool too; a pool that runs into sinks ends early
    rs, rst = run_both(csaw, g, rp, col, [sinks[:3], np.zeros(0, np.int32), live[:5], sinks[:1]], 50, rng_seed=5)
    assert rst[0] == 0 and rst[1] == 0 and rst[3] == 0
    run_both(csaw, g, rp, col, [], 10)
    with pytest.raises(csaw.CsawError):
        g.mdrw(np.array([0, 1]), np.array([len(rp) + 3], dtype=np.int32), 4)      # vertex out of range
    with pytest.raises(csaw.CsawError) as ei:
        g.mdrw(np.array([0, 2049]), np.zeros(2049, dtype=np.int32), 4)             # pool too large
    assert ei.value.status == 6
    run_both(csaw, g, rp, col, [live[:7]], 20, rng_seed=6)                         # a clean call after errors
