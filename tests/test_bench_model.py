"""The bench's algorithmic byte model on CPU: computed from the oracle's
output of a small call, it must count every frontier entry and edge once,
and the sub-wave split must not change the total."""
import importlib.util
import os

import numpy as np

import oracle
from paper_2009_09103_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_byte_model_counts_entries_and_edges():
    bench = load_bench()
    rp, col = inputs.rmat_csr(12, 40000, 3)
    deg = np.diff(rp)
    ppos = np.add.reduceat(np.append((deg[col] > 0).astype(np.int64), 0), rp[:-1])
    ppos[deg == 0] = 0
    offs, seeds = inputs.single_instance_seeds(rp, col, 300, 4)
    fan = [10, 5]
    for weighted, kind in ((False, oracle.UNIFORM), (True, oracle.NEIGHBOR_DEGREE)):
        ref = oracle.sample(rp, col, None, offs, seeds, fan, bias_kind=kind, rng_seed=2)
        base = bench.path_bytes(rp, ppos, seeds, ref.dst, ref.offsets, fan, weighted, 0)
        split = bench.path_bytes(rp, ppos, seeds, ref.dst, ref.offsets, fan, weighted, 16)
        assert base["select_small"] == 0
        assert abs(sum(base.values()) - sum(split.values())) < 1e-6
        assert split["select_small"] > 0
        # without weights every frontier entry costs 24 B and every edge 12 B
        if not weighted:
            frontier, visited, entries = np.unique(seeds), set(np.unique(seeds).tolist()), 0
            for l in range(len(fan)):
                entries += len(frontier)
                a, b = ref.offsets[l], ref.offsets[l + 1]
                nxt = sorted(set(ref.dst[a:b].tolist()) - visited)
                visited |= set(nxt)
                frontier = np.array(nxt, dtype=np.int64)
            assert sum(base.values()) == 24.0 * entries + 12.0 * ref.num_edges


def test_walk_step_bytes_by_route():
    """Per step 16 B (two 32-bit row offsets, the pick's id, the path entry)
    plus the cheaper selection: 4 d for a list of at most 512 weights read
    whole, or 24 B through the guide (total, bracket, one prefix); steps after
    a walk ended (-1) are not counted."""
    bench = load_bench()
    deg = np.array([3, 600, 512, 0, 1])
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    paths = np.array([[0, 1, 2, 4, 0],
                      [1, 1, 3, -1, -1],
                      [2, -1, -1, -1, -1]], dtype=np.int32)
    b, steps = bench.walk_step_bytes(rp, paths)
    # taken steps leave 0, 1, 2, 4 (row 0); 1, 1 (row 1)
    assert steps == 6
    assert b == 16 * 6 + 4 * 3 + 24 + 24 + 4 * 1 + 24 + 24


def test_node2vec_bytes_by_route():
    """A node2vec step costs 20 + 4 d_v + 4 d_t, or with a short previous
    list (d_t < 64) and a long current one (d_v >= 2,048) 20 + 4 d_t plus
    8 (d_t + 1) ceil(log2(d_v + 1)) + 4; the first step 24."""
    bench = load_bench()
    deg = np.array([3, 3000, 10, 100])
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    paths = np.array([[0, 1, 2, 3, -1]], dtype=np.int32)
    b, steps = bench.walk_bytes_node2vec(rp, paths)
    assert steps == 3
    lv = np.ceil(np.log2(3001.0))
    exp = 24 + (20 + 8 * 4 * lv + 4 + 4 * 3) + (20 + 4 * 10 + 4 * 3000)
    assert abs(b - exp) < 1e-6
