"""CPU oracle for C-SAW's bias-based vertex selection (arXiv 2009.09103).

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library (``paper_2009_09103_amd``) and never imports it; both only
share the seeded input generators in ``paper_2009_09103_amd.inputs``, which
hold none of the method's arithmetic.

The arithmetic lives in ``csaw_oracle.c`` (plain C, one loop per definition);
this module compiles it with gcc and wraps it with ctypes/numpy. Functions and
the passages they follow:

* ``philox``      -- Philox4x32-10 (Salmon et al., SC'11); the paper's cuRAND
                     stand-in (Section VI).
* ``range_reduce``-- r = floor(u*W/2^64), the integer form of drawing r in
                     (0,1) against the normalised CTPS (Section II-B).
* ``its``         -- inverse transform search (Section II-B, Eq. equ:tp).
* ``skip_map``    -- Theorem 2's inverse (Eq. eq:brs_random), integer form,
                     any number of pre-selected candidates.
* ``select``      -- Select over one pool, without replacement (Section IV-B).
* ``sample``      -- the generic loop of fig:api(b) for neighbor sampling.
* ``walk``        -- first-order biased random walks and node2vec (Section II-A).

Parity status: every function above is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csaw_oracle.c")
_LIB = os.path.join(_HERE, "libcsaw_oracle.so")
_lock = threading.Lock()
_lib = None

UNIFORM, EDGE_WEIGHT, NEIGHBOR_DEGREE, NODE2VEC, METROPOLIS = 0, 1, 2, 3, 4
FANOUT_ALL = -1
DEFAULT_ROUNDS = 8   # repeated-sampling rounds before the direct draw


def _host_stamp() -> str:
    """The host CPU's model and feature flags: -march=native code is only
    reused on the CPU it was built for."""
    model = flags = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not model and line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                elif not flags and line.startswith("flags"):
                    flags = line.split(":", 1)[1].strip()
                if model and flags:
                    break
    except OSError:
        pass
    return hashlib.sha256((model + "|" + flags).encode()).hexdigest()[:16]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 -march=native, OpenMP). Returns the
    library path. Without force, an existing library is reused only if it is
    newer than the source and was built on a CPU with the same features."""
    stamp = _LIB + ".host"
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        try:
            with open(stamp) as f:
                if f.read().strip() == _host_stamp():
                    return _LIB
        except OSError:
            pass
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    with open(stamp + ".tmp%d" % os.getpid(), "w") as f:
        f.write(_host_stamp() + "\n")
    os.replace(stamp + ".tmp%d" % os.getpid(), stamp)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
            vp = ctypes.c_void_p
            L.orc_philox4x32_10.argtypes = [vp, vp, vp]
            L.orc_philox4x32_10.restype = None
            L.orc_range.argtypes = [u64, u64]
            L.orc_range.restype = u64
            L.orc_draw.argtypes = [u64, u32, u32, u32, u32, u64]
            L.orc_draw.restype = u64
            L.orc_prefix.argtypes = [vp, i64, vp]
            L.orc_prefix.restype = None
            L.orc_its.argtypes = [vp, i64, u64]
            L.orc_its.restype = i64
            L.orc_skip_map.argtypes = [vp, vp, vp, i32, u64]
            L.orc_skip_map.restype = u64
            L.orc_select.argtypes = [vp, i64, i64, i32, u64, u32, u32, u32, vp, vp, vp]
            L.orc_select.restype = i32
            L.orc_sample.argtypes = [i64, vp, vp, vp, i32, vp, vp, u64, vp, i32, vp, i32, vp, i32,
                                     u64, i32, u32, i64, vp, vp, vp, vp, vp, i32]
            L.orc_burn_count.argtypes = [u64, u32, u32, u32, u32, i32]
            L.orc_burn_count.restype = i32
            L.orc_sample.restype = i32
            L.orc_walk.argtypes = [i64, vp, vp, vp, i32, u32, u32, u32, i64, vp, u64, vp, i32, u64,
                                   u32, u32, vp, vp, vp, i32]
            L.orc_walk.restype = i32
            L.orc_layer_sample.argtypes = [i64, vp, vp, vp, i32, vp, vp, u64, i32, vp, i32, u64, i32, vp, vp, vp]
            L.orc_layer_sample.restype = i32
            L.orc_mdrw.argtypes = [i64, vp, vp, i32, vp, vp, u64, i64, u64, vp, vp, vp]
            L.orc_mdrw.restype = i32
            L.orc_max_threads.argtypes = []
            L.orc_max_threads.restype = i32
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox(key, ctr):
    """Philox4x32-10 block: key (k0, k1), counter (c0..c3) -> 4 uint32 words."""
    k = np.asarray(key, dtype=np.uint32)
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(k), _p(c), _p(out))
    return out


def range_reduce(u: int, W: int) -> int:
    return int(lib().orc_range(u, W))


def draw(rng_seed: int, c0: int, c1: int, c2: int, c3: int, W: int) -> int:
    return int(lib().orc_draw(rng_seed, c0, c1, c2, c3, W))


def prefix(b):
    """Exclusive prefix sum S[0..d] of the biases (uint64)."""
    b = np.ascontiguousarray(b, dtype=np.uint32)
    S = np.zeros(len(b) + 1, dtype=np.uint64)
    lib().orc_prefix(_p(b), len(b), _p(S))
    return S


def its(S, r: int) -> int:
    S = np.ascontiguousarray(S, dtype=np.uint64)
    return int(lib().orc_its(_p(S), len(S) - 1, r))


def skip_map(S, b, acc_sorted, r: int) -> int:
    S = np.ascontiguousarray(S, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    a = np.ascontiguousarray(acc_sorted, dtype=np.int64)
    return int(lib().orc_skip_map(_p(S), _p(b), _p(a), len(a), r))


def burn_count(rng_seed: int, c0: int, c1: int, c2: int, burn: int, cap: int) -> int:
    """Forest fire NeighborSize of one vertex (see ``orc_burn_count``)."""
    return int(lib().orc_burn_count(rng_seed, c0, c1, c2, burn, cap))


def select(b, k: int, rng_seed: int, c0: int, c1: int, c2: int, rounds: int = DEFAULT_ROUNDS,
           with_fallback: bool = False):
    """Select min(k, P) distinct positions of the bias list ``b`` (slot order)."""
    b = np.ascontiguousarray(b, dtype=np.uint32)
    d = len(b)
    out = np.zeros(max(d, 1), dtype=np.int64)
    nfb = ctypes.c_int32(0)
    c = lib().orc_select(_p(b), d, k, rounds, rng_seed, c0, c1, c2, _p(out), ctypes.byref(nfb), None)
    res = out[:c].copy()
    return (res, nfb.value) if with_fallback else res


class SampleResult:
    def __init__(self, src, dst, offsets, num_layers, num_instances, stats):
        self.src, self.dst, self.offsets = src, dst, offsets
        self.num_layers, self.num_instances = num_layers, num_instances
        self.alg_bytes, self.expanded, self.fallbacks, self.sum_degree, self.draws = stats

    def segment(self, layer: int, instance: int):
        o = self.offsets
        a, b = o[layer * self.num_instances + instance], o[layer * self.num_instances + instance + 1]
        return self.src[a:b], self.dst[a:b]

    @property
    def num_edges(self) -> int:
        return int(self.offsets[-1])


def sample(rowptr, col, ew, seed_offsets, seeds, fanouts, bias_kind=UNIFORM, rng_seed=1,
           instance_base=0, instance_ids=None, bias_kinds=None, rounds=DEFAULT_ROUNDS,
           nthreads=0, burn=0) -> SampleResult:
    """Neighbor sampling for a batch of instances (see ``orc_sample``).

    fanouts: 1-D (shared by all instances) or 2-D [num_instances, num_layers]."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    ew = None if ew is None else np.ascontiguousarray(ew, dtype=np.uint32)
    seed_offsets = np.ascontiguousarray(seed_offsets, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    fo = np.ascontiguousarray(fanouts, dtype=np.int32)
    ni = len(seed_offsets) - 1
    if fo.ndim == 1:
        L, stride = fo.shape[0], 0
    else:
        assert fo.shape[0] == ni
        L, stride = fo.shape[1], fo.shape[1]
    n = len(rowptr) - 1
    ids = None if instance_ids is None else np.ascontiguousarray(instance_ids, dtype=np.uint64)
    bk = None if bias_kinds is None else np.ascontiguousarray(bias_kinds, dtype=np.int32)
    offsets = np.zeros(L * ni + 1, dtype=np.int64)
    stats = np.zeros(5, dtype=np.float64)
    ne = ctypes.c_int64(0)
    cap = 0
    src = np.zeros(1, dtype=np.int32)
    dst = np.zeros(1, dtype=np.int32)
    for _ in range(2):
        rc = lib().orc_sample(n, _p(rowptr), _p(col), _p(ew), ni, _p(seed_offsets), _p(seeds),
                              instance_base, _p(ids), L, _p(fo), stride, _p(bk), bias_kind,
                              rng_seed, rounds, burn, cap, _p(src), _p(dst), _p(offsets),
                              ctypes.byref(ne), _p(stats), nthreads)
        if rc == 1:
            raise ValueError("oracle: invalid sampling input")
        if rc == 0:
            break
        cap = ne.value
        src = np.zeros(max(cap, 1), dtype=np.int32)
        dst = np.zeros(max(cap, 1), dtype=np.int32)
    m = ne.value
    return SampleResult(src[:m].copy(), dst[:m].copy(), offsets, L, ni, tuple(stats))


def walk(rowptr, col, ew, starts, length, bias_kind=UNIFORM, rng_seed=1, walker_base=0,
         walker_ids=None, node2vec=(1, 1, 1), nthreads=0, restart=0, jump=0):
    """Random walks (see ``orc_walk``); restart / jump are the per-step
    thresholds in [0, 2^32] (probability * 2^32). Returns (paths [nw,
    length+1], steps [nw], stats)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    ew = None if ew is None else np.ascontiguousarray(ew, dtype=np.uint32)
    starts = np.ascontiguousarray(starts, dtype=np.int32)
    nw = len(starts)
    ids = None if walker_ids is None else np.ascontiguousarray(walker_ids, dtype=np.uint64)
    paths = np.zeros((nw, length + 1), dtype=np.int32)
    steps = np.zeros(nw, dtype=np.int64)
    stats = np.zeros(2, dtype=np.float64)
    wr, wc, wo = node2vec
    rc = lib().orc_walk(len(rowptr) - 1, _p(rowptr), _p(col), _p(ew), bias_kind, wr, wc, wo, nw,
                        _p(starts), walker_base, _p(ids), length, rng_seed, restart, jump, _p(paths),
                        _p(steps), _p(stats), nthreads)
    if rc != 0:
        raise ValueError("oracle: invalid walk input")
    return paths, steps, tuple(stats)


def layer_sample(rowptr, col, ew, seed_offsets, seeds, fanouts, bias_kind=UNIFORM, rng_seed=1,
                 instance_base=0, rounds=DEFAULT_ROUNDS):
    """Layer sampling (see ``orc_layer_sample``). Returns (src [ni, L, K],
    dst [ni, L, K], counts [ni, L]) with K = max(fanouts), -1 padded."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    ew = None if ew is None else np.ascontiguousarray(ew, dtype=np.uint32)
    so = np.ascontiguousarray(seed_offsets, dtype=np.int64)
    sd = np.ascontiguousarray(seeds, dtype=np.int32)
    fo = np.ascontiguousarray(fanouts, dtype=np.int32)
    ni, L = len(so) - 1, len(fo)
    K = int(fo.max()) if L else 0
    src = np.zeros((ni, L, K), dtype=np.int32)
    dst = np.zeros((ni, L, K), dtype=np.int32)
    counts = np.zeros((ni, L), dtype=np.int32)
    rc = lib().orc_layer_sample(len(rowptr) - 1, _p(rowptr), _p(col), _p(ew), ni, _p(so), _p(sd), instance_base,
                                L, _p(fo), bias_kind, rng_seed, rounds, _p(src), _p(dst), _p(counts))
    if rc != 0:
        raise ValueError("oracle: invalid layer-sampling input")
    return src, dst, counts


def mdrw(rowptr, col, pool_offsets, pool, budget, rng_seed=1, instance_base=0):
    """Multi-dimensional random walks (see ``orc_mdrw``): one frontier pool
    per instance. Returns (src [ni, budget], dst [ni, budget], steps [ni]);
    -1 marks edges after an instance has ended."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    pool_offsets = np.ascontiguousarray(pool_offsets, dtype=np.int64)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    ni = len(pool_offsets) - 1
    src = np.zeros((ni, budget), dtype=np.int32)
    dst = np.zeros((ni, budget), dtype=np.int32)
    steps = np.zeros(max(ni, 1), dtype=np.int64)
    rc = lib().orc_mdrw(len(rowptr) - 1, _p(rowptr), _p(col), ni, _p(pool_offsets), _p(pool), instance_base,
                        budget, rng_seed, _p(src), _p(dst), _p(steps))
    if rc != 0:
        raise ValueError("oracle: invalid multi-dimensional random walk input")
    return src, dst, steps[:ni]


def max_threads() -> int:
    return int(lib().orc_max_threads())
