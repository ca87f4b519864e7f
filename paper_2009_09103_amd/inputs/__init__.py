"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module generates INPUTS only (graphs, seed sets, walker starts, request
traces). It holds none of the sampling method's arithmetic, so both the GPU
library and the CPU oracle may consume what it produces.

Graphs are R-MAT (a=.57, b=.19, c=.19, d=.05) built by ``rmat.c``: power-law
stand-ins for the paper's SNAP/KONECT datasets (Section VI, Table of datasets),
which are not available here. Scale 22 is about LiveJournal's size and scale 26
about Friendster's vertex count.

Workload recipes (sizes and distributions) are named after what they are:

* ``tiny_uniform``           -- R-MAT 12 (4,096 vertices, 65,536 edge draws),
  one instance of 256 distinct seeds, fanouts [10, 5], unbiased, Philox seed 1.
* ``degree_biased_rmat22``   -- R-MAT 22, edge factor 16; one instance of 8,192
  distinct seeds; fanouts [25, 10, 5]; bias = out-degree of the neighbor.
* ``node2vec_rmat24``        -- symmetrised R-MAT 24; 2^20 walkers; length 80;
  node2vec weights {return 1, common 2, outward 4}.
* ``batched_rmat22``         -- R-MAT 22; 4,096 instances; seeds per instance
  clip(round(lognormal(ln 256, 1)), 16, 4096); fanouts per instance uniform over
  {[10,5], [25,10], [15,10,5]}; unbiased for even ids, degree-biased for odd.
* ``served_rmat26``          -- R-MAT 26 with edge weights = out-degree of the
  destination; Poisson request trace (60% sampling, 40% weighted walks).

Seeds and walker starts are drawn uniformly from vertices with at least one
incident edge (an edge-list graph has no isolated vertices).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "librmat.so")
_lock = threading.Lock()
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", tmp,
                    _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _rmat():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            vp = ctypes.c_void_p
            L.rmat_build_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_int, vp, vp, ctypes.c_int64, ctypes.c_int]
            L.rmat_build_csr.restype = ctypes.c_int64
            L.rmat_dst_outdeg_weights.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp,
                                                  ctypes.c_int]
            L.rmat_dst_outdeg_weights.restype = None
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def rmat_csr(scale: int, num_edges: int, gen_seed: int, symmetrize: bool = False,
             abc=RMAT_ABC, nthreads: int = 0):
    """R-MAT graph as CSR: (rowptr int64[n+1], col int32[m]), sorted, no
    self-loops, no duplicates; n = 2**scale."""
    n = 1 << scale
    slots = 2 * num_edges if symmetrize else num_edges
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(slots, 1), dtype=np.int32)
    a, b, c = abc
    m = _rmat().rmat_build_csr(scale, num_edges, a, b, c, gen_seed, int(bool(symmetrize)),
                               _p(rowptr), _p(col), slots, nthreads)
    if m < 0:
        raise MemoryError("rmat_build_csr failed (%d)" % m)
    return rowptr, col[:m]


def dst_outdeg_weights(rowptr, col, nthreads: int = 0):
    """uint32 edge weights w[e] = out-degree of col[e]."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.empty(len(col), dtype=np.uint32)
    _rmat().rmat_dst_outdeg_weights(len(rowptr) - 1, len(col), _p(rowptr), _p(col), _p(w), nthreads)
    return w


def csr_from_edges(n: int, edges):
    """CSR of a small explicit edge list (sorted lists, duplicates and
    self-loops kept out by the caller)."""
    edges = sorted(set((int(u), int(v)) for u, v in edges))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    for u, _ in edges:
        rowptr[u + 1] += 1
    rowptr = np.cumsum(rowptr).astype(np.int64)
    col = np.array([v for _, v in edges], dtype=np.int32)
    return rowptr, col


def non_isolated(rowptr, col):
    """Vertices with at least one incident (in or out) edge."""
    n = len(rowptr) - 1
    outd = np.diff(rowptr)
    ind = np.bincount(col, minlength=n)
    return np.nonzero((outd > 0) | (ind > 0))[0].astype(np.int32)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def distinct_seeds(gen: np.random.Generator, pool, k: int):
    pool = np.asarray(pool)
    k = min(k, len(pool))
    return np.sort(gen.choice(pool, size=k, replace=False)).astype(np.int32)


# ---------------------------------------------------------------------------
# Toy graph of the paper's worked example: v8's neighbors v5, v7, v9, v10,
# v11 have degrees 3, 6, 2, 2, 2 (fig:example(a); the image itself is not
# available, so the rest of the graph is filled in to give those degrees).
# ---------------------------------------------------------------------------
def paper_toy_graph():
    edges = set()

    def link(u, v):
        edges.add((u, v))
        edges.add((v, u))

    for x in (5, 7, 9, 10, 11):
        link(8, x)
    # v5: degree 3 -> two more neighbors
    link(5, 0); link(5, 1)
    # v7: degree 6 -> five more neighbors
    for x in (0, 1, 2, 3, 4):
        link(7, x)
    # v9, v10, v11: degree 2 -> one more neighbor each (distinct new ids)
    link(9, 12); link(10, 13); link(11, 14)
    # the extra ids only touch the vertices above, so the listed degrees hold
    return csr_from_edges(15, edges)


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------
TINY = dict(name="tiny_uniform", scale=12, num_edges=65536, gen_seed=12, symmetrize=False,
            num_seeds=256, seed_rng=1001, fanouts=[10, 5], bias="uniform", rng_seed=1)
DEGREE_BIASED = dict(name="degree_biased_rmat22", scale=22, num_edges=16 << 22, gen_seed=22,
                     symmetrize=False, num_seeds=8192, seed_rng=2202, fanouts=[25, 10, 5],
                     bias="neighbor_degree", rng_seeds=(1, 2, 3))
NODE2VEC = dict(name="node2vec_rmat24", scale=24, num_edges=16 << 24, gen_seed=24,
                symmetrize=True, num_walkers=1 << 20, start_rng=2404, length=80,
                node2vec=(1, 2, 4), rng_seeds=(1, 2, 3))
BATCHED = dict(name="batched_rmat22", scale=22, num_edges=16 << 22, gen_seed=22,
               symmetrize=False, num_instances=4096, seed_rng=4404,
               fanout_choices=([10, 5], [25, 10], [15, 10, 5]), rng_seeds=(1, 2, 3))
SERVED = dict(name="served_rmat26", scale=26, num_edges=16 << 26, gen_seed=26, symmetrize=False,
              trace_rng=5505, sample_fraction=0.6)


def graph_for(recipe, scale=None, num_edges=None, nthreads=0):
    """Build the recipe's graph (optionally at a reduced scale for tests)."""
    s = recipe["scale"] if scale is None else scale
    m = recipe["num_edges"] if num_edges is None else num_edges
    return rmat_csr(s, m, recipe["gen_seed"], recipe["symmetrize"], nthreads=nthreads)


def single_instance_seeds(rowptr, col, num_seeds: int, seed_rng: int):
    """(seed_offsets int64[2], seeds int32[k]): one instance of distinct seeds."""
    seeds = distinct_seeds(rng(seed_rng), non_isolated(rowptr, col), num_seeds)
    return np.array([0, len(seeds)], dtype=np.int64), seeds


def walker_starts(rowptr, col, num_walkers: int, start_rng: int):
    """Uniform (with replacement) starts over vertices with an incident edge."""
    pool = non_isolated(rowptr, col)
    return pool[rng(start_rng).integers(0, len(pool), size=num_walkers)].astype(np.int32)


def batched_instances(rowptr, col, num_instances: int, seed_rng: int,
                      fanout_choices=BATCHED["fanout_choices"], lo=16, hi=4096, median=256.0,
                      sigma=1.0):
    """Per-instance seed sets, fanout rows and bias kinds of the batched workload.

    Returns (seed_offsets int64[ni+1], seeds int32, fanouts int32[ni, Lmax]
    zero-padded, bias_kinds int32[ni]: 0 = unbiased for even instance ids,
    2 = out-degree of the neighbor for odd ids)."""
    g = rng(seed_rng)
    pool = non_isolated(rowptr, col)
    counts = np.clip(np.rint(g.lognormal(np.log(median), sigma, size=num_instances)), lo, hi)
    counts = counts.astype(np.int64)
    choice = g.integers(0, len(fanout_choices), size=num_instances)
    lmax = max(len(f) for f in fanout_choices)
    fanouts = np.zeros((num_instances, lmax), dtype=np.int32)
    seeds = []
    for i in range(num_instances):
        f = fanout_choices[choice[i]]
        fanouts[i, :len(f)] = f
        seeds.append(distinct_seeds(g, pool, int(counts[i])))
    offs = np.zeros(num_instances + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in seeds])
    bias = np.where(np.arange(num_instances) % 2 == 0, 0, 2).astype(np.int32)
    return offs, np.concatenate(seeds).astype(np.int32), fanouts, bias


def request_trace(rowptr, col, num_requests: int, qps: float, trace_rng: int,
                  sample_fraction: float = 0.6, fanout_choices=BATCHED["fanout_choices"]):
    """Poisson arrivals of mixed requests for the served workload.

    Each request is a dict with ``kind`` ('sample' or 'walk'), ``arrival_s``,
    ``rng_seed`` (= request id) and its arguments: sampling requests have
    log-uniform [64, 8192] distinct seeds, a fanout row of the batched set and
    a bias kind (unbiased for even ids, out-degree for odd); walk requests
    have log-uniform [1024, 65536] walkers and a length uniform in [10, 80]
    (edge-weight biased)."""
    g = rng(trace_rng)
    pool = non_isolated(rowptr, col)
    t = np.cumsum(g.exponential(1.0 / qps, size=num_requests))
    reqs = []
    for rid in range(num_requests):
        if g.random() < sample_fraction:
            k = int(np.rint(np.exp(g.uniform(np.log(64), np.log(8192)))))
            f = list(fanout_choices[int(g.integers(0, len(fanout_choices)))])
            reqs.append(dict(kind="sample", id=rid, arrival_s=float(t[rid]), rng_seed=rid,
                             seeds=distinct_seeds(g, pool, k), fanouts=f,
                             bias=0 if rid % 2 == 0 else 2))
        else:
            nw = int(np.rint(np.exp(g.uniform(np.log(1024), np.log(65536)))))
            reqs.append(dict(kind="walk", id=rid, arrival_s=float(t[rid]), rng_seed=rid,
                             starts=pool[g.integers(0, len(pool), size=nw)].astype(np.int32),
                             length=int(g.integers(10, 81)), bias=1))
    return reqs
