#!/usr/bin/env python3
"""Benchmark of the biased neighbor-selection hot path on one MI355X.

Default workload (--workload served): the served stream on R-MAT 26 (edge
weights = out-degree of the destination), resident in HBM. A Poisson trace of
mixed requests (60% neighbor sampling with 64-8,192 seeds, 40% weighted
walks of 1k-64k walkers, length 10-80) is swept over QPS through the
continuous-batching server and through the plain path (one request at a
time); each QPS point is one step. Prints one JSON line: served SEPS (sampled
edges and walk steps per second of wall time) with p50/p99 latency per
point against the plain path, the roofline of the dominant kernel (the
weighted walk) from HIP-event kernel times and the algorithmic byte model,
and the CPU oracle timed on a sample of the trace on the host.

--workload degree_biased: one full csaw_sample call per step (every layer:
frontier build, select, long-list search) over R-MAT 22 (edge factor 16), one
instance of 8,192 distinct seeds, fanouts [25, 10, 5], bias = out-degree of
the neighbor, Philox seeds cycling over {1, 2, 3}; the sub-wave bucket
setting is autotuned on the timed call first (--tuning).

Other workloads: batched (4,096 instances in one call against 4,096 plain
calls), node2vec (R-MAT 24 walks), mdrw (multi-dimensional random walks),
forest_fire (burning probability 0.7, depth 2), metropolis
(Metropolis-Hastings walks), layer (layer sampling), walks (edge-weight
walks on the served R-MAT 26 graph, --walkers per call, one lane per walker
from 12,288), copy (a 1 GiB device copy, the HBM counter calibration).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import faulthandler
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


WAVE_MAX_D = 512  # longer (or 2^32-heavy) weighted lists that need draws take the long-list path


def small_bucket(c, d, k, take, wflag, long_, bound):
    """Entries served by the sub-wave kernel (select_small) under the bucket
    bound max(bound16, bound32): take-all and weighted lists of at most
    `bound` candidates, unbiased draws of at most `bound` slots."""
    if bound <= 0:
        return np.zeros(len(c), dtype=bool)
    size = np.where(take | wflag, d, k)
    return (c > 0) & ~long_ & (size <= bound)


def path_bytes(rowptr, ppos, seeds, dst, offsets, fanouts, weighted, bound=0):
    """Algorithmic bytes of one call, per kernel, from the graph and the
    call's own output. Per frontier vertex: 8 (frontier entry) + 16 (row-offset
    pair) bytes of metadata. Lists drawn by the wavefront kernels (select_small
    for the sub-wave buckets, select_wave for the rest) add 4*deg if the bias
    reads a weight array; a long weighted list (select_big) reads one 8-byte
    group prefix per 16 weights from the graph's chunk prefix table (built once
    per graph, so not part of a call). Every emitted edge costs 12 (neighbor id
    read + edge written) in the kernel that draws it."""
    deg = np.diff(rowptr)
    L = len(fanouts)
    visited = np.unique(seeds)
    frontier = visited
    out = {"select_small": 0.0, "select_wave": 0.0, "select_big": 0.0}
    for l in range(L):
        a, b = offsets[l], offsets[l + 1]
        k = int(fanouts[l])
        d = deg[frontier].astype(np.float64)
        P = ppos[frontier] if weighted else deg[frontier]
        c = np.where((k == 0) | (P == 0), 0, np.where((k < 0) | (k >= P), P, k)).astype(np.float64)
        assert int(c.sum()) == b - a
        long_ = weighted & (k > 0) & (k < P) & (deg[frontier] > WAVE_MAX_D)
        sm = small_bucket(c, d, k, (k < 0) | (k >= P), np.full(len(c), weighted), long_, bound)
        for name, w in (("select_small", sm), ("select_wave", ~long_ & ~sm)):
            out[name] += 24.0 * w.sum() + 12.0 * c[w].sum() + (4.0 * d[w].sum() if weighted else 0.0)
        groups = np.ceil(d[long_] / 16.0)
        out["select_big"] += 24.0 * long_.sum() + 8.0 * groups.sum() + 12.0 * c[long_].sum()
        if l + 1 < L:
            nxt = np.setdiff1d(np.unique(dst[a:b]), visited, assume_unique=True)
            visited = np.union1d(visited, nxt)
            frontier = nxt
    return out


def cpu_baseline(rp, col, offs, seeds, fanouts, bias, min_s=10.0, max_runs=60):
    """The CPU oracle on the host: the whole call, cycling over Philox seeds
    1, 2, 3 until at least min_s seconds of oracle time have been spent, on
    every host thread (each layer's frontier split over them; bit-identical
    to one thread) and on one thread."""
    import oracle
    out = {}
    for nthreads in (oracle.max_threads(), 1):
        t_used, edges, runs = 0.0, 0, 0
        while t_used < (min_s if nthreads > 1 else min_s / 2) and runs < max_runs:
            s = 1 + runs % 3
            t0 = time.perf_counter()
            ref = oracle.sample(rp, col, None, offs, seeds, fanouts, bias_kind=bias, rng_seed=s, nthreads=nthreads)
            t_used += time.perf_counter() - t0
            edges += ref.num_edges
            runs += 1
        out[nthreads] = (edges / t_used, runs, t_used)
    nt = max(out)
    return dict(value=out[nt][0], unit="sampled edges/s", cores=int(nt), kind="oracle", value_1thread=out[1][0],
                sample="full workload (all %d seeds, all layers), %d calls cycling over Philox seeds 1..3, %.1f s "
                       "on %d host threads; 1 thread: %d calls, %.1f s" % (
                           len(seeds), out[nt][1], out[nt][2], nt, out[1][1], out[1][2]))


def apply_tuning(g, args, *call, **kw):
    """Sub-wave bucket setting for the timed calls: the library default, a
    fixed "b16,b32", or "auto" (the library's autotuner run on the timed call
    itself; every setting gives the same edges)."""
    if args.tuning == "auto":
        _, t = g.autotune_sample(*call, reps=3, **kw)
        log("autotuner chose bound16=%d bound32=%d" % t)
    elif args.tuning != "default":
        g.set_tuning(*(int(x) for x in args.tuning.split(",")))
    return {"bound16": g.get_tuning()[0], "bound32": g.get_tuning()[1], "source": args.tuning}


def bench_degree_biased(args):
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.DEGREE_BIASED
    log("generating R-MAT %d graph" % rec["scale"])
    t0 = time.perf_counter()
    rp, col = inputs.graph_for(rec)
    offs, seeds = inputs.single_instance_seeds(rp, col, rec["num_seeds"], rec["seed_rng"])
    log("graph n=%d m=%d in %.1fs" % (len(rp) - 1, len(col), time.perf_counter() - t0))
    g = csaw.Graph(rp, col)
    dev = g.device
    fan = np.asarray(rec["fanouts"], dtype=np.int32)
    bias = csaw.NEIGHBOR_DEGREE
    seeds_d = torch.from_numpy(seeds).to(dev)
    cap = g.sample_bound(offs, fan, bias)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    offsets = torch.empty(len(fan) + 1, dtype=torch.int64, device=dev)
    rng_seeds = list(rec["rng_seeds"])

    # per-seed edge counts and algorithmic bytes (deterministic per seed)
    deg = np.diff(rp)
    ppos = np.add.reduceat(np.append((deg[col] > 0).astype(np.int64), 0), rp[:-1])
    ppos[deg == 0] = 0
    edges_of, bytes_of = {}, {}
    tuning = apply_tuning(g, args, offs, seeds_d, fan, bias, rng_seed=rng_seeds[0], rounds=args.rounds,
                          out=(src, dst, offsets))
    bound = max(tuning["bound16"], tuning["bound32"])
    for s in rng_seeds:
        r = g.sample(offs, seeds_d, fan, bias, rounds=args.rounds, rng_seed=s, out=(src, dst, offsets))
        o = offsets.cpu().numpy()
        edges_of[s] = r.num_edges
        bytes_of[s] = path_bytes(rp, ppos, seeds, dst[:r.num_edges].cpu().numpy(), o, fan, True, bound)
        log("seed %d: %d edges" % (s, r.num_edges))

    for i in range(args.warmup):
        g.sample(offs, seeds_d, fan, bias, rounds=args.rounds, rng_seed=rng_seeds[i % 3], out=(src, dst, offsets))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_edges = 0
    for i in range(args.steps):
        s = rng_seeds[i % 3]
        g.sample(offs, seeds_d, fan, bias, rounds=args.rounds, rng_seed=s, out=(src, dst, offsets))
        total_edges += edges_of[s]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    seps = total_edges / dt

    # kernel times from HIP events on the call's stream (separate pass)
    csaw.profile_reset()
    csaw.profile_enable(True)
    alg = {"select_small": 0.0, "select_wave": 0.0, "select_big": 0.0}
    for i in range(args.steps):
        s = rng_seeds[i % 3]
        g.sample(offs, seeds_d, fan, bias, rounds=args.rounds, rng_seed=s, out=(src, dst, offsets))
        for k in alg:
            alg[k] += bytes_of[s][k]
    torch.cuda.synchronize()
    times = {k: csaw.profile_read(k) for k in ("frontier_init", "select_small", "select_wave", "select_big",
                                                "frontier_build", "visited_clear")}
    csaw.profile_enable(False)
    csaw.profile_reset()
    sel_ms, sel_n = times["select_wave"]
    achieved = alg["select_wave"] / (sel_ms / 1e3) / 1e9 if sel_ms > 0 else 0.0
    per_kernel = {k: {"alg_bytes_per_step": alg[k] / args.steps, "ms_per_step": times[k][0] / args.steps,
                      "GB_per_s": alg[k] / (times[k][0] / 1e3) / 1e9 if times[k][0] > 0 else 0.0}
                  for k in alg}
    step_bytes = sum(alg.values()) / args.steps
    log("kernel ms per step: " + ", ".join("%s %.3f" % (k, v[0] / args.steps) for k, v in times.items()))

    line = {
        "metric": "sampled edges/sec (SEPS) + HBM roofline % on 1 GPU; p50/p99 served latency",
        "value": seps,
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bias / u64 prefix (integer)",
        "data": "synthetic",
        "config": {"workload": rec["name"], "graph": "R-MAT scale 22, edge factor 16 (a=.57,b=.19,c=.19)",
                   "n": int(len(rp) - 1), "m": int(len(col)), "instances": 1,
                   "seeds": int(len(seeds)), "fanouts": rec["fanouts"], "bias": "out-degree of neighbor",
                   "rng_seeds": rng_seeds, "edges_per_step": float(np.mean(list(edges_of.values()))),
                   "tuning": tuning, "rounds": args.rounds or 8},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("traffic_select_degree_biased_rmat22.md"),
                     "kernel": "select_wave (k_select)", "launches": sel_n,
                     "avg_launch_us": sel_ms / max(sel_n, 1) * 1e3,
                     "alg_bytes_per_launch": alg["select_wave"] / max(sel_n, 1)},
        "roofline_step": {"alg_bytes": step_bytes, "achieved": step_bytes / (dt / args.steps) / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_bytes / (dt / args.steps) / 1e9 / HBM_PEAK_GBS},
        "kernels": per_kernel,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in times.items()},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(rp, col, offs, seeds, rec["fanouts"], 2)
    return line


def path_bytes_multi(rowptr, ppos, seed_offs, seeds, dst, offsets, fanouts, bias, bound=0):
    """path_bytes for a multi-instance call: frontier entries are (instance,
    vertex) pairs (keys instance * n + vertex), each instance with its own
    fanout row and bias kind; offsets[l * ni + i] is the first edge of (layer
    l, instance i). Same per-entry figures as path_bytes."""
    n = len(rowptr) - 1
    deg = np.diff(rowptr)
    ni = len(seed_offs) - 1
    L = fanouts.shape[1]
    inst_of_seed = np.repeat(np.arange(ni, dtype=np.int64), np.diff(seed_offs))
    visited = np.unique(inst_of_seed * n + seeds.astype(np.int64))
    frontier = visited
    out = {"select_small": 0.0, "select_wave": 0.0, "select_big": 0.0}
    for l in range(L):
        inst = frontier // n
        v = frontier % n
        k = fanouts[inst, l].astype(np.int64)
        wflag = bias[inst] != 0
        d = deg[v].astype(np.float64)
        P = np.where(wflag, ppos[v], deg[v])
        c = np.where((k == 0) | (P == 0), 0, np.where((k < 0) | (k >= P), P, k)).astype(np.float64)
        assert int(c.sum()) == offsets[(l + 1) * ni] - offsets[l * ni]
        long_ = wflag & (k > 0) & (k < P) & (deg[v] > WAVE_MAX_D)
        sm = small_bucket(c, d, k, (k < 0) | (k >= P), wflag, long_, bound)
        for name, w in (("select_small", sm), ("select_wave", ~long_ & ~sm)):
            out[name] += 24.0 * w.sum() + 12.0 * c[w].sum() + 4.0 * d[w & wflag].sum()
        groups = np.ceil(d[long_] / 16.0)
        out["select_big"] += 24.0 * long_.sum() + 8.0 * groups.sum() + 12.0 * c[long_].sum()
        if l + 1 < L:
            a, b = offsets[l * ni], offsets[(l + 1) * ni]
            edge_inst = np.repeat(np.arange(ni, dtype=np.int64), np.diff(offsets[l * ni:(l + 1) * ni + 1]))
            keys = np.unique(edge_inst * n + dst[a:b].astype(np.int64))
            keys = keys[fanouts[keys // n, l + 1] != 0]  # picks are claimed only for a next layer
            nxt = np.setdiff1d(keys, visited, assume_unique=True)
            visited = np.union1d(visited, nxt)
            frontier = nxt
    return out


def bench_batched(args):
    """4,096 uneven instances in one csaw_sample call (the launch sequence is
    replayed from a captured graph) against the same instances as 4,096 plain
    calls; both outputs are identical by construction of the draws."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.BATCHED
    log("generating R-MAT %d graph" % rec["scale"])
    rp, col = inputs.graph_for(rec)
    offs, seeds, fanouts, bias = inputs.batched_instances(rp, col, rec["num_instances"], rec["seed_rng"])
    g = csaw.Graph(rp, col)
    dev = g.device
    ni = len(offs) - 1
    seeds_d = torch.from_numpy(seeds).to(dev)
    cap = g.sample_bound(offs, fanouts, bias)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    offsets = torch.empty(fanouts.shape[1] * ni + 1, dtype=torch.int64, device=dev)
    r = g.sample(offs, seeds_d, fanouts, bias, rng_seed=1, rounds=args.rounds, out=(src, dst, offsets))
    edges = r.num_edges
    tuning = apply_tuning(g, args, offs, seeds_d, fanouts, bias, rng_seed=1, rounds=args.rounds,
                          out=(src, dst, offsets))
    for _ in range(args.warmup):
        g.sample(offs, seeds_d, fanouts, bias, rng_seed=1, rounds=args.rounds, out=(src, dst, offsets))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sample(offs, seeds_d, fanouts, bias, rng_seed=1, rounds=args.rounds, out=(src, dst, offsets))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # algorithmic bytes of the call and kernel times from one event-timed pass
    deg = np.diff(rp)
    ppos = np.add.reduceat(np.append((deg[col] > 0).astype(np.int64), 0), rp[:-1])
    ppos[deg == 0] = 0
    alg = path_bytes_multi(rp, ppos, offs, seeds, dst[:edges].cpu().numpy(), offsets.cpu().numpy(), fanouts, bias,
                           max(tuning["bound16"], tuning["bound32"]))
    csaw.profile_reset()
    csaw.profile_enable(True)
    g.sample(offs, seeds_d, fanouts, bias, rng_seed=1, rounds=args.rounds, out=(src, dst, offsets))
    torch.cuda.synchronize()
    times = {k: csaw.profile_read(k) for k in ("frontier_init", "select_small", "select_wave", "select_big",
                                                "frontier_build", "visited_clear")}
    csaw.profile_enable(False)
    csaw.profile_reset()
    sel_ms, sel_n = times["select_wave"]
    achieved = alg["select_wave"] / (sel_ms / 1e3) / 1e9 if sel_ms > 0 else 0.0
    step_bytes = sum(alg.values())
    # plain: one call per instance (same ids, same seed)
    per = []
    for i in range(ni):
        so = np.array([0, offs[i + 1] - offs[i]], dtype=np.int64)
        per.append((so, seeds_d[offs[i]:offs[i + 1]], fanouts[i], int(bias[i])))
    pcap = max(g.sample_bound(so, f, b) for so, _, f, b in per)
    psrc = torch.empty(max(pcap, 1), dtype=torch.int32, device=dev)
    pdst = torch.empty(max(pcap, 1), dtype=torch.int32, device=dev)
    poff = torch.empty(fanouts.shape[1] + 1, dtype=torch.int64, device=dev)
    plain_edges = 0
    for i, (so, sd, f, b) in enumerate(per[:64]):
        g.sample(so, sd, f, b, rng_seed=1, instance_base=i, rounds=args.rounds, out=(psrc, pdst, poff))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (so, sd, f, b) in enumerate(per):
        plain_edges += g.sample(so, sd, f, b, rng_seed=1, instance_base=i, rounds=args.rounds, out=(psrc, pdst, poff)).num_edges
    torch.cuda.synchronize()
    pdt = time.perf_counter() - t0
    assert plain_edges == edges
    split = batched_split(g, offs, seeds, fanouts, bias, args, edges)
    return {
        "metric": "sampled edges/sec (SEPS), batched multi-instance vs plain per-instance calls",
        "value": edges / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": rec["name"], "instances": ni, "seeds": int(len(seeds)),
                   "edges_per_step": int(edges), "tuning": tuning, "rounds": args.rounds or 8},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "select_wave (k_select)",
                     "launches": sel_n, "avg_launch_us": sel_ms / max(sel_n, 1) * 1e3,
                     "alg_bytes_per_launch": alg["select_wave"] / max(sel_n, 1)},
        "roofline_step": {"alg_bytes": step_bytes, "achieved": step_bytes / dt / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_bytes / dt / 1e9 / HBM_PEAK_GBS},
        "kernels": {k: {"alg_bytes_per_step": alg[k], "ms_per_step": times[k][0],
                        "GB_per_s": alg[k] / (times[k][0] / 1e3) / 1e9 if times[k][0] > 0 else 0.0} for k in alg},
        "kernel_ms_per_step": {k: v[0] for k, v in times.items()},
        "plain_calls": {"value": plain_edges / pdt, "calls": ni, "seconds": pdt},
        "batched_over_plain": (edges / dt) / (plain_edges / pdt),
        "split_streams_ms": split,
    }


def batched_split(g, offs, seeds, fanouts, bias, args, edges):
    """The batch's layer barrier, measured: the instances split into k
    interleaved sub-batches (instance i in sub-batch i mod k, ids kept, so
    every instance draws the same edges) run as k concurrent calls on k
    streams from k host threads. If the barrier's tail (a layer waiting for
    its slowest instances) cost time, independent sub-batches would fill each
    other's tails and finish sooner; per-instance layer progression is the
    limit k = number of instances. Returns ms per step for each k."""
    import threading
    import torch
    dev = g.device
    ni = len(offs) - 1
    out = {}
    for k in (1, 2, 4):
        subs = []
        for j in range(k):
            ids = np.arange(j, ni, k)
            cnt = (offs[ids + 1] - offs[ids]).astype(np.int64)
            so = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
            sd = np.concatenate([seeds[offs[i]:offs[i + 1]] for i in ids]).astype(np.int32)
            fo, bi = fanouts[ids], bias[ids]
            cap = g.sample_bound(so, fo, bi)
            o = (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
                 torch.empty(fanouts.shape[1] * len(ids) + 1, dtype=torch.int64, device=dev))
            subs.append(dict(so=so, sd=torch.from_numpy(sd).to(dev), fo=fo, bi=bi, ids=ids.astype(np.uint64), out=o,
                             stream=torch.cuda.Stream(device=dev)))
        counts = [0] * k

        def run(j):
            b = subs[j]
            r = g.sample(b["so"], b["sd"], b["fo"], b["bi"], rng_seed=1, rounds=args.rounds, out=b["out"],
                         instance_ids=b["ids"], stream=b["stream"])
            counts[j] = r.num_edges

        def step():
            th = [threading.Thread(target=run, args=(j,)) for j in range(k)]
            for t in th:
                t.start()
            for t in th:
                t.join()

        for _ in range(max(args.warmup, 1)):
            step()
        torch.cuda.synchronize()
        assert sum(counts) == edges, (k, sum(counts), edges)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        out[str(k)] = (time.perf_counter() - t0) / args.steps * 1e3
        log("batched split into %d concurrent sub-batches: %.2f ms per step" % (k, out[str(k)]))
    return out


def walk_step_bytes(rowptr, paths):
    """Algorithmic bytes of first-order weighted walk steps, per step from v
    with d = deg(v): 8 (the two 32-bit row offsets) + 4 (the pick's neighbor
    id) + 4 (the path entry), plus what the selection reads at least: through
    the walk guide, the list's total (8), the two bracket bounds (8) and one
    exact prefix (8); a list of at most 512 weights may instead be read whole
    (4 d), which a wavefront per walker does, so the smaller of the two is
    counted. A bracket holds one position or a few, so this is a lower bound
    on the bytes any route needs."""
    deg = np.diff(rowptr)
    cur, nxt = paths[:, :-1], paths[:, 1:]
    taken = nxt >= 0
    d = deg[cur[taken]].astype(np.float64)
    sel = np.where(d <= WAVE_MAX_D, np.minimum(4.0 * d, 24.0), 24.0)
    return 16.0 * taken.sum() + sel.sum(), int(taken.sum())


def run_server(csaw, g, trace, kw, profile=False):
    """One pass of a request trace through a fresh server: Poisson arrivals
    from a client thread, then every result. Returns throughput, latency
    percentiles and the results."""
    import threading
    srv = csaw.Server(g, **kw)
    tickets = [None] * len(trace)
    errors = []
    if profile:
        csaw.profile_reset()
        csaw.profile_enable(True)
    start = time.perf_counter()

    def client():
        try:
            for k, r in enumerate(trace):
                delay = r["arrival_s"] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
                if r["kind"] == "sample":
                    tickets[k] = srv.submit_sample(r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"],
                                                   request_id=r["id"])
                else:
                    tickets[k] = srv.submit_walk(r["starts"], r["length"], r["bias"], rng_seed=r["rng_seed"],
                                                 request_id=r["id"])
        except Exception as e:  # reported by the caller
            errors.append(e)
    th = threading.Thread(target=client)
    th.start()
    th.join()
    if errors:
        srv.close()
        raise errors[0]
    lat, edges, results = [], 0, []
    for t in tickets:
        res = srv.wait(t)
        if res.status != 0:
            srv.close()
            raise RuntimeError("a served request failed with status %d" % res.status)
        lat.append(res.total_us)
        edges += res.num_edges
        results.append(res)
    wall = time.perf_counter() - start
    if profile:
        csaw.profile_enable(False)
    srv.close()
    lat = np.array(lat) / 1e3
    row = {"seps": edges / wall, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "wall_s": wall, "edges": int(edges), "requests": len(trace)}
    return row, results


def served_cpu_baseline(rp, col, ew, trace, qps, min_s=10.0):
    """The CPU oracle on a bounded sample of the served trace: requests in
    trace order (sampling requests whole, walk requests on every 16th walker
    id, an exact subset) until min_s seconds of oracle time; edges/s on all
    host threads and on one."""
    import oracle
    out = {}
    for nthreads in (oracle.max_threads(), 1):
        t_used, edges, done = 0.0, 0, 0
        for r in trace:
            t0 = time.perf_counter()
            if r["kind"] == "sample":
                ref = oracle.sample(rp, col, ew, np.array([0, len(r["seeds"])], dtype=np.int64), r["seeds"],
                                    r["fanouts"], bias_kind=r["bias"], rng_seed=r["rng_seed"],
                                    instance_base=r["id"], nthreads=nthreads)
                edges += ref.num_edges
            else:
                sub = np.arange(0, len(r["starts"]), 16)
                _, steps, _ = oracle.walk(rp, col, ew, r["starts"][sub], r["length"], bias_kind=r["bias"],
                                          rng_seed=r["rng_seed"], walker_ids=r["id"] + sub.astype(np.uint64),
                                          nthreads=nthreads)
                edges += int(steps.sum())
            t_used += time.perf_counter() - t0
            done += 1
            if t_used >= min_s / 2 and nthreads == 1 or t_used >= min_s:
                break
        out[nthreads] = (edges / t_used, done, t_used)
    nt = max(out)
    return dict(value=out[nt][0], unit="sampled edges/s", cores=int(nt), kind="oracle",
                value_1thread=out[1][0],
                sample="the first %d requests of the %g-QPS trace (sampling whole, walks on every 16th walker id), "
                       "%.1f s on %d host threads; 1 thread: %d requests, %.1f s" % (
                           out[nt][1], qps, out[nt][2], nt, out[1][1], out[1][2]))


def bench_served(args):
    """Served stream on R-MAT 26 (edge weights = destination out-degree): a
    Poisson trace of mixed requests (60% sampling, 40% weighted walks) swept
    over QPS, through the continuous-batching server (three executors, batches
    of up to 256 requests) and through the plain path (one executor, one
    request at a time). A step is one QPS point of the served server."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.SERVED
    scale = args.served_scale or rec["scale"]
    log("generating R-MAT %d graph" % scale)
    t0 = time.perf_counter()
    rp, col = inputs.graph_for(rec, scale=scale, num_edges=16 << scale)
    ew = inputs.dst_outdeg_weights(rp, col)
    g = csaw.Graph(rp, col, ew)
    log("graph n=%d m=%d ready in %.1fs" % (len(rp) - 1, len(col), time.perf_counter() - t0))
    pool = 2 << 30  # pinned host result memory, touched at creation, for both paths
    served_kw = dict(num_streams=3, max_batch=256, memory_budget_bytes=48 << 30, max_batch_walkers=1 << 18,
                     result_pool_bytes=pool)
    plain_kw = dict(num_streams=1, max_batch=1, memory_budget_bytes=16 << 30, result_pool_bytes=pool)
    # up to 102,400 QPS, where the 400 requests arrive within 4 ms and the
    # server runs saturated
    qps_list = args.qps or [400.0, 1600.0, 6400.0, 25600.0, 102400.0]
    points = []
    for qps in qps_list:
        trace = inputs.request_trace(rp, col, args.requests, qps, rec["trace_rng"], rec["sample_fraction"])
        row = {"qps": qps}
        for name, kw in (("served", served_kw), ("plain", plain_kw)):
            # a pass lasts tens of milliseconds, so one pass is noisy: the
            # point reports the pass with the median throughput of several
            runs = []
            for t in range(args.passes):
                st, _ = run_server(csaw, g, trace, kw)
                runs.append(st)
                log("qps %g %s pass %d: %d requests, %.3g SEPS, p50 %.1f ms, p99 %.1f ms, %.3f s" % (
                    qps, name, t, len(trace), st["seps"], st["p50_ms"], st["p99_ms"], st["wall_s"]))
            runs.sort(key=lambda st: st["seps"])
            row[name] = dict(runs[len(runs) // 2], passes_seps=[st["seps"] for st in runs])
        row["served_over_plain"] = row["served"]["seps"] / row["plain"]["seps"]
        points.append(row)
    best = max(points, key=lambda r: r["served"]["seps"])
    # roofline: one more served pass at the best point with kernel events on
    trace = inputs.request_trace(rp, col, args.requests, best["qps"], rec["trace_rng"], rec["sample_fraction"])
    _, results = run_server(csaw, g, trace, served_kw, profile=True)
    kernels = {}
    for name in ("walk", "select_wave", "select_big", "select_small", "frontier_build", "frontier_init",
                 "visited_clear"):
        ms, n = csaw.profile_read(name)
        kernels[name] = {"ms": ms, "launches": n}
    wbytes, wsteps = 0.0, 0
    for r, res in zip(trace, results):
        if r["kind"] == "walk":
            b, st = walk_step_bytes(rp, res.paths)
            wbytes += b
            wsteps += st
    walk_ms = kernels["walk"]["ms"]
    achieved = wbytes / (walk_ms * 1e-3) / 1e9 if walk_ms > 0 else 0.0
    copy_gbps = measured_copy_gbps()
    # HBM bytes per walk launch of this pass: the counter record's bytes per
    # step (taken on the same trace) times this pass's steps per launch
    per_step = measured_traffic("traffic_walk_served_rmat26.md", WALK_SOURCES, "hbm_bytes_per_step")
    walk_traffic = per_step * wsteps / max(kernels["walk"]["launches"], 1) if per_step else None
    line = {
        "metric": "sampled edges/sec (SEPS) + HBM roofline % on 1 GPU; p50/p99 served latency",
        "value": best["served"]["seps"], "unit": "sampled edges/s", "n_gpus": 1, "steps": len(points),
        "warmup": 0, "ms_per_step": best["served"]["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": rec["name"], "graph": "R-MAT scale %d, edge factor 16, edge weight = out-degree of "
                   "the destination" % scale, "n": len(rp) - 1, "m": len(col),
                   "requests_per_point": args.requests, "passes_per_point": args.passes, "qps": qps_list,
                   "sample_fraction": rec["sample_fraction"],
                   "served": served_kw, "plain": plain_kw},
        "p50_ms": best["served"]["p50_ms"], "p99_ms": best["served"]["p99_ms"],
        "points": points,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": walk_traffic,
                     "measured_copy_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                     "kernel": "walk (k_walk_lane and k_walk_wave_first, edge-weight walks)", "launches": kernels["walk"]["launches"],
                     "avg_launch_us": walk_ms * 1e3 / max(kernels["walk"]["launches"], 1),
                     "alg_bytes_per_launch": wbytes / max(kernels["walk"]["launches"], 1),
                     "steps": wsteps,
                     # the walk step is a chain of dependent loads: its rate is
                     # bound by wavefront slots over the chain's latency, not HBM
                     "steps_per_s": wsteps / (walk_ms * 1e-3) if walk_ms > 0 else 0.0},
        "kernels_ms": {k: v["ms"] for k, v in kernels.items()},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample of the trace")
        line["cpu_baseline"] = served_cpu_baseline(rp, col, ew, trace, best["qps"])
    return line


def bench_streamed(args):
    """Out-of-memory sampling: the degree-biased R-MAT 22 call with the
    graph's adjacency and weights in pinned host memory, in 4 vertex-range
    partitions of which at most 2 are resident (partition loads inside the
    timed region), against the same call on the resident graph."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.DEGREE_BIASED
    log("generating R-MAT %d graph" % rec["scale"])
    rp, col = inputs.graph_for(rec)
    offs, seeds = inputs.single_instance_seeds(rp, col, rec["num_seeds"], rec["seed_rng"])
    g = csaw.Graph(rp, col)
    dev = g.device
    seeds_d = torch.from_numpy(seeds).to(dev)
    cap = g.sample_bound(offs, rec["fanouts"], csaw.NEIGHBOR_DEGREE)
    out = (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
           torch.empty(len(rec["fanouts"]) + 1, dtype=torch.int64, device=dev))
    pg = csaw.PartitionedGraph(rp, col, None, num_partitions=args.partitions, max_resident=args.resident)

    def timed(graph, stats):
        for k in range(args.warmup):
            graph.sample(offs, seeds_d, rec["fanouts"], csaw.NEIGHBOR_DEGREE, rng_seed=1 + k % 3, out=out)
        torch.cuda.synchronize()
        edges, loads, nbytes = 0, 0, 0
        t0 = time.perf_counter()
        for k in range(args.steps):
            r = graph.sample(offs, seeds_d, rec["fanouts"], csaw.NEIGHBOR_DEGREE, rng_seed=1 + k % 3, out=out)
            edges += r.num_edges
            if stats:
                loads += graph.last_stats[0]
                nbytes += graph.last_stats[1]
        torch.cuda.synchronize()
        return edges, time.perf_counter() - t0, loads, nbytes

    e_s, t_s, loads, nbytes = timed(pg, True)
    e_m, t_m, _, _ = timed(g, False)
    log("streamed %.3g edges/s (%.2f loads, %.1f MB per call), in memory %.3g edges/s" % (
        e_s / t_s, loads / args.steps, nbytes / args.steps / 1e6, e_m / t_m))
    return {
        "metric": "sampled edges/sec, graph streamed from host memory in partitions",
        "value": e_s / t_s, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_s / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": "streamed_degree_biased_rmat22", "partitions": args.partitions,
                   "max_resident": args.resident, "n": len(rp) - 1, "m": len(col), "seeds": len(seeds),
                   "fanouts": rec["fanouts"]},
        "partition_loads_per_call": loads / args.steps, "bytes_loaded_per_call": nbytes / args.steps,
        "load_GB_per_s": nbytes / t_s / 1e9,
        "in_memory": {"value": e_m / t_m, "ms_per_step": t_m / args.steps * 1e3},
    }


def bench_forest_fire(args):
    """Forest fire sampling at the paper's setting (burning probability 0.7,
    depth 2, unbiased) on the R-MAT 22 graph, 8,192 seeds in one instance;
    the fanout -1 caps each burn count at 64."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.DEGREE_BIASED
    log("generating R-MAT %d graph" % rec["scale"])
    rp, col = inputs.graph_for(rec)
    offs, seeds = inputs.single_instance_seeds(rp, col, rec["num_seeds"], rec["seed_rng"])
    g = csaw.Graph(rp, col)
    dev = g.device
    fan = np.array([-1, -1], dtype=np.int32)
    burn = int(0.7 * 2 ** 32)
    seeds_d = torch.from_numpy(seeds).to(dev)
    cap = g.sample_bound(offs, fan, csaw.UNIFORM)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    dst = torch.empty(cap, dtype=torch.int32, device=dev)
    offsets = torch.empty(len(fan) + 1, dtype=torch.int64, device=dev)
    call = dict(rng_seed=1, burn=burn, rounds=args.rounds, out=(src, dst, offsets))
    tuning = apply_tuning(g, args, offs, seeds_d, fan, csaw.UNIFORM, **call)
    r = g.sample(offs, seeds_d, fan, csaw.UNIFORM, **call)
    edges = r.num_edges
    # per layer: frontier entries (24 B each: entry + row offsets) and edges (12 B each)
    o = offsets.cpu().numpy()
    d_host = dst[:edges].cpu().numpy()
    visited = np.unique(seeds)
    frontier = visited
    alg = 0.0
    for l in range(len(fan)):
        alg += 24.0 * len(frontier) + 12.0 * (o[l + 1] - o[l])
        nxt = np.setdiff1d(np.unique(d_host[o[l]:o[l + 1]]), visited, assume_unique=True)
        visited = np.union1d(visited, nxt)
        frontier = nxt
    for _ in range(args.warmup):
        g.sample(offs, seeds_d, fan, csaw.UNIFORM, **call)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sample(offs, seeds_d, fan, csaw.UNIFORM, **call)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    for _ in range(args.steps):
        g.sample(offs, seeds_d, fan, csaw.UNIFORM, **call)
    torch.cuda.synchronize()
    times = {k: csaw.profile_read(k) for k in ("frontier_init", "select_small", "select_wave", "select_big",
                                                "frontier_build", "visited_clear")}
    csaw.profile_enable(False)
    csaw.profile_reset()
    sel_ms = (times["select_small"][0] + times["select_wave"][0]) / args.steps
    achieved = alg / (sel_ms / 1e3) / 1e9 if sel_ms > 0 else 0.0
    return {
        "metric": "sampled edges/sec (SEPS), forest fire sampling",
        "value": edges / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": "forest_fire_rmat22", "seeds": int(len(seeds)), "burning_probability": 0.7,
                   "depth": 2, "cap": 64, "edges_per_step": int(edges), "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "select_small + select_wave (k_select_small, k_select)",
                     "ms_per_step": sel_ms, "alg_bytes_per_step": alg},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in times.items()},
    }


def bench_metropolis(args):
    """Metropolis-Hastings walks on the symmetrised R-MAT 22 graph: 2^20
    walkers from uniform starts, length 80."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    log("generating symmetrised R-MAT 22 graph")
    rp, col = inputs.rmat_csr(22, 16 << 22, 22, symmetrize=True)
    starts = torch.from_numpy(inputs.walker_starts(rp, col, 1 << 20, 2404)).to("cuda")
    g = csaw.Graph(rp, col)
    paths = torch.empty((1 << 20, 81), dtype=torch.int32, device=g.device)
    for i in range(args.warmup):
        g.walk(starts, 80, csaw.METROPOLIS_HASTINGS, rng_seed=1 + i % 3, paths=paths)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    for i in range(args.steps):
        steps += g.walk(starts, 80, csaw.METROPOLIS_HASTINGS, rng_seed=1 + i % 3, paths=paths)[1]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    _, st = g.walk(starts, 80, csaw.METROPOLIS_HASTINGS, rng_seed=1, paths=paths)
    torch.cuda.synchronize()
    kms, kn = csaw.profile_read("walk")
    csaw.profile_enable(False)
    csaw.profile_reset()
    # per step: v's row offsets (16), the proposal's id (4), its row offsets
    # (16), the path entry (4)
    alg = 40.0 * st
    achieved = alg / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    return {
        "metric": "walk steps/s, Metropolis-Hastings random walk",
        "value": steps / args.steps / dt, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 draws (integer)", "data": "synthetic",
        "config": {"workload": "metropolis_hastings_rmat22_sym", "walkers": 1 << 20, "length": 80},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_walk_uniform<metropolis>",
                     "launches": kn, "avg_launch_us": kms / max(kn, 1) * 1e3, "alg_bytes_per_launch": alg},
    }


def bench_walks(args):
    """Edge-weight walks on the served graph (R-MAT 26, weight = out-degree of
    the destination), resident in HBM with the walk guide built: --walkers
    walkers (default 262,144: one lane each) from uniform starts, length 80,
    Philox seeds cycling 1..3. The roofline is the lane kernel's: algorithmic
    bytes per step (walk_step_bytes) over its event time, and the measured
    HBM bytes per step of the committed counter record."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.SERVED
    scale = args.served_scale or rec["scale"]
    nw, L = args.walkers, 80
    log("generating R-MAT %d graph" % scale)
    rp, col = inputs.graph_for(rec, scale=scale, num_edges=16 << scale)
    ew = inputs.dst_outdeg_weights(rp, col)
    g = csaw.Graph(rp, col, ew)
    starts = torch.from_numpy(inputs.walker_starts(rp, col, nw, 2026)).to(g.device)
    paths = torch.empty((nw, L + 1), dtype=torch.int32, device=g.device)
    t0 = time.perf_counter()
    g.walk(starts[:64], 1, csaw.EDGE_WEIGHT, rng_seed=1)  # builds the walk guide
    torch.cuda.synchronize()
    log("walk guide built in %.1f ms" % ((time.perf_counter() - t0) * 1e3))
    for i in range(args.warmup):
        g.walk(starts, L, csaw.EDGE_WEIGHT, rng_seed=1 + i % 3, paths=paths)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    for i in range(args.steps):
        steps += g.walk(starts, L, csaw.EDGE_WEIGHT, rng_seed=1 + i % 3, paths=paths)[1]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    _, st = g.walk(starts, L, csaw.EDGE_WEIGHT, rng_seed=1, paths=paths)
    torch.cuda.synchronize()
    kms, kn = csaw.profile_read("walk")
    csaw.profile_enable(False)
    csaw.profile_reset()
    alg, wsteps = walk_step_bytes(rp, paths.cpu().numpy())
    achieved = alg / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    per_step = measured_traffic("traffic_walk_lane_rmat26.md", WALK_SOURCES, "hbm_bytes_per_step")
    copy_gbps = measured_copy_gbps()
    line = {
        "metric": "walk steps/s (sampled edges/s), edge-weight random walk",
        "value": steps / args.steps / dt, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": "walks_rmat%d" % scale, "graph": "R-MAT scale %d, edge factor 16, edge weight = "
                   "out-degree of the destination" % scale, "n": len(rp) - 1, "m": len(col), "walkers": nw,
                   "length": L},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": per_step * wsteps / max(kn, 1) if per_step else None,
                     "traffic_GBps": per_step * wsteps / (kms / 1e3) / 1e9 if per_step and kms > 0 else None,
                     "measured_copy_GBps": copy_gbps, "kernel": "k_walk_lane<false>" if nw >= 12288 else
                     "k_walk_wave_first", "launches": kn, "avg_launch_us": kms / max(kn, 1) * 1e3,
                     "alg_bytes_per_launch": alg / max(kn, 1), "steps_per_s": wsteps / (kms / 1e3)},
    }
    if not args.no_cpu_baseline:
        # the oracle on every 64th walker id (ids fix the draws), timed
        import oracle
        idx = np.arange(0, nw, 64)
        st_h = starts.cpu().numpy()[idx]
        t0 = time.perf_counter()
        _, osteps, _ = oracle.walk(rp, col, ew, st_h, L, bias_kind=1, rng_seed=1, walker_ids=idx.astype(np.uint64),
                                   nthreads=1)
        t1 = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": float(osteps.sum()) / t1, "unit": "steps/s", "cores": 1, "kind": "oracle",
                                "sample": "%d walkers (every 64th id) x %d steps, %.1f s on one thread" % (
                                    len(idx), L, t1)}
    return line


def bench_layer(args):
    """Layer sampling on the degree-biased R-MAT 22 graph: 2,000 instances of
    512 sorted seeds, fanouts [64, 64], out-degree bias."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.DEGREE_BIASED
    log("generating R-MAT %d graph" % rec["scale"])
    rp, col = inputs.graph_for(rec)
    g = csaw.Graph(rp, col)
    gen = inputs.rng(8808)
    pool = inputs.non_isolated(rp, col)
    ni, S = 2000, 512
    sets = [np.sort(gen.choice(pool, size=S, replace=False)) for _ in range(ni)]
    offs = np.arange(ni + 1, dtype=np.int64) * S
    seeds = torch.from_numpy(np.concatenate(sets).astype(np.int32)).to(g.device)
    fan = [64, 64]
    # edges per Philox seed (deterministic), counted outside the timed region
    edges_of = {s: int(g.layer_sample(offs, seeds, fan, csaw.NEIGHBOR_DEGREE, rng_seed=s)[2].sum())
                for s in (1, 2, 3)}
    for i in range(args.warmup):
        g.layer_sample(offs, seeds, fan, csaw.NEIGHBOR_DEGREE, rng_seed=1 + i % 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges = 0
    for i in range(args.steps):
        g.layer_sample(offs, seeds, fan, csaw.NEIGHBOR_DEGREE, rng_seed=1 + i % 3)
        edges += edges_of[1 + i % 3]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    g.layer_sample(offs, seeds, fan, csaw.NEIGHBOR_DEGREE, rng_seed=1)
    torch.cuda.synchronize()
    kms, kn = csaw.profile_read("layer_sample")
    csaw.profile_enable(False)
    csaw.profile_reset()
    return {
        "metric": "sampled edges/sec (SEPS), layer sampling",
        "value": edges / args.steps / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": "layer_rmat22", "instances": ni, "seeds": S, "fanouts": fan,
                   "bias": "out-degree of neighbor", "edges_per_step": edges / args.steps},
        "kernel_ms": kms, "kernel": "k_layer_sample",
    }


def bench_mdrw(args):
    """Multi-dimensional random walks at the paper's setting (2,000
    instances, frontier pools of 2,000 vertices, 1,703 sampled edges each) on
    the degree-biased R-MAT 22 graph."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.DEGREE_BIASED
    log("generating R-MAT %d graph" % rec["scale"])
    rp, col = inputs.graph_for(rec)
    g = csaw.Graph(rp, col)
    ni, P, budget = 2000, 2000, 1703
    pool_vertices = inputs.non_isolated(rp, col)
    gen = inputs.rng(7707)
    pool = pool_vertices[gen.integers(0, len(pool_vertices), size=ni * P)].astype(np.int32)
    po = np.arange(ni + 1, dtype=np.int64) * P
    pool_d = torch.from_numpy(pool).to(g.device)
    src = torch.empty((ni, budget), dtype=torch.int32, device=g.device)
    dst = torch.empty_like(src)
    steps = torch.empty(ni, dtype=torch.int64, device=g.device)
    out = (src, dst, steps)
    _, _, _, total = g.mdrw(po, pool_d, budget, rng_seed=1, out=out)
    for i in range(args.warmup):
        g.mdrw(po, pool_d, budget, rng_seed=1 + (i % 3), out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges = 0
    for i in range(args.steps):
        edges += g.mdrw(po, pool_d, budget, rng_seed=1 + (i % 3), out=out)[3]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    g.mdrw(po, pool_d, budget, rng_seed=1, out=out)
    torch.cuda.synchronize()
    kms, kn = csaw.profile_read("mdrw")
    csaw.profile_enable(False)
    csaw.profile_reset()
    # per instance: the pool (4 B id + 16 B row offsets per slot), per step the
    # sampled neighbor id (4), its row offsets (16) and the edge written (8)
    alg = ni * P * 20.0 + total * 28.0
    achieved = alg / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    return {
        "metric": "sampled edges/sec (SEPS), multi-dimensional random walk",
        "value": edges / args.steps / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": "mdrw_rmat22", "instances": ni, "pool": P, "edges_per_instance": budget},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_mdrw", "launches": kn,
                     "avg_launch_us": kms / max(kn, 1) * 1e3, "alg_bytes_per_launch": alg},
    }


def walk_bytes_node2vec(rowptr, paths):
    """Algorithmic bytes of node2vec walks from their paths: a step from v
    with previous vertex t reads v's row offsets (16), N(v) (4 d_v: biases
    and the pick), N(t) (4 d_t: membership) and writes the next vertex (4);
    when N(t) is short (d_t < 64) and N(v) long (d_v >= 2048) the step reads
    N(t) and, for each of its entries and t, the two ends of a binary search
    in N(v) (8 per level, ceil(log2(d_v + 1)) levels) plus the pick's id,
    instead of N(v) whole; the first step (no t) is an unbiased draw:
    offsets, one neighbor id, the write (24)."""
    deg = np.diff(rowptr).astype(np.float64)
    P = paths
    steps = (P[:, 1:] >= 0)
    first = steps[:, 0].sum() * 24.0
    later = steps[:, 1:]
    v = np.where(later, P[:, 1:-1], 0)
    t = np.where(later, P[:, :-2], 0)
    dv, dt = deg[v], deg[t]
    short = (dt < 64) & (dv >= 2048)
    levels = np.ceil(np.log2(dv + 1.0))
    nv = np.where(short, 8.0 * (dt + 1.0) * levels + 4.0, 4.0 * dv)
    rest = ((20.0 + nv + 4.0 * dt) * later).sum()
    return float(first + rest), int(steps.sum())


def bench_node2vec(args):
    """node2vec walks on symmetrised R-MAT 24 (or a smaller scale) with
    weights {1, 2, 4}, length 80; walkers strided over the 2^20 workload."""
    import torch
    from paper_2009_09103_amd import csaw, inputs

    rec = inputs.NODE2VEC
    scale = args.n2v_scale or rec["scale"]
    log("generating symmetrised R-MAT %d graph" % scale)
    rp, col = inputs.graph_for(rec, scale=scale, num_edges=16 << scale)
    g = csaw.Graph(rp, col)
    starts_all = inputs.walker_starts(rp, col, rec["num_walkers"], rec["start_rng"])
    ids = np.arange(0, rec["num_walkers"], args.n2v_stride, dtype=np.uint64)
    starts = torch.from_numpy(starts_all[ids.astype(np.int64)]).to(g.device)
    paths, steps = g.walk(starts, rec["length"], csaw.NODE2VEC, rng_seed=1, node2vec=rec["node2vec"], walker_ids=ids)
    torch.cuda.synchronize()
    alg, nsteps = walk_bytes_node2vec(rp, paths.cpu().numpy())
    assert nsteps == steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, steps = g.walk(starts, rec["length"], csaw.NODE2VEC, rng_seed=1, node2vec=rec["node2vec"],
                          walker_ids=ids, paths=paths)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    csaw.profile_reset()
    csaw.profile_enable(True)
    g.walk(starts, rec["length"], csaw.NODE2VEC, rng_seed=1, node2vec=rec["node2vec"], walker_ids=ids, paths=paths)
    torch.cuda.synchronize()
    kms, kn = csaw.profile_read("walk_node2vec")
    csaw.profile_enable(False)
    csaw.profile_reset()
    achieved = alg / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    return {
        "metric": "sampled edges/sec (walk steps/s), node2vec",
        "value": steps / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bias / u64 prefix (integer)", "data": "synthetic",
        "config": {"workload": rec["name"], "scale": scale, "walkers": int(len(ids)), "length": rec["length"],
                   "node2vec_weights": list(rec["node2vec"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_walk_wave_n2v",
                     "launches": kn, "avg_launch_us": kms / max(kn, 1) * 1e3, "alg_bytes_per_launch": alg},
    }


def measured_copy_gbps(reps=5):
    """Read + write bandwidth of a plain 1 GiB device copy (the measured
    ceiling beside the published 8 TB/s)."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / dt / 1e9


def bench_copy(args):
    """A plain device-to-device copy of 1 GiB (torch), K times: the known
    byte count that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(max(args.warmup, 1)):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    return {"metric": "device copy bandwidth (read + write)", "value": 2 * nbytes / dt / 1e9, "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "copy_1GiB", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes}}


KERNEL_SOURCES = ("paper_2009_09103_amd/csrc/sample_kernels.hip", "paper_2009_09103_amd/csrc/device_common.h",
                  "paper_2009_09103_amd/csrc/kernels.h")
WALK_SOURCES = ("paper_2009_09103_amd/csrc/walk_kernels.hip", "paper_2009_09103_amd/csrc/device_common.h",
                "paper_2009_09103_amd/csrc/kernels.h")


def kernel_source_sha(files=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(record, sources=KERNEL_SOURCES, field="hbm_bytes_per_launch"):
    """HBM bytes per launch (or, with field="hbm_bytes_per_step", per walk
    step) of the dominant kernel from the committed counter summary, or None
    when the kernel sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha(sources)
    fields = {}
    with open(path) as f:
        for ln in f:
            if ":" in ln and ln.startswith("- "):
                k, v = ln[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def main():
    faulthandler.enable()  # a crash prints every thread's Python stack to stderr
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="served")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--qps", type=float, nargs="*", default=None)
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--walkers", type=int, default=1 << 18, help="walks workload: walkers per call")
    ap.add_argument("--passes", type=int, default=5,
                    help="served workload: passes of the trace per QPS point and path; the median is reported")
    ap.add_argument("--served-scale", type=int, default=0)
    ap.add_argument("--n2v-scale", type=int, default=0)
    ap.add_argument("--rounds", type=int, default=0,
                    help="repeated-sampling rounds before the direct draws: 0 (default 8), 1..8, -1 (none)")
    ap.add_argument("--tuning", default="auto",
                    help='sub-wave buckets of the sampling kernel: "auto", "default" or "bound16,bound32"')
    ap.add_argument("--n2v-stride", type=int, default=64)
    ap.add_argument("--partitions", type=int, default=4)
    ap.add_argument("--resident", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true",
                    help="served workload: skip the batched multi-instance summary added to its line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole path on a single MI355X "
              "(instances would shard across GPUs with no exchange); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "degree_biased":
        line = bench_degree_biased(args)
    elif args.workload == "batched":
        line = bench_batched(args)
    elif args.workload == "served":
        line = bench_served(args)
        if not args.no_batched:
            # the batched multi-instance workload (4,096 instances in one call
            # against 4,096 plain calls, and split over concurrent streams),
            # summarised beside the served line
            b = bench_batched(argparse.Namespace(**dict(vars(args), steps=5, warmup=2)))
            line["batched_rmat22"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "config", "roofline",
                                                        "plain_calls", "batched_over_plain", "split_streams_ms")}
    elif args.workload == "streamed":
        line = bench_streamed(args)
    elif args.workload == "node2vec":
        line = bench_node2vec(args)
    elif args.workload == "forest_fire":
        line = bench_forest_fire(args)
    elif args.workload == "metropolis":
        line = bench_metropolis(args)
    elif args.workload == "layer":
        line = bench_layer(args)
    elif args.workload == "mdrw":
        line = bench_mdrw(args)
    elif args.workload == "copy":
        line = bench_copy(args)
    elif args.workload == "walks":
        line = bench_walks(args)
    else:
        print("unknown workload %s" % args.workload, file=sys.stderr)
        sys.exit(2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
