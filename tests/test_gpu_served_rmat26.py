"""The request server on the served workload's graph: R-MAT 26 (67M vertices,
about 1.06e9 edges, 4.2 GB of column ids and as much of edge weights, edge
weights = out-degree of the destination), with requests of the served mix,
and one batch of 320 sampling requests whose instance bitmaps take 5.4 GB
(more than 2^32 bytes, indexed past 2^30 words). Every request's result
equals the same request run alone; a subset is checked against the oracle
(sampling whole, walks on every 16th walker id, an exact subset since each
walker's draws are keyed by its own id). The walks workload's own launch on
this graph (262,144 edge-weight walkers of length 80, one lane each) and a
launch of 4,096 walkers (a wavefront each) are checked against the oracle on
strided walker ids, with every step of every 8th walker an edge of positive
weight."""
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
def served():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_09103_amd import csaw
    rec = inputs.SERVED
    say("R-MAT 26 graph")
    rp, col = inputs.graph_for(rec)
    ew = inputs.dst_outdeg_weights(rp, col)
    g = csaw.Graph(rp, col, ew)
    trace = inputs.request_trace(rp, col, 24, 1000.0, 2606, rec["sample_fraction"])
    for r in trace:  # the served mix, requests capped so that the oracle check stays short
        if r["kind"] == "sample":
            r["seeds"] = r["seeds"][:2048]
        else:
            r["starts"] = r["starts"][:8192]
    return csaw, rp, col, ew, g, trace


def check_sample(csaw, g, rp, col, ew, r, res, with_oracle):
    assert res.status == 0
    offs = np.array([0, len(r["seeds"])], dtype=np.int64)
    alone = g.sample(offs, r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"], instance_base=r["id"])
    np.testing.assert_array_equal(res.src, alone.src.cpu().numpy())
    np.testing.assert_array_equal(res.dst, alone.dst.cpu().numpy())
    np.testing.assert_array_equal(res.layer_offsets, alone.offsets.cpu().numpy())
    if with_oracle:
        ref = oracle.sample(rp, col, ew, offs, r["seeds"], r["fanouts"], bias_kind=r["bias"],
                            rng_seed=r["rng_seed"], instance_base=r["id"])
        np.testing.assert_array_equal(res.dst, ref.dst)
        np.testing.assert_array_equal(res.src, ref.src)


def test_batch_with_bitmaps_over_4_gib(served):
    csaw, rp, col, ew, g, trace = served
    n = len(rp) - 1
    nreq = 320
    nwp = ((n + 31) // 32 + 3) // 4 * 4
    assert 2 * nreq * nwp * 4 > (1 << 32)
    gen = inputs.rng(2626)
    pool = inputs.non_isolated(rp, col)
    reqs = [dict(id=10_000 + i, rng_seed=i + 1, seeds=inputs.distinct_seeds(gen, pool, 64),
                 fanouts=[10, 5], bias=i % 3) for i in range(nreq)]
    say("one executor: a long walk, then %d sampling requests that queue behind it" % nreq)
    srv = csaw.Server(g, num_streams=1, max_batch=512, memory_budget_bytes=12 << 30)
    walk = srv.submit_walk(inputs.walker_starts(rp, col, 65536, 26), 80, 1, rng_seed=5, request_id=1)
    tickets = [srv.submit_sample(r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"], request_id=r["id"])
               for r in reqs]
    w = srv.poll(walk)
    # while the walk runs every sampling request waits, and the next batch takes
    # all of them (their exact need, about 5.5 GB, fits the 12 GiB block)
    say("walk still running after the submissions: %s" % (w is None))
    if w is None:
        w = srv.wait(walk)
    assert w.status == 0
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, res) in enumerate(zip(reqs, results)):
        check_sample(csaw, g, rp, col, ew, r, res, with_oracle=(k % 40 == 0))


def test_served_rmat26_mix_equals_alone_and_oracle(served):
    csaw, rp, col, ew, g, trace = served
    say("served %d requests, 3 executors" % len(trace))
    srv = csaw.Server(g, num_streams=3, max_batch=256, memory_budget_bytes=24 << 30)
    tickets = []
    for r in trace:
        if r["kind"] == "sample":
            tickets.append(srv.submit_sample(r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"],
                                             request_id=r["id"]))
        else:
            tickets.append(srv.submit_walk(r["starts"], r["length"], r["bias"], rng_seed=r["rng_seed"],
                                           request_id=r["id"]))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, res) in enumerate(zip(trace, results)):
        say("request %d (%s)" % (k, r["kind"]))
        assert res.status == 0
        if r["kind"] == "sample":
            offs = np.array([0, len(r["seeds"])], dtype=np.int64)
            alone = g.sample(offs, r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"],
                             instance_base=r["id"])
            np.testing.assert_array_equal(res.src, alone.src.cpu().numpy())
            np.testing.assert_array_equal(res.dst, alone.dst.cpu().numpy())
            np.testing.assert_array_equal(res.layer_offsets, alone.offsets.cpu().numpy())
            if k % 3 == 0:
                ref = oracle.sample(rp, col, ew, offs, r["seeds"], r["fanouts"], bias_kind=r["bias"],
                                    rng_seed=r["rng_seed"], instance_base=r["id"])
                np.testing.assert_array_equal(res.dst, ref.dst)
                np.testing.assert_array_equal(res.src, ref.src)
        else:
            paths, steps = g.walk(r["starts"], r["length"], r["bias"], rng_seed=r["rng_seed"],
                                  walker_base=r["id"])
            np.testing.assert_array_equal(res.paths, paths.cpu().numpy())
            assert res.steps == steps
            if k % 3 == 0:
                sub = np.arange(0, len(r["starts"]), 16)
                ref, _, _ = oracle.walk(rp, col, ew, r["starts"][sub], r["length"], bias_kind=r["bias"],
                                        rng_seed=r["rng_seed"], walker_ids=r["id"] + sub.astype(np.uint64))
                np.testing.assert_array_equal(res.paths[sub], ref)


def check_steps_are_edges(rp, col, ew, paths):
    """Every consecutive pair (u, v) of a path is an edge of positive weight
    (vectorised lower bound of v in N(u)), and a path that stops early stops
    at a vertex whose list has no positive weight."""
    u = paths[:, :-1].reshape(-1).astype(np.int64)
    v = paths[:, 1:].reshape(-1)
    keep = v >= 0
    u, v = u[keep], v[keep]
    assert np.all(u >= 0)
    lo, hi = rp[u].copy(), rp[u + 1].copy()
    end = hi.copy()
    while True:
        open_ = lo < hi
        if not open_.any():
            break
        mid = (lo + hi) // 2
        below = col[np.minimum(mid, len(col) - 1)] < v
        lo = np.where(open_ & below, mid + 1, lo)
        hi = np.where(open_ & ~below, mid, hi)
    assert np.all(lo < end)
    np.testing.assert_array_equal(col[lo], v)
    assert np.all(ew[lo] > 0)
    stopped = (paths[:, -1] < 0) & (paths[:, 0] >= 0)
    last = (paths[stopped] >= 0).sum(axis=1) - 1
    for x in np.unique(paths[stopped][np.arange(len(last)), last]):
        assert int(ew[rp[x]:rp[x + 1]].astype(np.uint64).sum()) == 0


@pytest.mark.parametrize("num_walkers,stride", [(262144, 256), (4096, 8)])
def test_walks_workload_against_oracle(served, num_walkers, stride):
    csaw, rp, col, ew, g, _ = served
    length = 80
    starts = inputs.walker_starts(rp, col, num_walkers, 2026)
    say("%d edge-weight walkers of length %d, Philox seed 1" % (num_walkers, length))
    paths, steps = g.walk(starts, length, csaw.EDGE_WEIGHT, rng_seed=1)
    paths = paths.cpu().numpy()
    assert 0 < steps <= num_walkers * length
    sub = np.arange(0, num_walkers, stride)
    say("oracle on %d walkers" % len(sub))
    ref, _, _ = oracle.walk(rp, col, ew, starts[sub], length, bias_kind=oracle.EDGE_WEIGHT, rng_seed=1,
                            walker_ids=sub.astype(np.uint64))
    np.testing.assert_array_equal(paths[sub], ref)
    say("steps of every 8th walker")
    check_steps_are_edges(rp, col, ew, paths[::8])
