"""The request server: continuous batching over a resident graph. Every
request's result equals the same request run alone (and the oracle), in a
mix, under a tight memory budget and with several executor streams;
cancellation and the server's fixed device memory."""
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
def setup():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_09103_amd import csaw
    rp, col = inputs.rmat_csr(15, 16 << 15, 31)
    ew = inputs.dst_outdeg_weights(rp, col)
    g = csaw.Graph(rp, col, ew)
    trace = inputs.request_trace(rp, col, 60, qps=1000.0, trace_rng=7)
    for r in trace:   # smaller than the served workload, same mix
        if r["kind"] == "sample":
            r["seeds"] = r["seeds"][:300]
        else:
            r["starts"] = r["starts"][:2000]
    return csaw, rp, col, ew, g, trace


def submit(srv, r):
    if r["kind"] == "sample":
        return srv.submit_sample(r["seeds"], r["fanouts"], r["bias"], rng_seed=r["rng_seed"], request_id=r["id"])
    return srv.submit_walk(r["starts"], r["length"], r["bias"], rng_seed=r["rng_seed"], request_id=r["id"])


def check_alone(csaw, g, rp, col, ew, r, res, with_oracle):
    assert res.status == 0
    if r["kind"] == "sample":
        alone = g.sample(np.array([0, len(r["seeds"])]), r["seeds"], r["fanouts"], r["bias"],
                         rng_seed=r["rng_seed"], instance_base=r["id"])
        np.testing.assert_array_equal(res.src, alone.src.cpu().numpy())
        np.testing.assert_array_equal(res.dst, alone.dst.cpu().numpy())
        np.testing.assert_array_equal(res.layer_offsets, alone.offsets.cpu().numpy())
        if with_oracle:
            ref = oracle.sample(rp, col, ew, np.array([0, len(r["seeds"])]), r["seeds"], r["fanouts"],
                                bias_kind=r["bias"], rng_seed=r["rng_seed"], instance_base=r["id"])
            np.testing.assert_array_equal(res.dst, ref.dst)
    else:
        paths, steps = g.walk(r["starts"], r["length"], r["bias"], rng_seed=r["rng_seed"], walker_base=r["id"])
        np.testing.assert_array_equal(res.paths, paths.cpu().numpy())
        assert res.steps == steps
        if with_oracle:
            ref, _, _ = oracle.walk(rp, col, ew, r["starts"], r["length"], bias_kind=r["bias"],
                                    rng_seed=r["rng_seed"], walker_base=r["id"])
            np.testing.assert_array_equal(res.paths, ref)


@pytest.mark.parametrize("streams,budget,pool", [(2, 1 << 30, 0), (3, 24 << 20, 0), (1, 1 << 30, 0),
                                                 (2, 1 << 30, 8 << 20)])
def test_mix_equals_alone(setup, streams, budget, pool):
    """pool: a result pool too small for every result (the rest from the heap)."""
    csaw, rp, col, ew, g, trace = setup
    say("server streams=%d budget=%d pool=%d, %d requests" % (streams, budget, pool, len(trace)))
    srv = csaw.Server(g, memory_budget_bytes=budget, num_streams=streams, max_batch=64, result_pool_bytes=pool)
    dev_bytes, pinned = srv.memory()
    assert budget - 256 * streams < dev_bytes <= budget and pinned > 0
    tickets = [submit(srv, r) for r in trace]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, res) in enumerate(zip(trace, results)):
        check_alone(csaw, g, rp, col, ew, r, res, with_oracle=(k % 10 == 0))
        assert res.total_us >= res.queued_us >= 0


def test_submit_errors_and_poll(setup):
    csaw, rp, col, ew, g, trace = setup
    say("server errors")
    srv = csaw.Server(g, memory_budget_bytes=1 << 20, num_streams=1)
    with pytest.raises(csaw.CsawError) as ei:
        srv.submit_sample(np.array([len(rp) + 5], dtype=np.int32), [5])        # vertex out of range
    assert ei.value.status == 1
    with pytest.raises(csaw.CsawError) as ei:
        srv.submit_walk(np.zeros(1 << 20, dtype=np.int32), 80)                  # alone exceeds the budget
    assert ei.value.status == 2
    walk = next(r for r in trace if r["kind"] == "walk")
    t = srv.submit_walk(walk["starts"][:10], 5, 1, rng_seed=3, request_id=9)
    res = srv.wait(t)
    assert res.status == 0 and res.paths.shape == (10, 6)
    with pytest.raises(csaw.CsawError):
        srv.poll(t)                                                              # already handed over
    srv.close()


def test_queue_full_reports_busy(setup):
    csaw, rp, col, ew, g, trace = setup
    say("server busy")
    srv = csaw.Server(g, num_streams=1, queue_capacity=2, memory_budget_bytes=1 << 30)
    starts = inputs.walker_starts(rp, col, 20000, 1)
    tickets, busy = [], 0
    for i in range(50):
        try:
            tickets.append(srv.submit_walk(starts, 60, 1, rng_seed=i, request_id=i))
        except csaw.CsawError as e:
            assert e.status == 4
            busy += 1
    assert busy > 0
    for t in tickets:
        assert srv.wait(t).status == 0
    srv.close()


def test_cancel_queued_requests(setup):
    csaw, rp, col, ew, g, trace = setup
    say("server cancel")
    srv = csaw.Server(g, num_streams=1, memory_budget_bytes=1 << 30)
    starts = inputs.walker_starts(rp, col, 20000, 2)
    tickets = [srv.submit_walk(starts, 80, 1, rng_seed=i, request_id=i) for i in range(8)]
    cancelled = [t for t in tickets[4:] if srv.cancel(t)]
    assert cancelled, "requests queued behind long walks can be cancelled"
    for t in tickets:
        res = srv.wait(t)
        if t in cancelled:
            assert res.status == 7  # CANCELLED
        else:
            assert res.status == 0 and res.paths.shape == (20000, 81)
    with pytest.raises(csaw.CsawError):
        srv.cancel(1 << 40)  # unknown ticket
    srv.close()


def test_walks_share_launches(setup):
    """Walk requests queued behind a running one are served by one launch per
    bias kind; each result is still the request alone (and the oracle)."""
    csaw, rp, col, ew, g, trace = setup
    say("server walk batching")
    srv = csaw.Server(g, num_streams=1, memory_budget_bytes=1 << 30, max_batch=64)
    busy = srv.submit_walk(inputs.walker_starts(rp, col, 40000, 5), 80, 1, rng_seed=1, request_id=1)
    reqs = []
    for i in range(12):
        r = dict(kind="walk", id=100 + i, rng_seed=7 * i + 3, bias=1 + (i % 2),
                 starts=inputs.walker_starts(rp, col, 300 + 250 * i, 20 + i), length=5 + 6 * i)
        reqs.append(r)
    tickets = [submit(srv, r) for r in reqs]
    assert srv.wait(busy).status == 0
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, res) in enumerate(zip(reqs, results)):
        check_alone(csaw, g, rp, col, ew, r, res, with_oracle=(k % 4 == 0))
    assert max(res.batch_requests for res in results) > 1, [res.batch_requests for res in results]
    assert all(1 <= res.batch_requests <= 6 for res in results)  # six requests of each bias kind


def test_walk_batch_one_lane_per_walker(setup):
    """A walk batch of several requests runs one lane per walker, with the
    lanes of one wavefront in different requests (their own keys, lengths,
    path rows and step counters); each result equals the request alone and,
    for some, the oracle."""
    csaw, rp, col, ew, g, trace = setup
    say("server walk batch above the lane threshold")
    srv = csaw.Server(g, num_streams=1, memory_budget_bytes=1 << 30, max_batch=64)
    busy = srv.submit_walk(inputs.walker_starts(rp, col, 200000, 6), 80, 2, rng_seed=2, request_id=1)
    reqs = [dict(kind="walk", id=200 + i, rng_seed=11 * i + 1, bias=1, length=7 + 9 * i,
                 starts=inputs.walker_starts(rp, col, 17000 + 333 * i, 40 + i)) for i in range(8)]
    tickets = [submit(srv, r) for r in reqs]
    assert srv.wait(busy).status == 0
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (r, res) in enumerate(zip(reqs, results)):
        check_alone(csaw, g, rp, col, ew, r, res, with_oracle=(k % 3 == 0))
    assert max(res.batch_requests for res in results) >= 2, [res.batch_requests for res in results]
