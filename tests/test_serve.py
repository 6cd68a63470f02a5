"""Serving: continuous batching, admission, failure paths.

CPU tests drive the server's scheduling with its placeholder executor
(BN_SERVE_FAKE=1): results depend only on the request and each request holds
its slot for a fixed time, so admission, ordering, cancellation and the
allocation-failure path can be checked without a GPU. The GPU tests check
that every served result equals the same problem solved alone (bitwise: the
kernels' reductions run in a fixed order), with and without a tight memory
budget, and agree with the oracle.
"""
import threading
import time

import numpy as np
import pytest

import paper_1408_1664_amd as bn
from paper_1408_1664_amd import datagen


def _problem(n, m=100, seed=0, arity=2):
    return datagen.random_dag_dataset(n, m, arity, 3, 1.0, seed=seed)


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setenv("BN_SERVE_FAKE", "1")
    monkeypatch.setenv("BN_SERVE_FAKE_MS", "30")
    monkeypatch.delenv("BN_SERVE_FAIL_ALLOC", raising=False)
    return monkeypatch


def test_fake_results_and_tickets(fake):
    srv = bn.Server(max_active=4)
    tickets = [(srv.submit(ds.data, ds.arity, 3), ds) for ds in
               (_problem(n, seed=n) for n in range(8, 14))]
    assert len(set(t for t, _ in tickets)) == len(tickets)
    for t, ds in tickets:
        s, post, rep = srv.poll(t, timeout_us=-1)
        assert s == bn.BN_OK
        n = ds.n
        want = np.array([[0.0 if u == v else ((u * 31 + v * 17 + n + ds.m) % 97) / 97.0
                          for v in range(n)] for u in range(n)])
        np.testing.assert_array_equal(post, want)
        assert rep["ms_latency"] >= rep["ms_queue"] >= 0
    # a served ticket is released
    s, _, _ = srv.poll(tickets[0][0])
    assert s == bn.BN_EINVAL
    srv.close()


def _latencies(budget, max_active, k=4):
    ds = _problem(10)
    fp = bn.workspace_bytes(10, 3, ds.m, "fp32") + 10 * 10 * 8 + 10 * ds.m
    srv = bn.Server(mem_budget_bytes=int(budget * fp) if budget else 0, max_active=max_active)
    ts = [srv.submit(ds.data, ds.arity, 3) for _ in range(k)]
    reps = [srv.poll(t, timeout_us=-1)[2] for t in ts]
    srv.close()
    return [r["ms_latency"] for r in reps], [r["ms_queue"] for r in reps]


def test_admission_by_memory_budget(fake):
    # room for one request at a time: the four requests run one after another
    lat, q = _latencies(budget=1.5, max_active=8)
    for a, b in zip(lat, lat[1:]):
        assert b - a > 20.0
    assert q[3] > 60.0
    # room for all: they overlap
    lat, q = _latencies(budget=None, max_active=8)
    assert max(lat) < 2 * 30.0 and max(q) < 15.0


def test_admission_by_slots(fake):
    lat, q = _latencies(budget=None, max_active=2)
    assert max(q[:2]) < 15.0 and min(q[2:]) > 20.0


def test_request_that_never_fits_is_rejected(fake):
    ds = _problem(20)   # about 60 MB of lattice
    srv = bn.Server(mem_budget_bytes=1 << 24, max_active=2)
    with pytest.raises(bn.BnError) as ei:
        srv.submit(ds.data, ds.arity, 3)
    assert ei.value.status == bn.BN_ENOMEM
    srv.close()


def test_invalid_request_rejected_at_submit(fake):
    ds = _problem(8)
    bad = ds.data.copy()
    bad[3, 5] = 7
    srv = bn.Server(max_active=2)
    with pytest.raises(bn.BnError) as ei:
        srv.submit(bad, ds.arity, 3)
    assert ei.value.status == bn.BN_EINVAL
    srv.close()


def test_poll_states(fake):
    ds = _problem(9)
    srv = bn.Server(max_active=1)
    t = srv.submit(ds.data, ds.arity, 2)
    assert srv.poll(t, timeout_us=0)[0] == bn.BN_EAGAIN
    assert srv.poll(t, timeout_us=-1)[0] == bn.BN_OK
    assert srv.poll(12345, timeout_us=0)[0] == bn.BN_EINVAL
    srv.close()


def test_destroy_cancels_pending_and_wakes_pollers(fake):
    ds = _problem(10)
    fp = bn.workspace_bytes(10, 3, ds.m, "fp32") + 10 * 10 * 8 + 10 * ds.m
    srv = bn.Server(mem_budget_bytes=int(1.5 * fp), max_active=1)
    ts = [srv.submit(ds.data, ds.arity, 3) for _ in range(5)]
    got = {}

    def waiter():
        got["s"] = srv.poll(ts[-1], timeout_us=-1)[0]

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.01)
    srv.close()          # the first request is on the device, four are queued
    th.join(timeout=10)
    assert not th.is_alive()
    assert got["s"] == bn.BN_ECANCELED


def test_injected_allocation_failure(fake):
    fake.setenv("BN_SERVE_FAIL_ALLOC", "2")
    srv = bn.Server(max_active=1)
    ts = [srv.submit(ds.data, ds.arity, 3) for ds in (_problem(9, seed=s) for s in range(3))]
    st = [srv.poll(t, timeout_us=-1)[0] for t in ts]
    assert st == [bn.BN_OK, bn.BN_ENOMEM, bn.BN_OK]
    srv.close()


def test_allocation_failure_while_others_run_is_retried(fake):
    # the second request's allocation fails while the first holds the device:
    # it goes back to the head of the queue and runs once the first completes
    fake.setenv("BN_SERVE_FAIL_ALLOC", "2")
    srv = bn.Server(max_active=2)
    ts = [srv.submit(ds.data, ds.arity, 3) for ds in (_problem(9, seed=s) for s in range(3))]
    out = [srv.poll(t, timeout_us=-1) for t in ts]
    assert [o[0] for o in out] == [bn.BN_OK, bn.BN_OK, bn.BN_OK]
    # it waited for the first request to finish (30 ms each)
    assert out[1][2]["ms_queue"] > 20.0
    srv.close()


# ------------------------------------------------------------------ GPU

def _mix(k=16):
    rng = np.random.default_rng(44)
    out = []
    for j in range(k):
        n = int(rng.integers(10, 17))
        m = int(rng.integers(100, 800))
        r = int(rng.integers(2, 4))
        out.append((datagen.random_dag_dataset(n, m, r, 3, 1.0, seed=500 + j),
                    "fp32" if j % 3 else "fp64"))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("tight", [False, True])
def test_served_equals_alone(tight, monkeypatch):
    monkeypatch.delenv("BN_SERVE_FAKE", raising=False)
    monkeypatch.delenv("BN_SERVE_FAIL_ALLOC", raising=False)
    mix = _mix()
    budget = 0
    if tight:   # room for about two of the largest requests at a time
        budget = 2 * max(bn.workspace_bytes(ds.n, 3, ds.m, "fp64") + ds.n * ds.m + 8 * ds.n ** 2
                         for ds, _ in mix) + (1 << 20)
    srv = bn.Server(mem_budget_bytes=budget, max_active=8)
    ts = [srv.submit(ds.data, ds.arity, 3, precision=pr) for ds, pr in mix]
    for (ds, pr), t in zip(mix, ts):
        s, post, rep = srv.poll(t, timeout_us=-1)
        assert s == bn.BN_OK
        alone, rep1 = bn.edge_posteriors(ds.data, ds.arity, 3, precision=pr)
        assert np.array_equal(post, alone)
        assert rep["log_LV"] == rep1["log_LV"]
    srv.close()


@pytest.mark.gpu
def test_served_equals_alone_on_the_serving_stream(monkeypatch):
    """The first 64 requests of the benchmark's serving stream (n in 10..22,
    m in 100..2000, arity 2 or 3, d = 3, FP32-scaled), submitted at once so
    that up to 16 overlap on the device: each result equals the same problem
    solved alone, bit for bit."""
    monkeypatch.delenv("BN_SERVE_FAKE", raising=False)
    monkeypatch.delenv("BN_SERVE_FAIL_ALLOC", raising=False)
    reqs = datagen.serving_stream(64, seed=4)
    data = [datagen.request_dataset(r) for r in reqs]
    assert max(r["n"] for r in reqs) >= 20 and max(r["m"] for r in reqs) >= 1500
    srv = bn.Server(max_active=16)
    ts = [srv.submit(ds.data, ds.arity, r["d"], precision="fp32", ess=r["ess"])
          for ds, r in zip(data, reqs)]
    for ds, r, t in zip(data, reqs, ts):
        s, post, rep = srv.poll(t, timeout_us=-1)
        assert s == bn.BN_OK
        alone, rep1 = bn.edge_posteriors(ds.data, ds.arity, r["d"], precision="fp32",
                                         ess=r["ess"])
        assert np.array_equal(post, alone), (r["idx"], r["n"], r["m"])
        assert rep["log_LV"] == rep1["log_LV"]
    srv.close()


@pytest.mark.gpu
def test_served_matches_oracle():
    from oracle import oracle as O
    srv = bn.Server(max_active=4)
    cases = [datagen.random_dag_dataset(n, 300, 2, 3, 1.0, seed=60 + n) for n in (10, 13, 15)]
    ts = [srv.submit(ds.data, ds.arity, 3, precision="fp32") for ds in cases]
    for ds, t in zip(cases, ts):
        s, post, _ = srv.poll(t, timeout_us=-1)
        assert s == bn.BN_OK
        ref = O.edge_posteriors(ds.data, ds.arity, 3)
        assert np.abs(post - ref["post"]).max() <= 1e-5
    srv.close()
