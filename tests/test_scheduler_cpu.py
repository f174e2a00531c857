"""The serving scheduler (admission, memory budget, slots, batching, latency
statistics) on a simulated device: the same scheduling core the GPU server
runs, driven in virtual time, so these checks need no GPU."""
import numpy as np
import pytest

from paper_2310_08528_amd import g4d

MB = 1 << 20


def _trace(n=400, rate=200.0, seed=0, classes=3):
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
    cls = rng.integers(classes, size=n).astype(np.int32)
    service = np.array([2e-3, 4e-3, 8e-3])[cls % 3]
    nbytes = np.array([120, 300, 900])[cls % 3] * MB
    shape = (cls == 2).astype(np.int32)       # two shape classes
    return arrival, service, nbytes, cls, shape


def test_budget_slots_fifo_and_completion():
    arrival, service, nbytes, cls, shape = _trace()
    budget, slots = 2048 * MB, 6
    r = g4d.simulate(arrival, service, nbytes, cls, shape, budget, slots, overlap=0.6)
    assert r["rejected"] == 0
    assert (r["latency_ms"] >= 0).all()                      # every request completes (no starvation)
    assert r["peak_bytes"] <= budget                         # the budget is never exceeded
    assert 1 < r["max_in_flight"] <= slots                   # overlap happens, within the slots
    assert list(r["admit_order"]) == list(range(len(arrival)))   # strict FIFO admission
    # latency >= service time alone
    assert (r["latency_ms"] >= 1e3 * service * (1 - 1e-9)).all()


def test_percentiles_match_numpy():
    arrival, service, nbytes, cls, shape = _trace(n=1000, seed=3)
    r = g4d.simulate(arrival, service, nbytes, cls, shape, 4096 * MB, 8, overlap=0.3)
    lat = r["latency_ms"]
    assert r["p50_ms"] == pytest.approx(np.percentile(lat, 50), rel=1e-12)
    assert r["p99_ms"] == pytest.approx(np.percentile(lat, 99), rel=1e-12)
    assert r["mean_ms"] == pytest.approx(lat.mean(), rel=1e-12)
    assert r["max_ms"] == pytest.approx(lat.max(), rel=1e-12)


def test_small_budget_makes_requests_wait_not_fail():
    arrival, service, nbytes, cls, shape = _trace(n=300, seed=1)
    big = g4d.simulate(arrival, service, nbytes, cls, shape, 8192 * MB, 8, overlap=0.6)
    small = g4d.simulate(arrival, service, nbytes, cls, shape, 1000 * MB, 8, overlap=0.6)
    assert small["rejected"] == 0 and (small["latency_ms"] >= 0).all()
    assert small["peak_bytes"] <= 1000 * MB
    assert small["max_in_flight"] < big["max_in_flight"]
    assert small["p99_ms"] > big["p99_ms"]


def test_request_larger_than_budget_is_rejected_alone():
    arrival, service, nbytes, cls, shape = _trace(n=50, seed=2)
    nbytes = nbytes.copy()
    nbytes[10] = 10_000 * MB
    r = g4d.simulate(arrival, service, nbytes, cls, shape, 2048 * MB, 4)
    assert r["rejected"] == 1 and r["latency_ms"][10] == -1.0
    assert (np.delete(r["latency_ms"], 10) >= 0).all()


def test_one_slot_is_the_plain_one_at_a_time_path():
    arrival, service, nbytes, cls, shape = _trace(n=200, seed=4, rate=50.0)
    r = g4d.simulate(arrival, service, nbytes, cls, shape, 4096 * MB, 1, batch_deform=False, overlap=1.0)
    assert r["max_in_flight"] == 1
    # one at a time in arrival order: completion = max(arrival, previous completion) + service
    t, done = 0.0, []
    for a, s in zip(arrival, service):
        t = max(t, a) + s
        done.append(t)
    np.testing.assert_allclose(r["latency_ms"], 1e3 * (np.array(done) - arrival), rtol=1e-9, atol=1e-9)
    assert r["batched_launches"] == len(arrival)             # one deform launch per request


def test_batching_groups_admissions_by_shape_class():
    # a burst of simultaneous arrivals of one shape class: one launch per 8 jobs
    n = 24
    arrival = np.zeros(n)
    r = g4d.simulate(arrival, np.full(n, 1e-3), np.full(n, MB), np.zeros(n, np.int32), np.zeros(n, np.int32),
                     1024 * MB, 32, batch_deform=True)
    assert r["batched_launches"] == 3
    r = g4d.simulate(arrival, np.full(n, 1e-3), np.full(n, MB), np.zeros(n, np.int32), np.zeros(n, np.int32),
                     1024 * MB, 32, batch_deform=False)
    assert r["batched_launches"] == n


def test_buffer_sets_are_reused_by_the_same_class():
    arrival, service, nbytes, cls, shape = _trace(n=200, seed=5)
    r = g4d.simulate(arrival, service, nbytes, cls, shape, 8192 * MB, 4)
    assert r["buffer_reuses"] > 150
