"""Admission and batching logic of the validation server, on the CPU with a
mock executor (simulated time)."""
import numpy as np
import pytest

from paper_2605_03208_amd import serve


def _reqs(n, rate, sizes_n, seed=0, max_k=8):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(1, max_k + 1))
        out.append(serve.Request(i, t, rng.choice(sizes_n, size=k, replace=False), int(rng.integers(0, 9)), i))
    return out


def test_budget_never_exceeded_and_fifo():
    rng = np.random.default_rng(1)
    sizes = rng.integers(1 << 20, 16 << 20, size=64)
    reqs = _reqs(300, 2000.0, len(sizes))
    ex = serve.MockExecutor(sizes, n_streams=3, rate_Bps=2e11)
    budget = 256 << 20
    srv = serve.Server(ex, budget)
    done = srv.run(reqs, real_time=False)
    assert len(done) == len(reqs)
    assert srv.budget.peak <= budget and srv.budget.used == 0
    assert srv.admit_order == sorted(srv.admit_order)          # head-of-line FIFO
    assert sorted(d.rid for d in done) == list(range(len(reqs)))
    for d in done:
        assert d.arrival_s <= d.admit_s <= d.launch_s <= d.done_s
        assert d.results == [dict(rid=d.rid)]


def test_overload_queues_but_completes():
    sizes = np.full(16, 32 << 20)
    reqs = _reqs(200, 1e6, len(sizes), seed=3)    # everything arrives at once
    ex = serve.MockExecutor(sizes, n_streams=2, rate_Bps=1e11)
    srv = serve.Server(ex, 300 << 20)
    done = srv.run(reqs, real_time=False)
    assert len(done) == 200
    q = [d.admit_s - d.arrival_s for d in done]
    assert max(q) > 0                                  # the budget binds
    assert srv.budget.peak <= 300 << 20


def test_batches_span_requests_admitted_together():
    sizes = np.full(8, 1 << 20)
    reqs = [serve.Request(i, 0.0, np.array([i % 8]), 0, i) for i in range(20)]
    ex = serve.MockExecutor(sizes, n_streams=1, rate_Bps=1e9)
    srv = serve.Server(ex, 1 << 30, max_batch=8)
    done = srv.run(reqs, real_time=False)
    launches = sorted({d.launch_s for d in done})
    assert len(launches) == 3                          # 8 + 8 + 4 requests per launch


def test_request_larger_than_budget_is_rejected():
    ex = serve.MockExecutor(np.array([1 << 30]), n_streams=1)
    with pytest.raises(ValueError):
        serve.Server(ex, 1 << 20).run([serve.Request(0, 0.0, np.array([0]), 0, 0)], real_time=False)


def test_summary_fields():
    d = [serve.Completed(i, 0.0, 0.001, 0.001, 0.002 + i * 1e-4, 100) for i in range(100)]
    s = serve.summarize(d, 1.0)
    assert s["requests"] == 100 and s["p50_ms"] <= s["p99_ms"] and s["compared_bytes"] == 20000


def test_summary_wait_and_host_split():
    d = [serve.Completed(i, 0.0, 0.001, 0.003, 0.004, 100, [], 0.0005, 0.0002, 0.0001 * (i % 3)) for i in range(10)]
    s = serve.summarize(d, 1.0)
    assert s["queue_p50_ms"] == 1.0 and s["wait_p50_ms"] == 3.0 and s["wait_p99_ms"] == 3.0
    assert s["host_launch_p99_ms"] <= 0.2 and s["materialize_p50_ms"] == 0.5 and s["compare_p99_ms"] == 0.2


def test_run_pauses_and_restores_the_cycle_collector():
    import gc
    ex = serve.MockExecutor(np.array([100, 200]), n_streams=1)
    reqs = [serve.Request(i, i * 1e-3, np.array([i % 2]), 0, i) for i in range(4)]
    assert gc.isenabled()
    assert len(serve.Server(ex, 1 << 20).run(reqs, real_time=False)) == 4
    assert gc.isenabled()
    gc.disable()
    try:
        serve.Server(serve.MockExecutor(np.array([100, 200]), n_streams=1), 1 << 20).run(reqs, real_time=False)
        assert not gc.isenabled()
    finally:
        gc.enable()


def test_busy_fraction_is_the_union_of_device_intervals():
    """Requests of one batch share its device interval; overlapping batches on
    different streams count once: busy = |[0,2] u [1,3] u [5,6]| = 4 of 10 s."""
    mk = lambda rid, a, b: serve.Completed(rid, 0.0, 0.0, 0.0, 1.0, 1, [], 0.0, 0.0, 0.0, a, b)
    done = [mk(0, 0.0, 2.0), mk(1, 0.0, 2.0), mk(2, 1.0, 3.0), mk(3, 5.0, 6.0)]
    s = serve.summarize(done, 10.0)
    assert s["busy_frac"] == 0.4 and s["requests"] == 4
    assert serve.summarize([mk(0, 2.0, 3.0), mk(1, 2.5, 2.75)], 2.0)["busy_frac"] == 0.5
