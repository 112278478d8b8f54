"""Serving loop on the CPU: the scheduler driven by an executor that merges
with the oracle in worker threads (no GPU).  Covers admission by budget,
arrival order, over-budget refusal, failure handling, cancellation,
continuous batching with overlapping batches, and latency statistics."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1303_4312_amd import serve, workloads


class CpuExecutor:
    """Each batch runs in its own thread after `delay` seconds (or when
    `gate` is set).  Failures can be injected at launch or at completion."""

    def __init__(self, delay=0.0, raise_on_launch=(), fail_on_done=(), gate=None):
        self.delay = delay
        self.raise_on_launch = set(raise_on_launch)
        self.fail_on_done = set(fail_on_done)
        self.gate = gate
        self.launched = 0
        self.running = 0
        self.max_running = 0
        self.lock = threading.Lock()
        self.order = []

    @staticmethod
    def footprint(A, B, A_val, B_val):
        per = A.itemsize + (4 if A_val is not None else 0)
        return 2 * (len(A) + len(B)) * per

    def launch(self, batch):
        idx = self.launched
        self.launched += 1
        if idx in self.raise_on_launch:
            raise RuntimeError(f"launch {idx} failed")
        self.order.extend(r.rid for r in batch)
        done = threading.Event()
        box = {}

        def run():
            with self.lock:
                self.running += 1
                self.max_running = max(self.max_running, self.running)
            if self.gate is not None:
                self.gate.wait(10)
            time.sleep(self.delay)
            box["out"] = [oracle.stable_merge(r.A, r.B, r.A_val, r.B_val) if r.A_val is not None
                          else oracle.stable_merge(r.A, r.B) for r in batch]
            with self.lock:
                self.running -= 1
            done.set()

        threading.Thread(target=run, daemon=True).start()
        return (done, box, idx)

    def done(self, handle):
        return handle[0].is_set()

    def results(self, handle):
        if handle[2] in self.fail_on_done:
            raise RuntimeError(f"batch {handle[2]} failed on the device")
        return handle[1]["out"]


def make_requests(count, seed=0, lo=1, hi=3000):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        m, n = (int(x) for x in workloads.log_uniform_lengths(rng, 2, lo, hi))
        A = np.sort(rng.integers(0, 50, m)).astype(np.uint32)
        B = np.sort(rng.integers(0, 50, n)).astype(np.uint32)
        reqs.append((A, B) + workloads.origin_payloads(m, n))
    return reqs


def expect(req):
    A, B, Av, Bv = req
    return oracle.stable_merge(A, B, Av, Bv)


def test_every_request_completes_exactly():
    reqs = make_requests(60)
    with serve.Server(CpuExecutor(delay=0.002), budget_bytes=1 << 30, max_batch=8) as srv:
        futs = [srv.submit(A, B, Av, Bv) for A, B, Av, Bv in reqs]
        outs = [f.result(timeout=30) for f in futs]
    for req, (C, Cv) in zip(reqs, outs):
        Ce, Cve = expect(req)
        assert np.array_equal(C, Ce) and np.array_equal(Cv, Cve)
    st = srv.stats()
    assert st["completed"] == 60 and st["failed"] == 0
    assert st["p50_s"] is not None and st["p99_s"] >= st["p50_s"]
    assert srv.budget.used == 0


def test_budget_limits_admission_and_keeps_order():
    reqs = make_requests(30, seed=1, lo=1000, hi=1000)  # equal sizes
    ex = CpuExecutor(delay=0.003)
    one = ex.footprint(reqs[0][0], reqs[0][1], reqs[0][2], reqs[0][3])
    srv = serve.Server(ex, budget_bytes=2 * one, max_batch=8)
    with srv:
        futs = [srv.submit(*r[:2], *r[2:]) for r in reqs]
        for f in futs:
            f.result(timeout=30)
    assert srv.budget.peak <= 2 * one
    assert srv.budget.used == 0
    assert ex.order == sorted(ex.order)  # admitted and launched in arrival order
    assert max(srv.batch_sizes) <= 2


def test_request_larger_than_budget_is_refused():
    big = make_requests(1, seed=2, lo=5000, hi=5000)[0]
    small = make_requests(5, seed=3, lo=10, hi=100)
    ex = CpuExecutor()
    srv = serve.Server(ex, budget_bytes=ex.footprint(*big[:2], big[2], big[3]) - 1)
    with srv:
        f_big = srv.submit(*big[:2], *big[2:])
        f_small = [srv.submit(*r[:2], *r[2:]) for r in small]
        with pytest.raises(serve.BudgetError):
            f_big.result(timeout=30)
        for f, r in zip(f_small, small):
            assert np.array_equal(f.result(timeout=30)[1], expect(r)[1])
    assert srv.stats()["rejected"] == 1


def test_failed_launch_fails_its_batch_and_frees_budget():
    reqs = make_requests(12, seed=4)
    ex = CpuExecutor(delay=0.001, raise_on_launch={0}, fail_on_done={2})
    srv = serve.Server(ex, budget_bytes=1 << 30, max_batch=3, max_inflight=1)
    with srv:
        futs = [srv.submit(*r[:2], *r[2:]) for r in reqs]
        results = []
        for f in futs:
            try:
                results.append(f.result(timeout=30))
            except RuntimeError:
                results.append(None)
    assert srv.budget.used == 0
    assert any(r is None for r in results) and any(r is not None for r in results)
    for req, out in zip(reqs, results):
        if out is not None:
            assert np.array_equal(out[1], expect(req)[1])
    st = srv.stats()
    assert st["failed"] == sum(r is None for r in results)
    assert st["completed"] + st["failed"] == len(reqs)


def test_cancelled_request_never_runs():
    gate = threading.Event()
    reqs = make_requests(6, seed=5, lo=500, hi=500)
    ex = CpuExecutor(gate=gate)
    one = ex.footprint(reqs[0][0], reqs[0][1], reqs[0][2], reqs[0][3])
    srv = serve.Server(ex, budget_bytes=one, max_batch=1, max_inflight=1)
    with srv:
        futs = [srv.submit(*r[:2], *r[2:]) for r in reqs]
        time.sleep(0.05)  # the first request holds the whole budget behind the gate
        assert futs[3].cancel()
        gate.set()
        for k, f in enumerate(futs):
            if k != 3:
                f.result(timeout=30)
    assert 3 not in ex.order
    assert srv.budget.used == 0


def test_requests_arriving_during_a_batch_join_later_batches():
    reqs = make_requests(40, seed=6)
    ex = CpuExecutor(delay=0.02)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_batch=64, max_inflight=2)
    with srv:
        futs = []
        for r in reqs:
            futs.append(srv.submit(*r[:2], *r[2:]))
            time.sleep(0.001)
        for f in futs:
            f.result(timeout=30)
    st = srv.stats()
    assert st["batches"] >= 2
    assert st["mean_batch"] > 1  # arrivals during a running batch were batched together
    assert ex.max_running == 2 and st["max_concurrent_batches"] == 2


def test_stop_drains_and_refuses_double_start():
    reqs = make_requests(5, seed=7)
    srv = serve.Server(CpuExecutor(delay=0.005), budget_bytes=1 << 30).start()
    futs = [srv.submit(*r[:2], *r[2:]) for r in reqs]
    with pytest.raises(RuntimeError):
        srv.start()
    srv.stop()
    assert all(f.done() and not f.exception() for f in futs)


def test_budget_accounting_errors():
    b = serve.Budget(100)
    assert b.try_reserve(60) and not b.try_reserve(50)
    b.release(60)
    with pytest.raises(RuntimeError):
        b.release(1)
    with pytest.raises(ValueError):
        serve.Budget(0)

