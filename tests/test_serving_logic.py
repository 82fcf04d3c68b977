"""Scheduler logic of the serving loop on the CPU (fake executor, fake clock):
admission by memory budget, FIFO back-pressure, continuous batching,
rejections, per-request device failures and latency accounting."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2411_09859_amd import inputs
from paper_2411_09859_amd.serving import FakeExecutor, Request, Server, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def drive(server, clock, reqs, dt=1e-3, limit=100000):
    reqs = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    for _ in range(limit):
        while i < len(reqs) and reqs[i].arrival <= clock.t:
            server.submit(reqs[i])
            i += 1
        server.tick()
        if i >= len(reqs) and not server.busy():
            return
        clock.t += dt
    raise AssertionError("fake run did not finish")


def test_budget_never_exceeded_and_all_complete():
    clock = Clock()
    ex = FakeExecutor(clock, duration=lambda r: 1e-4 * r.n)
    srv = Server(ex, budget_bytes=64 << 20, clock=clock)
    rng = np.random.default_rng(1)
    reqs = [Request(rid=k, n=int(n), arrival=k * 2e-4) for k, n in
            enumerate(2 * rng.integers(16, 1024, 300))]
    drive(srv, clock, reqs)
    assert len(srv.results) == 300
    assert srv.peak_used <= srv.budget
    assert srv.used == 0
    s = summarize(srv.results, wall_s=clock.t)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_fifo_back_pressure():
    """A request too large for the remaining budget holds back later ones."""
    clock = Clock()
    ex = FakeExecutor(clock, duration=lambda r: 0.01, bytes_of=lambda r: r.n)
    srv = Server(ex, budget_bytes=100, small_n=0, clock=clock)
    srv.submit(Request(0, 60, arrival=0.0))
    srv.submit(Request(1, 60, arrival=0.0))   # must wait for 0
    srv.submit(Request(2, 10, arrival=0.0))   # fits, but FIFO keeps it behind 1
    srv.tick()
    assert [r.rid for r in srv.waiting] == [1, 2]
    clock.t = 0.02
    srv.tick()
    assert 0 in [r.rid for r in srv.results]
    assert [r.rid for r in srv.waiting] == []  # 1 and 2 admitted together now
    clock.t = 0.05
    srv.tick()
    assert sorted(r.rid for r in srv.results) == [0, 1, 2]


def test_continuous_batching_joins_next_batch():
    clock = Clock()
    launches = []
    ex = FakeExecutor(clock, duration=lambda r: 0.01)
    orig = ex.launch_batch
    ex.launch_batch = lambda reqs: (launches.append([r.rid for r in reqs]), orig(reqs))
    srv = Server(ex, budget_bytes=1 << 30, clock=clock)
    srv.submit(Request(0, 64, arrival=0.0))
    srv.tick()                      # batch [0] starts
    srv.submit(Request(1, 64))
    srv.submit(Request(2, 32))
    srv.tick()                      # batch busy: 1, 2 admitted, waiting
    assert launches == [[0]]
    clock.t = 0.011
    srv.tick()                      # 0 done, next batch [1, 2] starts at once
    assert launches == [[0], [1, 2]]


def test_rejections_and_device_errors():
    clock = Clock()
    bad = np.zeros((8, 8))
    bad[5, 2] = np.nan
    ex = FakeExecutor(clock, duration=lambda r: 1e-3, fail=lambda r: r.rid == 3,
                      bytes_of=lambda r: 8 * r.n * r.n)
    srv = Server(ex, budget_bytes=1 << 20, clock=clock)
    srv.submit(Request(0, 8, matrix=bad))                 # non-finite
    srv.submit(Request(1, 4096))                          # exceeds the budget
    for k in (2, 3, 4):
        srv.submit(Request(k, 64))
    drive(srv, clock, [])
    assert sorted(r.rid for r, _ in srv.rejected) == [0, 1]
    res = {r.rid: r for r in srv.results}
    assert res[3].error == "device error" and math.isnan(res[3].log_abs_pf)
    assert res[2].error is None and res[4].error is None


def test_fake_executor_with_oracle_pfaffians():
    """End to end on the CPU: the oracle stands in for the device."""
    clock = Clock()

    def pf(r):
        res = oracle.ltlt(r.matrix)
        return oracle.pfaffian(r.n, res["t"], res["ipiv"])

    ex = FakeExecutor(clock, duration=lambda r: 1e-3, pf=pf)
    srv = Server(ex, budget_bytes=1 << 30, clock=clock)
    mats = [inputs.skew_normal(n, 10 + n) for n in (4, 6, 10, 40)]
    reqs = [Request(k, M.shape[0], matrix=M, arrival=0.0) for k, M in enumerate(mats)]
    drive(srv, clock, reqs)
    for r in srv.results:
        la, sg = pf(reqs[r.rid])
        assert r.log_abs_pf == la and r.sign == sg


def test_gpu_executor_stream_choice():
    """The executor's stream choice (host logic only: no stream is created):
    least queued work first, ties in round-robin order; round robin rotates
    whatever the load."""
    from paper_2411_09859_amd.serving import GpuExecutor

    def bare(policy):
        ex = object.__new__(GpuExecutor)
        ex.streams = [None] * 4
        ex.policy = policy
        ex.next_stream = 0
        ex.load = [0] * 4
        return ex

    ex = bare("least_loaded")
    assert [ex._pick_stream(100) for _ in range(4)] == [0, 1, 2, 3]  # idle pool: in turn
    ex.load[0] -= 100                       # stream 0's request completed
    assert ex._pick_stream(2000) == 0
    assert ex._pick_stream(50) == 1          # 1, 2, 3 tie at 100: next in turn
    ex.load = [2000, 150, 100, 100]
    ex.next_stream = 3
    assert ex._pick_stream(10) == 3 and ex._pick_stream(10) == 2
    rr = bare("round_robin")
    rr.load = [0, 10 ** 6, 0, 0]
    assert [rr._pick_stream(1) for _ in range(6)] == [0, 1, 2, 3, 0, 1]
    with pytest.raises(ValueError):
        GpuExecutor.__init__(object.__new__(GpuExecutor), policy="random")

