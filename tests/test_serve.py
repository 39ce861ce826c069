"""Serving scheduler on the CPU: admission, continuous batching, cancellation
and error isolation, with a fake backend that simulates tile steps.  The
planning call itself is the library's host-side planner where noted."""
import math

import numpy as np
import pytest

from paper_2509_07974_amd._lib import E_BUDGET, E_CANCELLED, E_INVALID_ARG, Fpcf4Error
from paper_2509_07974_amd.serve import Job, Server, latency_stats, pair_cost


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Footprint = base + per-centre bytes of one tile; a tile step is ready
    `delay` polls after it was issued.  Records the peak number of bytes in
    use and the order in which tiles were issued."""

    def __init__(self, clock, base=1000, per_centre=10, delay=2, fail_start=(), fail_step=()):
        self.clock, self.base, self.per_centre, self.delay = clock, base, per_centre, delay
        self.fail_start, self.fail_step = set(fail_start), set(fail_step)
        self.live = {}
        self.issued = []
        self.polls = 0

    def free_bytes(self):
        return 10 ** 9

    def plan(self, job, tile):
        if not np.all(np.isfinite(job.x)):
            raise Fpcf4Error(E_INVALID_ARG, "non-finite")
        t = min(tile, max(job.n, 1))
        return self.base + self.per_centre * t, math.ceil(job.n / tile) if job.n else 0

    def start(self, job, tile):
        if job.rid in self.fail_start:
            raise Fpcf4Error(E_INVALID_ARG, "start failed")
        self.live[job.rid] = job.footprint
        return {"rid": job.rid, "n": job.n}

    def step(self, h, tile):
        if h["rid"] in self.fail_step:
            raise Fpcf4Error(E_INVALID_ARG, "step failed")
        self.issued.append((h["rid"], tile))
        return [self.delay]

    def ready(self, ev):
        self.clock.t += 0.001
        ev[0] -= 1
        return ev[0] <= 0

    def finalize(self, h):
        return np.full(3, float(h["rid"]))

    def release(self, h):
        if h is not None:
            self.live.pop(h["rid"], None)


def make_job(rid, n, arrival=0.0, side=100.0, seed=0):
    rng = np.random.default_rng(seed + rid)
    x = rng.uniform(0, side, n)
    y = rng.uniform(0, side, n)
    z = np.zeros(n)
    return Job(rid, x, y, z, z, np.ones(n), np.array([1.0, 10.0]), 2, arrival=arrival)


def test_all_done_and_budget_respected():
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=30000, tile_centers=1000, clock=clk, inflight=2)
    jobs = [make_job(r, n) for r, n in enumerate([3000, 500, 2500, 1200, 800])]
    for j in jobs:
        srv.submit(j)
    peak_live = 0
    while not srv.idle():
        srv.poll()
        peak_live = max(peak_live, sum(be.live.values()))
    assert all(j.state == "done" for j in jobs)
    assert all(np.all(j.result == j.rid) for j in jobs)
    assert srv.peak_used <= srv.budget and peak_live <= srv.budget
    # every tile of every job issued exactly once
    for j in jobs:
        assert sorted(t for r, t in be.issued if r == j.rid) == list(range(j.ntiles))


def test_budget_too_small_fails_alone():
    clk = FakeClock()
    be = FakeBackend(clk, base=5000, per_centre=10)
    srv = Server(be, hbm_budget=6000, tile_centers=1000, min_tile_centers=50, clock=clk)
    big = make_job(0, 3000)   # base alone fits; 50-centre tiles fit too
    huge = make_job(1, 100)
    be2 = FakeBackend(clk, base=7000)
    srv.submit(big)
    assert big.tile_centers < 1000 and big.footprint <= 6000
    srv2 = Server(be2, hbm_budget=6000, tile_centers=1000, clock=clk)
    srv2.submit(huge)
    assert huge.state == "failed" and huge.error.status == E_BUDGET
    srv.drain()
    assert big.state == "done"


def test_error_isolation():
    clk = FakeClock()
    be = FakeBackend(clk, fail_start={1}, fail_step={3})
    srv = Server(be, hbm_budget=10 ** 6, tile_centers=400, clock=clk)
    bad_input = make_job(2, 50)
    bad_input.x[3] = np.nan
    jobs = [make_job(0, 1000), make_job(1, 1000), bad_input, make_job(3, 900), make_job(4, 700)]
    for j in jobs:
        srv.submit(j)
    srv.drain()
    st = {j.rid: j.state for j in jobs}
    assert st == {0: "done", 1: "failed", 2: "failed", 3: "failed", 4: "done"}
    assert srv.used == 0 and not be.live


def test_cancel_queued_and_running():
    clk = FakeClock()
    be = FakeBackend(clk, delay=3)
    srv = Server(be, hbm_budget=1000 + 10 * 500, tile_centers=500, clock=clk, max_active=1)
    jobs = [make_job(r, 2000) for r in range(3)]
    for j in jobs:
        srv.submit(j)
    srv.poll()
    srv.poll()
    srv.cancel(0)    # running
    srv.cancel(2)    # queued
    srv.drain()
    assert jobs[0].state == "cancelled" and jobs[0].error.status == E_CANCELLED
    assert jobs[2].state == "cancelled"
    assert jobs[1].state == "done"
    assert len([t for r, t in be.issued if r == 0]) < jobs[0].ntiles
    assert not any(r == 2 for r, _ in be.issued)


def test_small_request_overtakes_large():
    clk = FakeClock()
    be = FakeBackend(clk, delay=1)
    srv = Server(be, hbm_budget=10 ** 6, tile_centers=100, clock=clk, inflight=1)
    big = make_job(0, 5000)
    srv.submit(big)
    for _ in range(10):
        srv.poll()
    small = make_job(1, 150)
    srv.submit(small)
    srv.drain()
    assert small.done_at < big.done_at
    # the small job's tiles were issued before the big job's remaining ones
    first_small = next(i for i, (r, _) in enumerate(be.issued) if r == 1)
    assert all(r == 1 for r, _ in be.issued[first_small:first_small + small.ntiles])


def test_timed_run_latency_stats():
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=10 ** 6, tile_centers=500, clock=clk)
    jobs = [make_job(r, 300 + 200 * r, arrival=0.002 * r) for r in range(6)]
    srv.run(jobs, sleep=0.0)
    s = latency_stats(jobs)
    assert s["n_done"] == 6 and s["p50_s"] <= s["p99_s"] <= s["max_s"]
    assert all(j.latency >= 0 for j in jobs)


def test_pair_cost_scales_with_density():
    a = make_job(0, 1000, side=100.0)
    b = make_job(1, 2000, side=100.0)
    assert 3.0 < pair_cost(b) / pair_cost(a) < 5.0


def test_library_planner_footprint_monotone_in_tile():
    from paper_2509_07974_amd import plan
    import synth
    edges = synth.log_edges(1.0, 100.0, 8)
    b1, t1 = plan(200000, edges, 8, "fp16", tile_centers=65536)
    b2, t2 = plan(200000, edges, 8, "fp16", tile_centers=16384)
    assert b2 < b1 and t2 > t1 and t1 == 4 and t2 == 13
