"""Serving loop: many independent 4PCF-multipole requests on one GPU.

Each request (a catalogue, radial bins, nmax) is planned with the request
API of the library (``fpcf4_plan``): its device footprint and its number of
centre tiles.  The server

* admits queued requests in arrival order while the sum of the footprints
  of admitted requests stays within an HBM budget (a request larger than
  the budget on its own is re-planned with smaller centre tiles, and fails
  with ``E_BUDGET`` if even that does not fit);
* gives every admitted request its own HIP stream (default priority) and a
  caller-owned workspace of exactly the planned size;
* keeps at most ``inflight`` tile steps queued on the GPU and picks the next
  (request, tile) by least estimated remaining work, so that small requests
  overtake large ones at tile granularity (continuous batching);
* finalizes a request when its last tile has completed (binary64 correction
  and copy-out), releases its workspace and admits the next requests;
* isolates failures: an error in one request (invalid input, budget,
  cancellation) completes that request with the error and leaves the others
  running.

Latency = completion time - arrival time, on the server's clock.  The
scheduling is host-side Python; every step of the estimate runs in the
library's kernels.  The backend is pluggable so the scheduling logic can be
exercised without a GPU.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable

import numpy as np

from ._lib import E_BUDGET, E_CANCELLED, Fpcf4Error

__all__ = ["Job", "Server", "LibBackend", "percentile", "latency_stats"]


@dataclasses.dataclass
class Job:
    """One estimate request.  Catalogue arrays are host NumPy float64."""
    rid: int
    x: np.ndarray
    y: np.ndarray
    g1: np.ndarray
    g2: np.ndarray
    w: np.ndarray
    edges: np.ndarray
    nmax: int
    precision: str = "fp16"
    subtract_degenerate: bool = True
    arrival: float = 0.0
    # --- filled in by the server
    state: str = "new"          # new, queued, active, done, failed, cancelled
    result: np.ndarray | None = None
    error: Exception | None = None
    admitted_at: float = math.nan
    done_at: float = math.nan
    footprint: int = 0
    ntiles: int = 0
    tile_centers: int = 0
    next_tile: int = 0
    completed_tiles: int = 0
    cost_per_tile: float = 0.0
    handle: object = None

    @property
    def n(self) -> int:
        return int(np.asarray(self.x).shape[0])

    @property
    def latency(self) -> float:
        return self.done_at - self.arrival

    def remaining_cost(self) -> float:
        return (self.ntiles - self.next_tile) * self.cost_per_tile


def pair_cost(job: Job) -> float:
    """Work estimate: ordered pairs in the radial range for uniform density
    over the catalogue's bounding box (square-field pair-count formula)."""
    n = job.n
    if n < 2:
        return 1.0
    x, y = np.asarray(job.x), np.asarray(job.y)
    lx = max(float(x.max() - x.min()), 1e-300)
    ly = max(float(y.max() - y.min()), 1e-300)
    area = lx * ly
    r_lo, r_hi = float(job.edges[0]), float(job.edges[-1])
    ann = math.pi * (min(r_hi * r_hi, area) - min(r_lo * r_lo, area))
    return max(1.0, n * n * ann / area)


class LibBackend:
    """The library's request API: one stream and one workspace per job."""

    def __init__(self, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)

    def free_bytes(self) -> int:
        return int(self.torch.cuda.mem_get_info(self.device)[0])

    def plan(self, job: Job, tile_centers: int):
        from . import plan
        return plan(job.n, job.edges, job.nmax, job.precision, tile_centers=tile_centers)

    def start(self, job: Job, tile_centers: int):
        from . import Request
        torch = self.torch
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            ws = torch.empty(job.footprint, dtype=torch.uint8, device=self.device)
        req = Request(job.x, job.y, job.g1, job.g2, job.w, job.edges, job.nmax,
                      precision=job.precision, subtract_degenerate=job.subtract_degenerate,
                      tile_centers=tile_centers, stream=stream.cuda_stream, workspace=ws)
        return {"req": req, "stream": stream, "ws": ws}

    def step(self, h, tile: int):
        h["req"].step(tile)
        ev = self.torch.cuda.Event()
        ev.record(h["stream"])
        return ev

    def ready(self, ev) -> bool:
        return bool(ev.query())

    def finalize(self, h) -> np.ndarray:
        return h["req"].finalize()

    def release(self, h):
        if h is None:
            return
        h["stream"].synchronize()
        h["req"].close()
        h["ws"] = None


class Server:
    """Admission by HBM footprint plus tile-level continuous batching."""

    def __init__(self, backend=None, hbm_budget: int | None = None, budget_fraction: float = 0.85,
                 max_active: int = 8, inflight: int = 2, tile_centers: int = 65536,
                 min_tile_centers: int = 1024, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend if backend is not None else LibBackend()
        if hbm_budget is None:
            hbm_budget = int(budget_fraction * self.backend.free_bytes())
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.inflight = max(1, int(inflight))
        self.tile_centers = int(tile_centers)
        self.min_tile_centers = int(min_tile_centers)
        self.clock = clock
        self.t0 = clock()
        self.queue: list[Job] = []
        self.active: list[Job] = []
        self.finished: list[Job] = []
        self.pending: list[tuple[object, Job, int]] = []   # (event, job, tile)
        self.used = 0
        self.peak_used = 0
        self.cancel_requests: set[int] = set()

    # ------------------------------------------------------------------ api
    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, job: Job):
        """Queue a job (arrival = now unless already set later than 0)."""
        if not job.arrival:
            job.arrival = self.now()
        job.state = "queued"
        try:
            self._plan(job)
        except Exception as e:   # invalid request: fails alone
            self._fail(job, e)
            return job
        self.queue.append(job)
        return job

    def cancel(self, rid: int):
        """Cancel a queued or running job between tiles."""
        self.cancel_requests.add(rid)

    def idle(self) -> bool:
        return not (self.queue or self.active or self.pending)

    def poll(self) -> bool:
        """One scheduler iteration; returns True if anything progressed."""
        progressed = self._complete()
        progressed |= self._cancel()
        progressed |= self._admit()
        progressed |= self._issue()
        return progressed

    def drain(self, sleep: float = 2e-4):
        while not self.idle():
            if not self.poll():
                time.sleep(sleep)

    def run(self, jobs: list[Job], sleep: float = 2e-4) -> list[Job]:
        """Serve jobs whose ``arrival`` times (seconds from now) are already
        set: each is submitted when the clock reaches its arrival."""
        self.t0 = self.clock()
        todo = sorted(jobs, key=lambda j: j.arrival)
        k = 0
        while k < len(todo) or not self.idle():
            t = self.now()
            while k < len(todo) and todo[k].arrival <= t:
                self.submit(todo[k])
                k += 1
            if not self.poll():
                time.sleep(sleep)
        return jobs

    # ------------------------------------------------------------ internals
    def _plan(self, job: Job):
        tile = self.tile_centers
        while True:
            nbytes, ntiles = self.backend.plan(job, tile)
            if nbytes <= self.budget or tile <= self.min_tile_centers:
                break
            tile = max(self.min_tile_centers, tile // 2)
        if nbytes > self.budget:
            raise Fpcf4Error(E_BUDGET, f"request {job.rid} needs {nbytes} B, budget {self.budget} B")
        job.footprint, job.ntiles, job.tile_centers = int(nbytes), int(ntiles), tile
        ncent = job.n
        job.cost_per_tile = pair_cost(job) * min(tile, max(ncent, 1)) / max(ncent, 1)

    def _fail(self, job: Job, err: Exception):
        job.state = "cancelled" if isinstance(err, Fpcf4Error) and err.status == E_CANCELLED else "failed"
        job.error = err
        job.done_at = self.now()
        self.finished.append(job)

    def _retire(self, job: Job):
        if job in self.active:
            self.active.remove(job)
            self.used -= job.footprint
        try:
            self.backend.release(job.handle)
        finally:
            job.handle = None

    def _admit(self) -> bool:
        progressed = False
        while self.queue and len(self.active) < self.max_active:
            job = self.queue[0]
            if self.used + job.footprint > self.budget:
                break     # arrival order: wait for memory
            self.queue.pop(0)
            try:
                job.handle = self.backend.start(job, job.tile_centers)
            except Exception as e:
                self._fail(job, e)
                progressed = True
                continue
            job.state = "active"
            job.admitted_at = self.now()
            self.active.append(job)
            self.used += job.footprint
            self.peak_used = max(self.peak_used, self.used)
            progressed = True
            if job.ntiles == 0:
                self._finish(job)
        return progressed

    def _issue(self) -> bool:
        progressed = False
        while len(self.pending) < self.inflight:
            cands = [j for j in self.active if j.next_tile < j.ntiles]
            if not cands:
                break
            job = min(cands, key=lambda j: (j.remaining_cost(), j.arrival))
            tile = job.next_tile
            try:
                ev = self.backend.step(job.handle, tile)
            except Exception as e:
                self._retire(job)
                self._fail(job, e)
                progressed = True
                continue
            job.next_tile += 1
            self.pending.append((ev, job, tile))
            progressed = True
        return progressed

    def _complete(self) -> bool:
        progressed = False
        keep = []
        for ev, job, tile in self.pending:
            if self.backend.ready(ev):
                job.completed_tiles += 1
                progressed = True
                if job.completed_tiles == job.ntiles and job.state == "active":
                    self._finish(job)
            else:
                keep.append((ev, job, tile))
        self.pending = keep
        return progressed

    def _finish(self, job: Job):
        try:
            job.result = self.backend.finalize(job.handle)
            job.state = "done"
            job.done_at = self.now()
            self.finished.append(job)
        except Exception as e:
            self._fail(job, e)
        finally:
            self._retire(job)

    def _cancel(self) -> bool:
        if not self.cancel_requests:
            return False
        progressed = False
        for job in list(self.queue):
            if job.rid in self.cancel_requests:
                self.queue.remove(job)
                self._fail(job, Fpcf4Error(E_CANCELLED, f"request {job.rid} cancelled"))
                progressed = True
        for job in list(self.active):
            if job.rid in self.cancel_requests and not any(p[1] is job for p in self.pending):
                self._retire(job)
                self._fail(job, Fpcf4Error(E_CANCELLED, f"request {job.rid} cancelled"))
                progressed = True
        self.cancel_requests = {r for r in self.cancel_requests
                                if any(j.rid == r for j in self.queue + self.active)}
        return progressed


def percentile(values, q: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return math.nan
    return float(np.percentile(v, q))


def latency_stats(jobs) -> dict:
    lat = [j.latency for j in jobs if j.state == "done"]
    return {"n_done": len(lat), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "mean_s": float(np.mean(lat)) if lat else math.nan,
            "max_s": float(np.max(lat)) if lat else math.nan}
