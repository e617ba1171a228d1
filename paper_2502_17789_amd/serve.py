"""Serving loop for gridding and degridding jobs: continuous batching on one GPU.

Jobs of uneven size (different observations, grids, subgrid sizes, directions)
arrive at any time.  The server:
  * admits queued jobs first-in first-out while the sum of their device
    footprints (plan metadata and A-terms, input, output) stays within an HBM
    budget, and refuses a job that could never fit;
  * builds each admitted job's plan (host partition + upload) and its device
    buffers, and keeps them resident until the job completes;
  * every scheduling round takes one range of subgrids from every admitted job
    (round-robin) and hands all ranges to one grouped execution call, which
    packs them into shared kernel launches (gridding decomposes into
    independent subgrids, Sec. 2.2).  A job that arrives while others run is
    in the very next round; a large job is interleaved with small ones instead
    of blocking them;
  * keeps a bounded number of rounds queued on the stream, retires a job when
    the round holding its last range has finished, records its latency
    (arrival to output final on the device) and frees its memory, which lets
    the next queued jobs in.

The device work is done by a backend (``GpuBackend``: the HIP library through
``Plan`` and ``Executor``); the scheduler itself only orders work, so it can be
exercised with any object that provides the same methods.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
import time

import numpy as np

from . import AIDG_E_NOMEM, DIR_DEGRID, DIR_GRID, FP32, AidgError, Executor, Geometry, Plan, footprint


@dataclasses.dataclass
class Job:
    """One gridding ("grid": data = visibilities [nbl, nt, nc, 4]) or degridding
    ("degrid": data = grid [W, 4, N, N]) request."""

    direction: str
    geometry: Geometry
    n_stations: int
    baselines: np.ndarray
    uvw: np.ndarray
    freqs: np.ndarray
    aterms: object   # host complex array or device tensor [n_int, n_st, L, L, 4], or a
                     # callable returning one (called when the job is admitted)
    data: object     # host array or device tensor, or a callable taking the expected
                     # shape and returning one
    tag: object = None
    table: object = None   # optional caller partition (aidg_subgrid records)


@dataclasses.dataclass
class JobResult:
    output: object          # device tensor: grid (gridding) or visibilities (degridding)
    tag: object
    n_vis: int
    n_subgrids: int
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    __slots__ = ("job", "future", "handle", "n_sg", "next_sg", "arrival", "admitted", "footprint",
                 "last_token")

    def __init__(self, job, future, arrival):
        self.job, self.future, self.arrival = job, future, arrival
        self.handle = None
        self.n_sg = self.next_sg = 0
        self.admitted = 0.0
        self.footprint = 0
        self.last_token = None


def plan_geometry(job: Job) -> Geometry:
    """The geometry a served job's plan is built with: the executor holds the group
    images, so the plan itself keeps a workspace of one image."""
    g = dataclasses.replace(job.geometry)
    elem = 8 if g.precision == FP32 else 16
    g.workspace_bytes = 4 * g.subgrid_size ** 2 * elem
    return g


def retry_out_of_memory(fn, torch):
    """fn(), tried once more after an out-of-memory error from the library (status
    NOMEM) or from torch.  The library allocates its plans outside torch's caching
    allocator, so free blocks that torch keeps (outputs of retired jobs) can hold memory
    that admission counted as free, and freed plan memory returns to the device at the
    next synchronisation: both are given back before the second try."""
    try:
        return fn()
    except (AidgError, torch.OutOfMemoryError) as e:
        if isinstance(e, AidgError) and e.status != AIDG_E_NOMEM:
            raise
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return fn()


def job_footprint_estimate(job: Job) -> int:
    """Device bytes a job holds while admitted: its plan (the library's host estimate,
    aidg_footprint_estimate: A-terms, tables, subgrid records, workspace), its grid and
    its visibilities (one is the input, the other the output)."""
    f = footprint(plan_geometry(job), job.n_stations, job.baselines, job.uvw, job.freqs)
    return int(f["plan_bytes"] + f["grid_bytes"] + f["vis_bytes"])


class GpuBackend:
    """Device side of the server: plans, buffers and grouped execution.  Plans and
    inputs are uploaded on their own stream; the compute stream waits for them."""

    def __init__(self, workspace_bytes: int = 1 << 30, stream=None, timing: bool = False):
        import torch
        self.torch = torch
        self.compute = stream if stream is not None else torch.cuda.current_stream()
        self.upload = torch.cuda.Stream()
        self.executor = Executor(workspace_bytes)
        # with timing, every round is bracketed by timing events on the compute stream
        self.timing = timing
        self._timed = []

    def footprint(self, job: Job) -> int:
        return job_footprint_estimate(job)

    def prepare(self, job: Job):
        torch = self.torch
        g = plan_geometry(job)
        cdt = torch.complex64 if g.precision == FP32 else torch.complex128

        def device(x):
            x = x() if callable(x) else x
            return x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x)).to(cdt).cuda()

        def retried(fn):
            return retry_out_of_memory(fn, torch)

        with torch.cuda.stream(self.upload):
            A = retried(lambda: device(job.aterms))
            plan = retried(lambda: Plan(g, job.n_stations, job.baselines, job.uvw, job.freqs,
                                        A.contiguous(), table=job.table, stream=self.upload))
            del A   # the plan holds its own copy
            if callable(job.data):   # a factory gets the shape the plan expects
                shape = plan.grid_shape() if job.direction == "degrid" else plan.vis_shape()
                data = retried(lambda: device(job.data(shape)))
            else:
                data = retried(lambda: device(job.data))
            if job.direction == "grid":
                out = retried(lambda: torch.zeros(plan.grid_shape(), dtype=cdt, device="cuda"))
            else:
                out = retried(lambda: torch.empty(plan.vis_shape(), dtype=cdt, device="cuda"))
            ready = torch.cuda.Event()
            ready.record(self.upload)
        self.compute.wait_event(ready)
        return {"plan": plan, "in": data.contiguous(), "out": out, "dir":
                DIR_GRID if job.direction == "grid" else DIR_DEGRID}

    def n_subgrids(self, h) -> int:
        return int(h["plan"].info["n_subgrids"])

    def n_vis(self, h) -> int:
        return int(h["plan"].info["n_vis"])

    def execute(self, ranges):
        """ranges: list of (handle, sg_begin, sg_end); returns a completion token."""
        torch = self.torch
        start = None
        if self.timing:
            start = torch.cuda.Event(enable_timing=True)
            start.record(self.compute)
        self.executor.execute([(h["plan"], h["dir"], h["in"], h["out"], b, e) for h, b, e in ranges],
                              stream=self.compute)
        ev = torch.cuda.Event(enable_timing=self.timing)
        ev.record(self.compute)
        if self.timing:
            self._timed.append((start, ev))
        return ev

    def busy_seconds(self) -> float:
        """Device time of the timed rounds: the sum over rounds of the time between the
        round's first and last kernel on the compute stream (a round that waits for its
        plans' uploads counts that wait too)."""
        total = 0.0
        for a, b in self._timed:
            b.synchronize()
            total += a.elapsed_time(b) * 1e-3
        return total

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token):
        token.synchronize()

    def output(self, h):
        return h["out"]

    def release(self, h):
        h["plan"].close()
        h.clear()


class Server:
    """Continuous-batching request loop (see module docstring)."""

    def __init__(self, backend=None, hbm_budget: int | None = None, range_subgrids: int = 2048,
                 rounds_in_flight: int = 2, clock=time.perf_counter, prepare_workers: int = 0,
                 max_active: int = 32):
        self.backend = backend if backend is not None else GpuBackend()
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.75 * free)
        self.hbm_budget = int(hbm_budget)
        self.range_subgrids = int(range_subgrids)
        self.rounds_in_flight = int(rounds_in_flight)
        # Jobs admitted (preparing or active) at once.  More than a few rounds' worth
        # only adds device allocations and preparation contention, not throughput.
        self.max_active = max(1, int(max_active))
        self.clock = clock
        self._queue: collections.deque[_Active] = collections.deque()
        self._active: list[_Active] = []
        self._rounds: collections.deque = collections.deque()   # (token, [jobs retiring])
        self._preparing: list = []                               # (state, future of prepare)
        self._pool = (concurrent.futures.ThreadPoolExecutor(prepare_workers, "aidg-prepare")
                      if prepare_workers > 0 else None)
        self._in_use = 0
        self._cv = threading.Condition()
        self._thread = None
        self._stop = False
        self.completed: list[JobResult] = []
        self.peak_in_use = 0
        self.rounds = 0
        self.ranges = 0                 # subgrid ranges launched, over all rounds
        self.t_wait = 0.0               # loop time blocked on the oldest round (device-bound)
        self.t_prepare = 0.0            # time inside backend.prepare, summed over jobs

    # ------------------------------------------------------------ client side
    def submit(self, job: Job) -> concurrent.futures.Future:
        fut: concurrent.futures.Future = concurrent.futures.Future()
        with self._cv:
            self._queue.append(_Active(job, fut, self.clock()))
            self._cv.notify()
        return fut

    def start(self):
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="aidg-server", daemon=True)
        self._thread.start()
        return self

    def stop(self):
        """Finish everything submitted so far, then stop the loop."""
        with self._cv:
            self._stop = True
            self._cv.notify()
        if self._thread is not None:
            self._thread.join()
            self._thread = None
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    # ------------------------------------------------------------ scheduler
    def idle(self) -> bool:
        return not self._queue and not self._active and not self._rounds and not self._preparing

    def step(self) -> bool:
        """One scheduler pass: retire, admit, launch.  Returns True if anything happened."""
        progressed = self._retire()
        progressed |= self._admit()
        progressed |= self._collect_prepared()
        progressed |= self._launch()
        return progressed

    def _loop(self):
        while True:
            with self._cv:
                if self._stop and self.idle():
                    return
            if not self.step():
                if self._rounds:
                    t0 = self.clock()
                    self.backend.wait(self._rounds[0][0])
                    self.t_wait += self.clock() - t0
                elif self._preparing:
                    concurrent.futures.wait([f for _, f in self._preparing], timeout=0.05,
                                            return_when=concurrent.futures.FIRST_COMPLETED)
                else:
                    with self._cv:
                        if not self._queue and not self._stop:
                            self._cv.wait(timeout=0.05)

    def _admit(self) -> bool:
        admitted = False
        while True:
            with self._cv:
                if not self._queue:
                    return admitted
                st = self._queue[0]
            try:
                fp = self.backend.footprint(st.job)
            except Exception as e:  # bad request
                with self._cv:
                    self._queue.popleft()
                st.future.set_exception(e)
                continue
            if fp > self.hbm_budget:
                with self._cv:
                    self._queue.popleft()
                st.future.set_exception(MemoryError(
                    f"job needs {fp} device bytes, more than the server's budget {self.hbm_budget}"))
                continue
            if (self._in_use + fp > self.hbm_budget or
                    len(self._active) + len(self._preparing) >= self.max_active):
                return admitted     # first-in first-out: wait for memory or a slot to free up
            with self._cv:
                self._queue.popleft()
            st.footprint = fp
            self._in_use += fp
            self.peak_in_use = max(self.peak_in_use, self._in_use)
            admitted = True
            if self._pool is not None:
                self._preparing.append((st, self._pool.submit(self._timed_prepare, st.job)))
                continue
            try:
                self._activate(st, self._timed_prepare(st.job))
            except Exception as e:
                self._in_use -= fp
                st.future.set_exception(e)

    def _timed_prepare(self, job):
        t0 = self.clock()
        try:
            return self.backend.prepare(job)
        finally:
            self.t_prepare += self.clock() - t0   # float add under the GIL: no lost updates

    def _activate(self, st, handle):
        st.handle = handle
        st.n_sg = self.backend.n_subgrids(handle)
        st.admitted = self.clock()
        self._active.append(st)

    def _collect_prepared(self) -> bool:
        progressed = False
        still = []
        for st, fut in self._preparing:
            if not fut.done():
                still.append((st, fut))
                continue
            progressed = True
            try:
                self._activate(st, fut.result())
            except Exception as e:
                self._in_use -= st.footprint
                st.future.set_exception(e)
        self._preparing = still
        return progressed

    def _launch(self) -> bool:
        if len(self._rounds) >= self.rounds_in_flight:
            return False
        ranges, owners = [], []
        for st in self._active:
            if st.next_sg < st.n_sg or (st.n_sg == 0 and st.last_token is None):
                b = st.next_sg
                e = min(st.n_sg, b + self.range_subgrids)
                ranges.append((st.handle, b, e))
                owners.append(st)
                st.next_sg = e
        if not ranges:
            return False
        token = self.backend.execute(ranges)
        self.ranges += len(ranges)
        retiring = []
        for st in owners:
            if st.next_sg >= st.n_sg:
                st.last_token = token
                retiring.append(st)
        self._rounds.append((token, retiring))
        self.rounds += 1
        return True

    def _retire(self) -> bool:
        progressed = False
        while self._rounds and self.backend.done(self._rounds[0][0]):
            _, retiring = self._rounds.popleft()
            now = self.clock()
            for st in retiring:
                res = JobResult(self.backend.output(st.handle), st.job.tag, self.backend.n_vis(st.handle),
                                st.n_sg, st.arrival, st.admitted, now)
                self._active.remove(st)
                self._in_use -= st.footprint
                self.backend.release(st.handle)   # the output stays with the result
                self.completed.append(res)
                st.future.set_result(res)
            progressed = True
        return progressed

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.completed])
        if lat.size == 0:
            return {"jobs": 0}
        t0 = min(r.arrival for r in self.completed)
        t1 = max(r.finished for r in self.completed)
        nvis = sum(r.n_vis for r in self.completed)
        return {"jobs": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "makespan_s": float(t1 - t0), "mvis_per_s": float(nvis / (t1 - t0) / 1e6),
                "rounds": self.rounds, "ranges_per_round": self.ranges / max(self.rounds, 1),
                "wait_s": self.t_wait, "prepare_s": self.t_prepare, "peak_bytes": int(self.peak_in_use)}
