"""Continuous-batching request loop for exact polynomial determinants on one GPU.

Clients call `Server.submit(coeffs)` and get a future. A background thread admits queued
jobs as soon as a stream slot and enough device memory are free, so jobs that arrive while
others run are started at once and overlap on the device (one HIP stream per admitted job,
all at the default priority). A job's device footprint is known from its plan before it
runs: coefficients + workspace (residues, evaluation passes, determinants, interpolation)
+ output limbs. Every intermediate stays on the device; only the input coefficients go in
and the result limbs come out.

Admission order. With policy "fifo" the oldest waiting job goes first. With policy "sjf"
(the default) the waiting job with the shortest predicted device time goes first (the plan's
running-time prediction, polydet_plan_info.predicted_ms), except that a job that has waited
longer than `starve_factor` times its own predicted time plus `starve_floor_s` takes
precedence over every job that has not, oldest first: short jobs stay ahead of long ones,
and long ones are not starved. In both policies the first job in that order that does not fit
reserves its memory, and later jobs may start only if they fit beside the reservation. A job
whose one-shot footprint exceeds the whole budget runs on a capped plan (polydet_plan_capped:
primes in groups, and below one prime's footprint each prime's grid in slabs; same result)
when that fits.

With `prime_chunk`, a job runs as a sequence of prime ranges (polydet_solve_primes), one range
in flight at a time, then the reconstruction (polydet_reconstruct). Between ranges the server
can stop it: `cancel` ends a waiting job at once and a running one at its next range boundary,
and its future raises CancelledError.

Failures are per job: if a job's buffers cannot be allocated or its solve cannot be enqueued,
that job's future raises the error, its stream and memory are given back, and the server goes
on with the others. A future the client cancels before its job starts is dropped.

The solve itself is the library's (binding.py); this module only schedules it. The device
calls are isolated in a few methods (`_init_device`, `_make_plan`, `_allocate`, `_enqueue_*`,
`_record`, `_is_done`, `_drain`, `_take_limbs`), so that the scheduling can be exercised
without a GPU.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import CancelledError, Future, ThreadPoolExecutor
from dataclasses import dataclass
from typing import Deque, List

import numpy as np

from . import binding as B


@dataclass
class Result:
    """Limbs (ncoeff x limbs, uint32 two's complement) and plan information of a job."""
    limbs: np.ndarray
    info: dict
    submitted: float
    started: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.submitted

    def coefficients(self) -> np.ndarray:
        """Object array of Python ints with shape (D1+1, ..., Dk+1)."""
        vals = B.limbs_to_ints(self.limbs)
        out = np.empty(len(vals), dtype=object)
        for i, v in enumerate(vals):
            out[i] = v
        box = tuple(d + 1 for d in self.info["D"])
        return out.reshape(box) if box else out.reshape(())


@dataclass(eq=False)  # jobs are compared by identity (they hold arrays)
class _Job:
    coeffs: np.ndarray
    plan: object
    footprint: int
    future: Future
    submitted: float
    predicted_s: float = 0.0
    started: float = 0.0
    stream: object = None
    buffers: tuple = ()
    host_out: object = None
    done_event: object = None
    next_prime: int = 0    # chunked jobs: first prime not yet enqueued
    final: bool = False    # the reconstruction and the copy-out are enqueued
    cancelled: bool = False
    holds: bool = False    # holds a stream and its footprint of the budget


class Server:
    """Admits determinant jobs by device memory footprint and runs them concurrently.

    memory_budget: device bytes the server may hold for jobs at once.
    slots: jobs in flight at once (one stream each).
    prime_chunk: primes per enqueued range (None: the whole solve at once).
    policy: "sjf" (shortest predicted first, with aging) or "fifo"."""

    # None: the loop sleeps until a waiter thread reports a finished device step (_watch); a
    # number: it polls _is_done that often instead (device stand-ins without events)
    poll_s = None

    def __init__(self, memory_budget: int = 64 << 30, slots: int = 4, device: str = "cuda:0",
                 flags: int = 0, prime_chunk=None, policy: str = "sjf",
                 starve_factor: float = 4.0, starve_floor_s: float = 0.05):
        if policy not in ("sjf", "fifo"):
            raise ValueError("policy must be 'sjf' or 'fifo'")
        self.budget = int(memory_budget)
        self.flags = flags
        self.prime_chunk = prime_chunk
        self.policy = policy
        self.starve_factor = float(starve_factor)
        self.starve_floor_s = float(starve_floor_s)
        self.jobs_by_future = {}
        self._init_device(device, slots)
        self.free_streams = list(range(slots))
        self.queue: Deque[_Job] = collections.deque()
        self.running: List[_Job] = []
        self.in_use = 0
        self.lock = threading.Condition()
        self.closed = False
        self.latencies: List[float] = []
        self.completed = 0
        self.failed = 0
        self.thread = threading.Thread(target=self._loop, name="polydet-server", daemon=True)
        self.thread.start()

    # ------------------------------------------------------------------ device calls
    def _init_device(self, device, slots):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # one outstanding device step per running job: a waiter per slot (and spares)
        self.waiters = ThreadPoolExecutor(max_workers=2 * slots, thread_name_prefix="polydet-wait")

    def _make_plan(self, coeffs, n, deg, max_workspace=None):
        return B.plan(n, deg, host_coeffs=coeffs, flags=self.flags, max_workspace=max_workspace)

    def _allocate(self, job: _Job):
        torch = self.torch
        info = job.plan.info
        with torch.cuda.stream(self.streams[job.stream]):
            host_in = torch.from_numpy(job.coeffs.reshape(-1)).pin_memory()
            d_in = torch.empty(host_in.numel(), dtype=torch.int64, device=self.device)
            d_in.copy_(host_in, non_blocking=True)
            d_out = torch.empty((info["ncoeff"], info["limbs"]), dtype=torch.int32,
                                device=self.device)
            ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=self.device)
            job.host_out = torch.empty(d_out.shape, dtype=torch.int32, pin_memory=True)
        job.buffers = (host_in, d_in, d_out, ws)

    def _enqueue_solve(self, job: _Job):
        stream = self.streams[job.stream]
        _, d_in, d_out, ws = job.buffers
        with self.torch.cuda.stream(stream):
            B.solve_device(job.plan, d_in, d_out, ws, stream=stream)

    def _enqueue_primes(self, job: _Job, b: int, e: int):
        _, d_in, _, ws = job.buffers
        B.solve_primes_device(job.plan, d_in, b, e, ws, stream=self.streams[job.stream])

    def _enqueue_reconstruct_and_copy(self, job: _Job):
        stream = self.streams[job.stream]
        _, _, d_out, ws = job.buffers
        if self.prime_chunk:
            B.reconstruct_device(job.plan, ws, d_out, stream=stream)
        with self.torch.cuda.stream(stream):
            job.host_out.copy_(d_out, non_blocking=True)

    def _record(self, job: _Job):
        # a blocking-sync event: its waiter sleeps until the step is done instead of spinning
        job.done_event = self.torch.cuda.Event(blocking=True)
        job.done_event.record(self.streams[job.stream])
        self.waiters.submit(self._watch, job.done_event)

    def _watch(self, event):
        # wakes the serving loop when the device step behind `event` has finished
        event.synchronize()
        with self.lock:
            self.lock.notify()

    def _is_done(self, job: _Job) -> bool:
        return job.done_event.query()

    def _drain(self, job: _Job):
        if job.stream is not None:
            self.streams[job.stream].synchronize()

    def _take_limbs(self, job: _Job) -> np.ndarray:
        return job.host_out.numpy().copy()

    # ------------------------------------------------------------------ client side
    def submit(self, coeffs: np.ndarray) -> Future:
        coeffs = np.ascontiguousarray(coeffs, dtype=np.int64)
        n, deg = B.shape_of(coeffs)
        pl = self._make_plan(coeffs, n, deg)
        info = pl.info
        footprint = int(info["in_bytes"] + info["workspace_bytes"] + info["out_bytes"])
        if footprint > self.budget:
            # primes in groups (and grid slabs): the workspace shrinks to what the budget leaves
            cap = self.budget - info["in_bytes"] - info["out_bytes"]
            too_big = ValueError(f"job needs {footprint} device bytes one-shot and does not fit "
                                 "the server budget even one prime at a time in grid slabs")
            if cap <= 0:
                raise too_big
            try:
                pl = self._make_plan(coeffs, n, deg, max_workspace=cap)
            except B.PolydetError:
                raise too_big from None
            info = pl.info
            footprint = int(info["in_bytes"] + info["workspace_bytes"] + info["out_bytes"])
        fut: Future = Future()
        job = _Job(coeffs, pl, footprint, fut, time.perf_counter(),
                   predicted_s=float(info.get("predicted_ms", 0.0)) / 1e3)
        with self.lock:
            if self.closed:
                raise RuntimeError("server is closed")
            self.queue.append(job)
            self.jobs_by_future[id(fut)] = job
            self.lock.notify()
        return fut

    def cancel(self, fut: Future) -> bool:
        """Stop a job: a waiting one now, a running chunked one at its next range boundary.
        Returns False when the job has already finished."""
        with self.lock:
            job = self.jobs_by_future.get(id(fut))
            if job is None or fut.done():
                return False
            if job in self.queue:
                self.queue.remove(job)
                del self.jobs_by_future[id(fut)]
                self._resolve(job, exc=CancelledError())
            else:
                job.cancelled = True
            self.lock.notify()
            return True

    def close(self, wait: bool = True):
        with self.lock:
            self.closed = True
            self.lock.notify()
        if wait:
            self.thread.join()
            waiters = getattr(self, "waiters", None)
            if waiters is not None:
                waiters.shutdown(wait=True)  # every recorded step has finished by now

    def stats(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"completed": self.completed, "failed": self.failed,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean())}

    # ------------------------------------------------------------------ server side
    def _resolve(self, job: _Job, result=None, exc=None):
        """Complete the job's future once; a future the client has cancelled stays so."""
        fut = job.future
        if fut.done():
            return
        if exc is not None:
            fut.set_exception(exc)
        else:
            fut.set_result(result)

    def _admission_order(self, now: float) -> List[_Job]:
        jobs = list(self.queue)
        if self.policy == "fifo":
            return jobs

        def key(j: _Job):
            starving = now - j.submitted > self.starve_factor * j.predicted_s + self.starve_floor_s
            return (0, j.submitted) if starving else (1, j.predicted_s, j.submitted)
        return sorted(jobs, key=key)

    def _admit(self):
        """Start every queued job that fits (called with the lock held)."""
        reserved = 0
        waiting = 0
        gone = set()  # jobs that leave the queue: started, failed or cancelled by the client
        try:
            for job in self._admission_order(time.perf_counter()):
                if job.future.cancelled():
                    gone.add(id(job))
                    self.jobs_by_future.pop(id(job.future), None)
                    continue
                if self.free_streams and self.in_use + reserved + job.footprint <= self.budget:
                    gone.add(id(job))
                    self._start(job)
                else:
                    if not waiting:
                        reserved += job.footprint  # the first waiting job holds its share
                    waiting += 1
        finally:
            # the jobs not started stay queued, in submission order
            self.queue = collections.deque(j for j in self.queue if id(j) not in gone)

    def _start(self, job: _Job):
        """Take a stream and the job's share of the budget, then enqueue its first work. A
        failure fails this job only."""
        job.stream = self.free_streams.pop()
        job.holds = True
        self.in_use += job.footprint
        job.started = time.perf_counter()
        try:
            self._allocate(job)
            if self.prime_chunk:
                self._enqueue_range(job)
            else:
                self._enqueue_solve(job)
                self._enqueue_copy_out(job)
        except Exception as e:
            self._fail(job, e)
            return
        self.running.append(job)

    def _fail(self, job: _Job, exc: BaseException):
        """A job whose enqueueing failed: wait for what it did enqueue, give back its stream
        and memory, and raise the error to its client."""
        try:
            self._drain(job)
        finally:
            self._release(job)
            self.failed += 1
            self._resolve(job, exc=exc)

    def _enqueue_range(self, job: _Job):
        """The next range of primes of a chunked job."""
        pn = job.plan.info["pn"]
        b, e = job.next_prime, min(pn, job.next_prime + int(self.prime_chunk))
        self._enqueue_primes(job, b, e)
        job.next_prime = e
        self._record(job)

    def _enqueue_copy_out(self, job: _Job):
        """(chunked jobs: the reconstruction, then) the copy of the limbs to pinned memory."""
        self._enqueue_reconstruct_and_copy(job)
        job.final = True
        self._record(job)

    def _release(self, job: _Job):
        """Give back the job's stream and budget share (once) and drop its buffers. Called
        only when nothing of the job is pending on its stream."""
        job.buffers = ()
        job.host_out = None
        if job.holds:
            job.holds = False
            self.in_use -= job.footprint
            self.free_streams.append(job.stream)
        self.jobs_by_future.pop(id(job.future), None)

    def _advance(self, job: _Job) -> bool:
        """A running job's last enqueued work is done: enqueue what comes next. Returns True
        when the job has left the running set."""
        if job.cancelled:
            self._release(job)
            self._resolve(job, exc=CancelledError())
            return True
        if job.final:
            self._finish(job)
            return True
        if job.next_prime < job.plan.info["pn"]:
            self._enqueue_range(job)
        else:
            self._enqueue_copy_out(job)
        return False

    def _finish(self, job: _Job):
        now = time.perf_counter()
        info = job.plan.info
        res = Result(self._take_limbs(job), info, job.submitted, job.started, now)
        self._release(job)
        self.latencies.append(res.latency)
        self.completed += 1
        self._resolve(job, result=res)

    def _loop(self):
        try:
            self._serve()
        except BaseException as e:  # pragma: no cover - fail every waiting client, loudly
            with self.lock:
                self.closed = True
                pending = list(self.running) + list(self.queue)
                self.running, self.queue = [], collections.deque()
            for j in pending:
                self._resolve(j, exc=e)
            raise

    def _serve(self):
        while True:
            with self.lock:
                done = [j for j in self.running if self._is_done(j)]
                for j in done:
                    try:
                        left = self._advance(j)
                    except Exception as e:  # surfaced to this job's client only
                        left = True
                        self._fail(j, e)
                    if left:
                        self.running.remove(j)
                self._admit()
                if self.closed and not self.queue and not self.running:
                    return
                if not done:
                    # until a waiter reports a finished step, a client submits or cancels, or
                    # close() is called (or the polling interval of a stand-in passes)
                    self.lock.wait(timeout=self.poll_s if self.poll_s else 0.05)


def poisson_arrivals(rng: np.random.Generator, count: int, rate: float) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
