"""The serving loop's scheduling on the CPU: the device calls of `serving.Server` are replaced
by stubs (no GPU, no library), so that admission order, per-job failures, client-side
cancellation and the bookkeeping of streams and memory can be checked deterministically."""
import threading
import time

import numpy as np
import pytest

from paper_2010_12117_amd import serving as S

FAIL_ALLOC, FAIL_ENQUEUE = -1, -2


class FakePlan:
    def __init__(self, n, cost_ms):
        self.info = {"in_bytes": 8 * n * n, "workspace_bytes": 1000 * n, "out_bytes": 4 * n,
                     "pn": 3, "predicted_ms": cost_ms, "D": (), "ncoeff": 1, "limbs": 1}


class StubServer(S.Server):
    """Jobs are (n x n) int64 arrays; entry [0, 0] holds the job's simulated device time in
    ms, or a FAIL_* code; entry [0, 1] a tag recorded in completion order."""

    poll_s = 0.0002  # simulated device time: no events to wait on, so the loop polls

    def __init__(self, *a, **kw):
        self.order = []
        self.gate = threading.Event()
        self.gate.set()
        super().__init__(*a, **kw)

    def _init_device(self, device, slots):
        self.torch = None
        self.streams = [None] * slots

    def _make_plan(self, coeffs, n, deg, max_workspace=None):
        return FakePlan(n, float(max(coeffs[0, 0], 0)))

    def _allocate(self, job):
        if job.coeffs[0, 0] == FAIL_ALLOC:
            raise RuntimeError("simulated out of memory")
        job.buffers = ("allocated",)

    def _enqueue_solve(self, job):
        if job.coeffs[0, 0] == FAIL_ENQUEUE:
            raise RuntimeError("simulated launch failure")

    def _enqueue_primes(self, job, b, e):
        pass

    def _enqueue_reconstruct_and_copy(self, job):
        pass

    def _record(self, job):
        job.done_event = time.perf_counter() + max(job.coeffs[0, 0], 0) / 1e3

    def _is_done(self, job):
        return self.gate.is_set() and time.perf_counter() >= job.done_event

    def _drain(self, job):
        pass

    def _take_limbs(self, job):
        self.order.append(int(job.coeffs[0, 1]))
        return np.zeros((1, 1), dtype=np.int32)


def job(ms, tag, n=2):
    a = np.zeros((n, n), dtype=np.int64)
    a[0, 0], a[0, 1] = ms, tag
    return a


def test_failed_allocation_and_enqueue_fail_only_their_job():
    srv = StubServer(memory_budget=1 << 30, slots=2, policy="fifo")
    futs = [srv.submit(job(5, 0)), srv.submit(job(FAIL_ALLOC, 1)), srv.submit(job(5, 2)),
            srv.submit(job(FAIL_ENQUEUE, 3)), srv.submit(job(5, 4))]
    with pytest.raises(RuntimeError, match="out of memory"):
        futs[1].result(timeout=10)
    with pytest.raises(RuntimeError, match="launch failure"):
        futs[3].result(timeout=10)
    for i in (0, 2, 4):
        futs[i].result(timeout=10)
    srv.close()
    assert srv.in_use == 0 and sorted(srv.free_streams) == [0, 1]
    assert srv.stats()["completed"] == 3 and srv.stats()["failed"] == 2
    assert not srv.jobs_by_future


def test_client_cancelled_future_is_dropped():
    srv = StubServer(memory_budget=1 << 30, slots=1, policy="fifo")
    srv.gate.clear()  # nothing completes until the gate opens
    first = srv.submit(job(1, 0))
    second = srv.submit(job(1, 1))
    third = srv.submit(job(1, 2))
    assert second.cancel()  # the client's own Future.cancel while the job waits
    srv.gate.set()
    first.result(timeout=10)
    third.result(timeout=10)
    srv.close()
    assert second.cancelled() and srv.order == [0, 2]
    assert srv.in_use == 0 and srv.free_streams == [0]


def test_release_is_idempotent():
    srv = StubServer(memory_budget=1 << 30, slots=1)
    f = srv.submit(job(1, 0))
    f.result(timeout=10)
    srv.close()
    j = S._Job(job(1, 9), FakePlan(2, 1.0), 123, f, 0.0)
    j.stream, j.holds = 0, True
    srv.free_streams.remove(0)
    srv.in_use += 123
    srv._release(j)
    srv._release(j)
    assert srv.in_use == 0 and srv.free_streams == [0]


def test_shortest_predicted_first_and_fifo():
    for policy, expect in (("sjf", [0, 3, 2, 1]), ("fifo", [0, 1, 2, 3])):
        srv = StubServer(memory_budget=1 << 30, slots=1, policy=policy, starve_factor=100.0,
                         starve_floor_s=10.0)
        srv.gate.clear()
        futs = [srv.submit(job(2, 0))]
        time.sleep(0.05)  # job 0 is running: the rest queue behind it
        futs += [srv.submit(job(30, 1)), srv.submit(job(10, 2)), srv.submit(job(1, 3))]
        srv.gate.set()
        for f in futs:
            f.result(timeout=10)
        srv.close()
        assert srv.order == expect, policy


def test_sjf_does_not_starve_long_jobs():
    # with no waiting allowance (factor 0, floor 0) every waiting job counts as starving,
    # and starving jobs go oldest first: the long job submitted first is not overtaken
    srv = StubServer(memory_budget=1 << 30, slots=1, policy="sjf", starve_factor=0.0,
                     starve_floor_s=0.0)
    srv.gate.clear()
    futs = [srv.submit(job(2, 0))]
    time.sleep(0.05)
    futs += [srv.submit(job(30, 1)), srv.submit(job(1, 2)), srv.submit(job(1, 3))]
    srv.gate.set()
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert srv.order == [0, 1, 2, 3]


def test_a_job_waiting_for_memory_is_not_overtaken():
    # room for the running 10x10 job and a 6x6 one: the 12x12 job that waits for memory
    # reserves its share, so the younger 6x6 and 2x2 jobs, which would fit by themselves,
    # do not start before it
    fp = lambda n: 8 * n * n + 1000 * n + 4 * n  # noqa: E731
    srv = StubServer(memory_budget=fp(10) + fp(6), slots=3, policy="fifo")
    srv.gate.clear()
    futs = [srv.submit(job(1, 0, n=10)), srv.submit(job(1, 1, n=12)),
            srv.submit(job(1, 2, n=6)), srv.submit(job(1, 3, n=2))]
    time.sleep(0.05)
    with srv.lock:
        running = sorted(int(j.coeffs[0, 1]) for j in srv.running)
        waiting = [int(j.coeffs[0, 1]) for j in srv.queue]
    assert running == [0] and waiting == [1, 2, 3]
    srv.gate.set()
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert srv.order[:2] == [0, 1] and srv.in_use == 0


def test_jobs_wait_for_a_free_stream():
    # two slots: jobs 0 and 1 run, jobs 2 and 3 wait for a stream although memory is free
    srv = StubServer(memory_budget=1 << 30, slots=2, policy="fifo")
    srv.gate.clear()
    futs = [srv.submit(job(1, t)) for t in range(4)]
    time.sleep(0.05)
    with srv.lock:
        assert sorted(int(j.coeffs[0, 1]) for j in srv.running) == [0, 1]
    srv.gate.set()
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert sorted(srv.order[:2]) == [0, 1] and sorted(srv.order[2:]) == [2, 3]
