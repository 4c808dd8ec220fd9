"""The serving loop: jobs admitted by device memory footprint, running concurrently on
several streams, give results bit-identical to the same job solved alone, and to the
oracle."""
import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
from paper_2010_12117_amd import serving as S
import workloads as W
from oracle import det as OD
from oracle import plan as PL

from helpers import box_to_dict

pytestmark = pytest.mark.gpu


def small_jobs(seed, count):
    rng = np.random.default_rng(900 + seed)
    jobs = []
    for _ in range(count):
        n = int(rng.integers(2, 11))
        k = int(rng.integers(2, 4))
        deg = tuple(int(x) for x in rng.integers(1, 3, size=k))
        jobs.append(W.random_matrix(rng, n, deg, -65536, 65536))
    return jobs


def alone(a):
    import torch
    n, deg = B.shape_of(a)
    pl = pdm.plan(n, deg, host_coeffs=a)
    out, _ = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(a)).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("budget_mb,slots", [(4096, 4), (48, 2)])
def test_mix_equals_alone(budget_mb, slots):
    jobs = small_jobs(budget_mb, 24)
    srv = S.Server(memory_budget=budget_mb << 20, slots=slots)
    futs = [srv.submit(a) for a in jobs]
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["p99_s"] >= st["p50_s"] > 0
    for a, r in zip(jobs, results):
        assert np.array_equal(r.limbs, alone(a))
    for a, r in list(zip(jobs, results))[:4]:
        n, deg = B.shape_of(a)
        expect = OD.det_pointwise(a, PL.det_degree_bound_from_shape(n, deg))
        assert box_to_dict(r.coefficients()) == box_to_dict(expect)


def test_oversized_job_is_rejected():
    srv = S.Server(memory_budget=1 << 20, slots=1)
    with pytest.raises(ValueError):
        srv.submit(W.config2())
    srv.close()


def test_out_of_order_completion():
    # a large job first, then small ones on the other slots: the small ones finish first and
    # leave the running list from the middle. One prime per enqueued range keeps the large
    # job in flight over many turns of the server loop, whatever the GPU's speed.
    rng = np.random.default_rng(77)
    big = W.random_matrix(rng, 24, (3, 3, 3), -1000, 1000)
    jobs = [big] + small_jobs(5, 16)
    srv = S.Server(memory_budget=8 << 30, slots=4, prime_chunk=1)
    futs = [srv.submit(a) for a in jobs]
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.stats()["completed"] == len(jobs)
    order = sorted(range(len(jobs)), key=lambda i: results[i].finished)
    assert order[0] != 0  # some small job finished before the first one
    for a, r in zip(jobs, results):
        assert np.array_equal(r.limbs, alone(a))


def test_chunked_jobs_equal_alone():
    jobs = small_jobs(11, 10) + [W.config2()]
    srv = S.Server(memory_budget=8 << 30, slots=3, prime_chunk=2)
    futs = [srv.submit(a) for a in jobs]
    results = [f.result(timeout=120) for f in futs]
    srv.close()
    for a, r in zip(jobs, results):
        assert np.array_equal(r.limbs, alone(a))


def test_cancel_waiting_and_running_jobs():
    from concurrent.futures import CancelledError
    # the job cancelled while running: 28 primes of a 256^3 grid, run one prime at a time
    # (tens of ms each), so it is still running when the cancel comes
    big = W.random_matrix(np.random.default_rng(7), 32, (5, 5, 5), -65536, 65536)
    smalls = small_jobs(12, 4)
    srv = S.Server(memory_budget=8 << 30, slots=1, prime_chunk=1)
    f_big = srv.submit(big)
    f_small = [srv.submit(a) for a in smalls]
    # the last small job is still waiting behind the others on the single slot
    assert srv.cancel(f_small[-1])
    with pytest.raises(CancelledError):
        f_small[-1].result(timeout=5)
    assert srv.cancel(f_big)  # running: stops at its next prime boundary
    with pytest.raises(CancelledError):
        f_big.result(timeout=60)
    for a, f in zip(smalls[:-1], f_small[:-1]):
        assert np.array_equal(f.result(timeout=60).limbs, alone(a))
    assert not srv.cancel(f_small[0])  # already finished
    srv.close()
    assert srv.in_use == 0


def test_job_above_budget_runs_on_a_capped_plan():
    a = W.config2()
    info = pdm.plan(12, (3, 3, 3), host_coeffs=a, flags=pdm.HOST_ONLY).info
    full = info["in_bytes"] + info["workspace_bytes"] + info["out_bytes"]
    srv = S.Server(memory_budget=full // 2, slots=2)
    r = srv.submit(a).result(timeout=120)
    srv.close()
    assert r.info["prime_group"] < r.info["pn"]
    assert np.array_equal(r.limbs, alone(a))


def test_job_above_one_prime_runs_on_grid_slabs():
    # a budget below one prime's footprint: the job's grid runs in slabs, same result
    a = W.config2()
    info = pdm.plan(12, (3, 3, 3), host_coeffs=a, flags=pdm.HOST_ONLY).info
    srv = S.Server(memory_budget=info["in_bytes"] + info["out_bytes"] + (7 << 20), slots=1)
    r = srv.submit(a).result(timeout=120)
    srv.close()
    assert r.info["prime_group"] == 1 and r.info["grid_slabs"] >= 2
    assert np.array_equal(r.limbs, alone(a))


def test_config5_mix_with_a_large_job_equals_alone():
    # jobs drawn like the serving workload's (n 4..32, 2-3 variables, degree 1-5, coefficients
    # in [-2^16, 2^16]) plus one 32 x 32 trivariate degree-5 job, four at a time: every result
    # in the mix is bit-identical to the same job solved alone
    rng = W.rng_for(5, salt=7)
    jobs = [W.config5_job(rng) for _ in range(10)]
    jobs.insert(3, W.random_matrix(np.random.default_rng(5032), 32, (5, 5, 5), -65536, 65536))
    srv = S.Server(memory_budget=120 << 30, slots=4)
    futs = [srv.submit(a) for a in jobs]
    results = [f.result(timeout=300) for f in futs]
    srv.close()
    assert srv.stats()["completed"] == len(jobs)
    assert results[3].info["N"] == (256, 256, 256)
    for a, r in zip(jobs, results):
        assert np.array_equal(r.limbs, alone(a))
