"""Throughput of the exact polynomial determinant on one MI355X.

Workload: a 12 x 12 matrix of trivariate polynomials of degree 3 per variable with
coefficients uniform in [-1000, 1000] and 30% zero entries (seeded), determinant degree
bound 36 per variable, 64^3 evaluation grid, 7 primes. One step = one full solve
(reduce, evaluate, determinants, interpolate, reconstruct) with the coefficients already in
HBM and a warm plan. The metric is modular determinants per second (prime x grid point),
whole job; exact polynomial determinants per second are reported beside it.

Prints one JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time
from concurrent.futures import TimeoutError as FutureTimeout

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peaks of MI355X used for the roofline (published figures; see the design notes).
HBM_PEAK_GBS = 8000.0
CU, CLOCK_HZ = 256, 2.4e9
# one elimination update = 3 v_mad_u64_u32 + 1 v_mul_lo_u32 (fp64-FMA rate, 64 lanes/clk/CU)
# + 2 plain 32-bit ops (128 lanes/clk/CU) -> 12.8 updates/clk/CU
UPDATES_PER_CLK_CU = 1.0 / (4 / 64 + 2 / 128)
ALU_PEAK_UPDATES = CU * CLOCK_HZ * UPDATES_PER_CLK_CU


# HBM bytes per launch of the fused elimination kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes scaled by a 1 GiB copy (profiles/config2_hbm_traffic.md),
# valid only for the kernel sources and tuning table they were taken with (their hash).
DET_TRAFFIC = {"sources_sha256_16": "1809aef6fb7ee63f", "bytes": 186.2e6 + 14.7e6}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in ("paper_2010_12117_amd/csrc/det_impl.h", "paper_2010_12117_amd/csrc/modarith.h",
                "paper_2010_12117_amd/tuning_gfx950.json"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def det_updates(n: int) -> int:
    """Elimination updates of one determinant: sum_{m=1}^{n-1} m^2."""
    return (n - 1) * n * (2 * n - 1) // 6


def expand_bytes(pn: int, nnz: int, m, N) -> int:
    """Algorithmic HBM bytes of the evaluation passes of one solve when the first variable is
    evaluated inside the elimination kernel: the passes run over variables k-1 .. 1 of every
    nonzero entry, each reading its input box and writing its output box (the residues
    m_0 x .. x m_{k-1} first, the pre-tensor m_0 x N_1 x .. x N_{k-1} last)."""
    shape = list(m)
    words = 0
    for v in range(len(m) - 1, 0, -1):
        words += math.prod(shape)
        shape[v] = N[v]
        words += math.prod(shape)
    return 4 * pn * nnz * words


def cpu_baseline(arr, D, pn, G):
    """The oracle (pointwise integer Bareiss + exact interpolation) on the same matrix, all
    host cores."""
    from oracle import det as OD
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        OD.det_pointwise(arr, D, pool=pool)
    t = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pn * G / t, "unit": "modular dets/s (equivalent)", "cores": cores,
            "kind": "oracle",
            "sample": (f"the whole 12x12 trivariate workload once: {int(__import__('numpy').prod([d + 1 for d in D]))} "
                       f"integer-node Bareiss determinants + exact interpolation in {t:.2f} s on "
                       f"{cores} processes ({model}); value = pn*G / wall time, i.e. the same "
                       f"exact polynomial determinant expressed in the GPU metric's unit"),
            "exact_dets_per_s": 1.0 / t}


def bench_batch(args):
    """4096 matrices of uneven order (4..24), variable count (2..3) and degree (1..4) with
    10-40% zero entries, coefficients in [-4096, 4096]: one batched solve (chunked persistent
    launches) against the plain per-matrix path on the same GPU and inputs."""
    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    import workloads as W

    mats = W.config4(count=args.batch_count)
    t0 = time.perf_counter()
    pl = pdm.plan_batch(mats)
    plan_s = time.perf_counter() - t0
    plain = pdm.plan_batch(mats, flags=pdm.BATCH_PLAIN)
    infos = pl.infos
    co, oo = [], []
    c = o = 0
    for a, info in zip(mats, infos):
        co.append(c)
        oo.append(o)
        c += a.size
        o += info["ncoeff"] * info["limbs"]
    dev = torch.device("cuda:0")
    d_coeffs = torch.from_numpy(np.concatenate([a.reshape(-1) for a in mats])).to(dev)
    d_out = torch.empty(o, dtype=torch.int32, device=dev)
    ws = torch.empty(max(infos[0]["workspace_bytes"], plain.infos[0]["workspace_bytes"]),
                     dtype=torch.uint8, device=dev)
    moddets = sum(i["pn"] * i["G"] for i in infos)
    updates = sum(i["pn"] * i["G"] * det_updates(i["n"]) for i in infos)

    def timed(p, steps, warmup):
        for _ in range(warmup):
            pdm.solve_batch_device(p, d_coeffs, co, d_out, oo, workspace=ws)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            pdm.solve_batch_device(p, d_coeffs, co, d_out, oo, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_batched = timed(pl, args.steps, args.warmup)
    ms_plain = timed(plain, max(1, args.steps // 2), 1)
    line = {
        "metric": "modular dets/sec (prime x point), exact poly dets/sec, batched vs plain, 1 GPU",
        "value": moddets / (ms_batched / 1e3), "unit": "modular dets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 (mod p < 2^30)", "data": "synthetic (seeded)",
        "config": {"workload": f"{len(mats)} matrices, n 4..24, 2-3 variables, degree 1-4, "
                               "10-40% zero entries, coefficients U[-4096,4096]",
                   "matrices": len(mats), "modular_dets": moddets, "updates": updates,
                   "chunks_workspace_bytes": infos[0]["workspace_bytes"]},
        "exact_dets_per_s": len(mats) / (ms_batched / 1e3),
        "plain_ms_per_step": ms_plain,
        "batched_over_plain": ms_plain / ms_batched,
        "elimination_updates_per_s": updates / (ms_batched / 1e3),
        "plan_seconds": plan_s,
    }
    print(json.dumps(line), flush=True)


def bench_serving(args):
    """Serving: a Poisson stream of determinant jobs (n 4..32, 2-3 variables, degree 1-5,
    coefficients in [-2^16, 2^16], 1% replaced by 32x32 trivariate degree-5 jobs) through the
    continuous-batching server; the rate is rho times the capacity measured by submitting
    every job at once. Reports p50/p99 latency and throughput per rho."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2010_12117_amd import serving as S

    rng = W.rng_for(5)
    jobs = [W.config5_job(rng) for _ in range(args.jobs)]
    large = sum(1 for a in jobs if a.shape[0] == 32 and a.ndim == 5 and a.shape[2] == 6)
    budget = int(args.serve_budget_gb * (1 << 30))

    def run(rate, label):
        srv = S.Server(memory_budget=budget, slots=args.slots)
        arr = S.poisson_arrivals(np.random.default_rng(77), len(jobs), rate) if rate else None
        t0 = time.perf_counter()
        last = t0
        futs = []

        def progress():
            nonlocal last
            now = time.perf_counter()
            if now - last > 15:
                done = sum(f.done() for f in futs)
                print(f"serving: {label}: {len(futs)} submitted, {done} done, "
                      f"{now - t0:.0f} s", file=sys.stderr, flush=True)
                last = now

        for i, a in enumerate(jobs):
            if arr is not None:
                wait = arr[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            futs.append(srv.submit(a))
            progress()
        for f in futs:
            while True:
                try:
                    f.result(timeout=5)
                    break
                except FutureTimeout:
                    progress()
        makespan = time.perf_counter() - t0
        srv.close()
        st = srv.stats()
        st["makespan_s"] = makespan
        st["jobs_per_s"] = len(jobs) / makespan
        return st

    run(0, "warm-up")  # plans, kernels, allocator
    torch.cuda.synchronize()
    print("serving: warm-up done", file=sys.stderr, flush=True)
    cap = run(0, "capacity")
    capacity = cap["jobs_per_s"]
    print(f"serving: capacity {capacity:.1f} jobs/s", file=sys.stderr, flush=True)
    out = {"capacity": cap}
    for rho in (0.5, 0.8):
        out[f"rho_{rho}"] = run(rho * capacity, f"rho {rho}")
        print(f"serving: rho {rho} done", file=sys.stderr, flush=True)
    line = {
        "metric": "serving: p50/p99 latency and throughput of exact determinant jobs, 1 GPU",
        "value": out["rho_0.8"]["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic (seeded)",
        "config": {"workload": f"{len(jobs)} Poisson-arriving jobs, n 4..32, 2-3 variables, "
                               f"degree 1-5, coefficients U[-2^16,2^16], {large} of them "
                               "32x32 trivariate degree 5",
                   "slots": args.slots, "memory_budget_gb": args.serve_budget_gb},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def det_kernel_name(info):
    n, lanes = info["n"], info["det_lanes"]
    m0 = info["deg"][0] + 1 if info["nvars"] else 1
    paired = 2 <= m0 <= 4  # first-variable points j0, j0 + N0/2 built by two lanes
    fused = ("det_fused_pair_kernel" if paired else "det_fused_kernel") + f"<{n},{lanes}>"
    if info["det_left_looking"]:
        return f"det_ll_kernel<{n}> + repair {fused}"
    return fused


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 solves at config 2, 2 batch solves at config 4)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 20 at config 2, 1 at config 4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="config2", choices=["config2", "config4", "config5"],
                    help="config2: the 12x12 trivariate matrix (default); config4: the batch "
                         "of 4096 uneven matrices, batched against plain")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--jobs", type=int, default=2000, help="serving: number of jobs")
    ap.add_argument("--slots", type=int, default=4, help="serving: jobs in flight")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0,
                    help="serving: device memory for jobs in flight")
    ap.add_argument("--det-lanes", type=int, default=0,
                    help="lanes per determinant (1, 2, 4, 8, 16); 0 = the plan's choice")
    ap.add_argument("--det-form", default="auto", choices=["auto", "left-looking", "exchange"],
                    help="elimination form of the determinant kernel (results are identical)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before the timed loop, copy 1 GiB device to device once (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the determinant path is a single-GPU "
              "kernel pipeline, and no figure at several GPUs is measured", file=sys.stderr)
        sys.exit(2)

    big = args.workload == "config4"
    if args.steps is None:
        args.steps = 2 if big else 200
    if args.warmup is None:
        args.warmup = 1 if big else 20
    if args.workload == "config4":
        bench_batch(args)
        return
    if args.workload == "config5":
        bench_serving(args)
        return

    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    import workloads as W

    arr = W.config2()
    n, deg = 12, (3, 3, 3)
    flags = 0
    if args.det_lanes:
        flags |= pdm.DET_LANES_LOG2(args.det_lanes.bit_length() - 1)
    flags |= {"auto": 0, "left-looking": pdm.DET_LEFT_LOOKING,
              "exchange": pdm.DET_EXCHANGE}[args.det_form]
    # the timed plan records no stage events (each costs a few microseconds of device time
    # between the kernels); a second plan with the library's stage events gives the kernels'
    # own durations over a second pass of the same number of solves
    pl = pdm.plan(n, deg, host_coeffs=arr, flags=flags)
    pl_stages = pdm.plan(n, deg, host_coeffs=arr, flags=flags | pdm.STAGE_TIMING)
    info = pl.info
    pn, G = info["pn"], info["G"]
    dev = torch.device("cuda:0")
    d_coeffs = torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    out = torch.empty((info["ncoeff"], info["limbs"]), dtype=torch.int32, device=dev)
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        pdm.solve_device(pl, d_coeffs, out, ws)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        pdm.solve_device(pl, d_coeffs, out, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps

    # the same solves again with stage events: the duration of each stage's kernels
    for _ in range(max(1, args.warmup // 4)):
        pdm.solve_device(pl_stages, d_coeffs, out, ws)
    torch.cuda.synchronize()
    pl_stages.stage_times()  # discard the warm-up solves
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for i in range(args.steps):
        pdm.solve_device(pl_stages, d_coeffs, out, ws)
    s1.record(stream)
    torch.cuda.synchronize()
    staged_ms_per_step = s0.elapsed_time(s1) / args.steps
    stage_ms, solves = pl_stages.stage_times()
    assert solves == args.steps
    value = pn * G / (ms_per_step / 1e3)

    # roofline of each kernel class from its measured average duration
    per = {k: v / args.steps for k, v in stage_ms.items()}
    nnz = int(np.count_nonzero(np.abs(arr).reshape(n * n, -1).sum(axis=1)))
    det_work = pn * G * det_updates(n)
    det_achieved = det_work / (per["determinants"] / 1e3) / 1e12
    eval_bytes = expand_bytes(pn, nnz, [d + 1 for d in deg], list(info["N"]))
    eval_gbs = eval_bytes / (per["evaluate"] / 1e3) / 1e9
    traffic = (DET_TRAFFIC["bytes"]
               if kernel_sources_hash() == DET_TRAFFIC["sources_sha256_16"] else None)
    det_roof = {"bound": "alu", "achieved": det_achieved, "peak": ALU_PEAK_UPDATES / 1e12,
                "unit": "T elimination-updates/s", "frac": det_achieved / (ALU_PEAK_UPDATES / 1e12),
                "traffic": traffic, "kernel": det_kernel_name(info),
                "work_per_launch": det_work, "avg_ms": per["determinants"]}
    eval_roof = {"bound": "hbm", "achieved": eval_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": eval_gbs / HBM_PEAK_GBS, "traffic": None,
                 "kernel": "expand_kernel<4> (2 launches)", "bytes_per_solve": eval_bytes,
                 "avg_ms": per["evaluate"]}
    dominant = det_roof if per["determinants"] >= per["evaluate"] else eval_roof

    line = {
        "metric": "modular dets/sec (prime x point), exact poly det end to end, 1 GPU",
        "value": value, "unit": "modular dets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 (mod p < 2^30)",
        "data": "synthetic (seeded)",
        "config": {"workload": "12x12 trivariate degree-3 matrix, coefficients U[-1000,1000], "
                               "30% zero entries, 64^3 grid, 7 primes",
                   "n": n, "nvars": 3, "deg": list(deg), "grid": list(info["N"]), "primes": pn,
                   "nonzero_entries": nnz},
        "exact_dets_per_s": 1e3 / ms_per_step,
        "ms_per_step_with_stage_events": staged_ms_per_step,
        "stage_ms": per,
        "roofline": dominant,
        "roofline_other": eval_roof if dominant is det_roof else det_roof,
    }
    if not args.no_cpu_baseline:
        from oracle import plan as PL
        line["cpu_baseline"] = cpu_baseline(arr, PL.det_degree_bound_from_shape(n, deg), pn, G)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
