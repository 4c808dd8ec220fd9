"""Throughput of exact polynomial determinants on one MI355X: batched against plain.

Default workload: 4096 matrices of uneven order (4..24), variable count (2..3) and degree
(1..4 per variable), 10-40% zero entries, coefficients uniform in [-4096, 4096] (seeded). One
step = one solve of the whole batch (reduce, evaluate, determinants, interpolate, reconstruct
for every matrix) with the coefficients already in HBM and warm plans. The batched solve (the
matrices' stages merged into a few launches per chunk) is captured once in a HIP graph and
replayed; the plain path solves the same matrices one by one with the single-matrix launches.
The metric is modular determinants per second (prime x grid point, summed over the batch),
whole job; exact polynomial determinants per second and the batched/plain ratio are reported
beside it. The line also carries the 12 x 12 trivariate single-matrix workload's kernel
roofline (`roofline_config2`) and the times of the 4 x 4 bivariate and 22 x 22 Sylvester
matrices alone (`single_matrix`).

Prints one JSON line (the repository's benchmark contract). Other modes:
  --workload config1   the single 4 x 4 bivariate matrix (16^2 grid, 1 prime; launch-bound)
  --workload config2   the single 12 x 12 trivariate matrix (64^3 grid, 7 primes)
  --workload config3   the single 22 x 22 Sylvester matrix (128^2 grid, 15 primes)
  --workload config5   the serving load (Poisson arrivals, p50/p99 latency)
  --calibrate-alu      vector-ALU throughput probes (one JSON line)
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import statistics
import sys
import time
from concurrent.futures import TimeoutError as FutureTimeout

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peaks of MI355X (published figures): 256 CUs at 2.4 GHz, HBM 8 TB/s. The elimination is
# bound by integer vector arithmetic. 64-bit integer multiply-adds (v_mad_u64_u32) and 32-bit
# multiplies (v_mul_lo_u32) issue at the fp64 vector rate (78.6 TFLOP/s = 64 lane-FMAs per
# clock per CU); plain 32-bit operations at the fp32 vector rate (157.3 TFLOP/s = 128 lane-ops
# per clock per CU). So one lane-op costs 1/64 or 1/128 of a CU-clock.
HBM_PEAK_GBS = 8000.0
CU, CLOCK_HZ = 256, 2.4e9
MULT_CLK, PLAIN_CLK = 1 / 64, 1 / 128
# A single-step (Chio) update, 4 multiply-class + 1 plain op, would peak at 14.2 per
# CU-clock, 8.74e12/s: the ceiling of a one-column-per-step elimination, kept for comparison.
SINGLE_STEP_PEAK_UPDATES = CU * CLOCK_HZ / (4 * MULT_CLK + 1 * PLAIN_CLK)


def det_issue_clk(n: int) -> float:
    """Minimal issue cost in CU-clocks per lane of one determinant of order n by two-column
    condensation, the kernels' algorithm: at each order m = n, n - 2, ... >= 3, the (m-2)^2
    three-product updates (4 v_mad_u64_u32 + 1 v_mul_lo_u32 + 1 mask each) and, for each of
    the m - 2 columns, its two factors (two reductions of two products, 3 mad + 1 mul_lo + 1
    mask each, two conditional subtractions of 2 ops and one negation); an even order ends with
    a 2 x 2 determinant (3 mad + 1 mul_lo, a conditional subtraction). Pivot search, the
    denominators and the evaluation fused into the same kernel are not counted."""
    clk = 0.0
    m = n
    while m >= 3:
        clk += (m - 2) ** 2 * (5 * MULT_CLK + 1 * PLAIN_CLK)
        clk += (m - 2) * (8 * MULT_CLK + 7 * PLAIN_CLK)
        m -= 2
    if m == 2:
        clk += 4 * MULT_CLK + 2 * PLAIN_CLK
    return clk


def eval_issue_clk(m0: int) -> float:
    """Minimal issue cost in CU-clocks per lane of evaluating one entry at one point along the
    first variable (m0 coefficients), as the elimination kernel does before eliminating: with
    2..6 coefficients the values at j and j + N/2 share the even and odd sums, so a point costs
    one reduction of two or three products (3 or 4 mad + 1 mul_lo + a conditional subtraction)
    and one addition; otherwise ceil(m0/2) two-product reductions and one modular addition
    (3 plain) between each."""
    if m0 <= 1:
        return 0.0
    mm2 = 4 * MULT_CLK + 2 * PLAIN_CLK
    if 2 <= m0 <= 4:
        return mm2 + PLAIN_CLK
    if m0 <= 6:
        return mm2 + MULT_CLK + PLAIN_CLK
    r = (m0 + 1) // 2
    return r * mm2 + (r - 1) * 3 * PLAIN_CLK


def alu_peak_updates(work):
    """Peak elimination-updates per second (the determinant's sum_{m<n} m^2 modular
    multiply-subtracts, the algorithmic unit) of the elimination launches of a mix of
    determinants, `work` = [(n, dets, nonzero entries, m0)]: the chip issuing, on every CU
    every clock, the launches' minimal instruction mix, which is the two-column elimination
    and the evaluation of each nonzero entry along the first variable that the same kernel
    does first."""
    upd = sum(d * det_updates(n) for n, d, _, _ in work)
    clk = sum(d * (det_issue_clk(n) + nnz * eval_issue_clk(m0)) for n, d, nnz, m0 in work)
    return upd / clk * CU * CLOCK_HZ if clk else 0.0


def alu_peak_updates_elimination_only(work):
    """The same peak with the elimination's instructions alone (no evaluation)."""
    upd = sum(d * det_updates(n) for n, d, _, _ in work)
    clk = sum(d * det_issue_clk(n) for n, d, _, _ in work)
    return upd / clk * CU * CLOCK_HZ if clk else 0.0


def nonzero_entries(a) -> int:
    """Entries of a coefficient array [n][n][...] with a nonzero coefficient."""
    import numpy as np
    n = a.shape[0]
    return int(np.count_nonzero(np.abs(a).reshape(n * n, -1).sum(axis=1)))


# HBM bytes per launch of the 12 x 12 trivariate workload's elimination kernel, from rocprofv3
# FETCH_SIZE (22,841 KiB) and WRITE_SIZE (14,336 KiB) passes, scaled by what the same counters
# read for a 1 GiB device copy (FETCH x 2.0, WRITE x 1.0), valid only for the kernel sources and
# tuning table they were taken with (their hash). The hash was last moved by the wave requests
# of the 2-lane kernels at orders 13 and 16, which leave that kernel's machine code as it was
# (its assembly compared instruction by instruction).
DET_TRAFFIC = {"sources_sha256_16": "e31a61af6229ffb3", "bytes": 46.78e6 + 14.68e6}

STAGES = ("reduce", "evaluate", "determinants", "finalize", "interpolate", "reconstruct")


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


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


def host_cpu():
    cores = len(os.sched_getaffinity(0))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def det_kernel_name(info, batched=False):
    n, lanes = info["n"], info["det_lanes"]
    m0 = info["deg"][0] + 1 if info["nvars"] else 1
    paired = 2 <= m0 <= 6  # first-variable points j0, j0 + N0/2 built by two lanes
    terms = 2 if m0 <= 4 else 3  # even or odd terms summed by each of the two
    fused = ("det_fused_pair" if paired else "det_fused") + ("_batch" if batched else "") + \
        (f"_kernel<{n},{lanes},{terms}>" if paired else f"_kernel<{n},{lanes}>")
    if info["det_left_looking"]:
        return f"det_ll_kernel<{n}> + repair {fused}"
    return fused


# ------------------------------------------------------------------------------- oracle legs
def _oracle_one(args):
    from oracle import det as OD
    from oracle import plan as PL
    i, a = args
    n = a.shape[0]
    deg = [a.shape[2 + v] - 1 for v in range(a.ndim - 2)]
    OD.det_pointwise(a, PL.det_degree_bound_from_shape(n, deg))
    return i


def oracle_cost_s(n, deg):
    """Rough single-core seconds of the pointwise oracle: node determinants plus the exact
    inverse Vandermonde matrices (measured on this repository's oracle, within a factor 2)."""
    nodes = math.prod(n * d + 1 for d in deg)
    return nodes * n ** 3 * 0.4e-6 + sum(1.5 * ((n * d) / 64) ** 3 for d in deg)


def cpu_baseline_batch(mats, infos, budget_s):
    """The oracle on a bounded sample of the batch: matrices whose estimated oracle cost is
    below one core-second, in seeded random order, solved by a pool over all host cores until
    `budget_s` seconds have passed."""
    import numpy as np
    cores, model = host_cpu()
    cheap = [i for i, a in enumerate(mats)
             if oracle_cost_s(a.shape[0], [x - 1 for x in a.shape[2:]]) < 1.0]
    order = list(np.random.default_rng(20).permutation(cheap))
    ctx = mp.get_context("spawn")
    done = []
    t0 = time.perf_counter()
    t_last = t0
    with ctx.Pool(cores) as pool:
        it = pool.imap_unordered(_oracle_one, ((int(i), mats[i]) for i in order), chunksize=1)
        while True:
            try:
                i = it.next(timeout=max(0.01, budget_s - (time.perf_counter() - t0)))
            except (StopIteration, mp.TimeoutError):
                break
            done.append(i)
            t_last = time.perf_counter()
            if t_last - t0 >= budget_s:
                break
        pool.terminate()
    t = t_last - t0
    moddets = sum(infos[i]["pn"] * infos[i]["G"] for i in done)
    return {"value": moddets / t, "unit": "modular dets/s (equivalent)", "cores": cores,
            "kind": "oracle",
            "sample": (f"{len(done)} of the {len(mats)} matrices (seeded random order among the "
                       f"{len(cheap)} whose pointwise oracle takes under about one core-second), "
                       f"solved exactly in {t:.1f} s on {cores} processes ({model}); value = "
                       "their pn*G summed / wall time, the same exact determinants expressed in "
                       "the GPU metric's unit"),
            "exact_dets_per_s": len(done) / t}


def cpu_baseline_single(arr, D, pn, G):
    """The oracle (pointwise integer Bareiss + exact interpolation) on the whole matrix on all
    host cores, plus a single-core figure extrapolated from (up to) 2000 of its node
    determinants."""
    import numpy as np
    from oracle import det as OD
    cores, model = host_cpu()
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        OD.det_pointwise(arr, D, pool=pool)
    t = time.perf_counter() - t0
    nodes = OD.node_matrices(arr, D).reshape((-1,) + arr.shape[:2])
    sample = [[[int(x) for x in r] for r in m] for m in nodes[:2000]]
    t1 = time.perf_counter()
    OD._det_rows(sample)
    single = (time.perf_counter() - t1) * len(nodes) / len(sample)
    return {"value": pn * G / t, "unit": "modular dets/s (equivalent)", "cores": cores,
            "kind": "oracle",
            "sample": (f"the whole {arr.shape[0]}x{arr.shape[0]} matrix once: "
                       f"{int(np.prod([d + 1 for d in D]))} integer-node Bareiss determinants + "
                       f"exact interpolation in {t:.2f} s on {cores} processes ({model}); "
                       "value = pn*G / wall time"),
            "exact_dets_per_s": 1.0 / t,
            "single_core_node_dets_s_extrapolated": single}


# ----------------------------------------------------------------------- timing helpers
def timed_each(fn, steps, stream):
    """Run fn() `steps` times between events on `stream`; returns (total ms, per-step ms)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]), per


def timed_total(fn, reps, stream):
    """ms of `reps` calls of fn() between one pair of events on `stream` (no event between the
    calls: each event costs a few microseconds of device time)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def stage_kernel_ms(pl, d_coeffs, out, ws, reps, stream):
    """Mean device ms of each stage's kernels, each stage run `reps` times back to back on a
    finished workspace (polydet_solve_stages) between two events: kernel durations without
    any event between the kernels of a stage or between the repetitions."""
    import paper_2010_12117_amd as pdm
    res = {}
    for s, name in enumerate(STAGES):
        total = timed_total(lambda: pdm.solve_stages_device(pl, s, s + 1, d_coeffs, out, ws,
                                                            stream=stream), reps, stream)
        res[name] = total / reps
    return res


# ------------------------------------------------------------------------------ workloads
def config2_roofline(reps=50):
    """The 12 x 12 trivariate matrix: per-stage kernel durations and the elimination kernel's
    ALU roofline."""
    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    import workloads as W

    arr = W.config2()
    n, deg = 12, (3, 3, 3)
    pl = pdm.plan(n, deg, host_coeffs=arr)
    info = pl.info
    pn, G = info["pn"], info["G"]
    dev = torch.device("cuda:0")
    d = torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
    out = torch.empty((info["ncoeff"], info["limbs"]), dtype=torch.int32, device=dev)
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(20):
        pdm.solve_device(pl, d, out, ws)
    total = timed_total(lambda: pdm.solve_device(pl, d, out, ws), reps, stream)
    _, per = timed_each(lambda: pdm.solve_device(pl, d, out, ws), reps, stream)
    stage = stage_kernel_ms(pl, d, out, ws, reps, stream)
    nnz = int(np.count_nonzero(np.abs(arr).reshape(n * n, -1).sum(axis=1)))
    work = pn * G * det_updates(n)
    achieved = work / (stage["determinants"] / 1e3) / 1e12
    mix = [(n, pn * G, nnz, deg[0] + 1)]
    peak = alu_peak_updates(mix) / 1e12
    traffic = (DET_TRAFFIC["bytes"]
               if kernel_sources_hash() == DET_TRAFFIC["sources_sha256_16"] else None)
    eval_bytes = expand_bytes(pn, nnz, [x + 1 for x in deg], list(info["N"]))
    return {
        "workload": "12x12 trivariate degree-3 matrix, coefficients U[-1000,1000], 30% zero "
                    "entries, 64^3 grid, 7 primes",
        "ms_per_solve": total / reps, "ms_per_solve_median": statistics.median(per),
        "modular_dets_per_s": pn * G / (total / reps / 1e3),
        "exact_dets_per_s": 1e3 / (total / reps),
        "stage_kernel_ms": stage,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "T elimination-updates/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": det_kernel_name(info),
                     "work_per_launch": work, "avg_ms": stage["determinants"],
                     "frac_elimination_only": achieved / (alu_peak_updates_elimination_only(mix) / 1e12),
                     "frac_of_single_step_peak": achieved / (SINGLE_STEP_PEAK_UPDATES / 1e12)},
        "evaluate_roofline": {"bound": "hbm", "bytes_per_solve": eval_bytes,
                              "achieved": eval_bytes / (stage["evaluate"] / 1e3) / 1e9,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": eval_bytes / (stage["evaluate"] / 1e3) / 1e9 / HBM_PEAK_GBS},
    }, (arr, info)


def bench_batch(args):
    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    import workloads as W

    mats = W.config4(count=args.batch_count)
    t0 = time.perf_counter()
    pl = pdm.plan_batch(mats)
    plan_s = time.perf_counter() - t0
    plain = pdm.plan_batch(mats, flags=pdm.BATCH_PLAIN)
    serial = None if args.no_extras else plan_batch_streams(pdm, mats, 1)  # one stream
    timing = pdm.plan_batch(mats, flags=pdm.STAGE_TIMING)
    progress(f"plans built ({plan_s:.1f} s for the batched one)")
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
    ws = torch.empty(max([infos[0]["workspace_bytes"], plain.infos[0]["workspace_bytes"],
                          timing.infos[0]["workspace_bytes"]] +
                         ([serial.infos[0]["workspace_bytes"]] if serial is not None else [])),
                     dtype=torch.uint8, device=dev)
    moddets = sum(i["pn"] * i["G"] for i in infos)
    updates = sum(i["pn"] * i["G"] * det_updates(i["n"]) for i in infos)
    stream = torch.cuda.Stream()

    def solve(p):
        pdm.solve_batch_device(p, d_coeffs, co, d_out, oo, workspace=ws, stream=stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            solve(pl)
        stream.synchronize()
        ref = d_out.clone()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            solve(pl)
        progress("warm-up and graph capture done")
        total, per = timed_each(graph.replay, args.steps, stream)  # the timed region
        ms_graph = total / args.steps
        assert torch.equal(d_out, ref), "graph replay differs from the eager solve"
        progress(f"batched (graph): {ms_graph:.1f} ms per solve")
        per_eager = [float("nan")]
        if args.eager_steps > 0:
            _, per_eager = timed_each(lambda: solve(pl), args.eager_steps, stream)
            progress(f"batched (eager): {statistics.median(per_eager):.1f} ms per solve")
        for _ in range(args.warmup):
            solve(plain)
        _, per_plain = timed_each(lambda: solve(plain), args.plain_steps, stream)
        assert torch.equal(d_out, ref), "plain path differs from the batched solve"
        progress(f"plain: {statistics.median(per_plain):.1f} ms per solve")
        per_serial = [float("nan")]
        if serial is not None:
            solve(serial)
            _, per_serial = timed_each(lambda: solve(serial), max(1, args.eager_steps), stream)
            assert torch.equal(d_out, ref), "batched solve on one stream differs"
            progress(f"batched on one stream (eager): {statistics.median(per_serial):.1f} ms")
        solve(timing)
        timing.stage_times()
        solve(timing)
        stage_ms, solves = timing.stage_times()
        assert solves == 1
    torch.cuda.synchronize()
    det_ms = stage_ms["determinants"]
    achieved = updates / (det_ms / 1e3) / 1e12
    mix = [(i["n"], i["pn"] * i["G"], nonzero_entries(a), (a.shape[2] if a.ndim > 2 else 1))
           for a, i in zip(mats, infos)]
    peak = alu_peak_updates(mix) / 1e12
    ms_plain = statistics.median(per_plain)
    ms_med = statistics.median(per)
    line = {
        "metric": "modular dets/sec (prime x point) and exact poly dets/sec, batched vs plain, "
                  "1 GPU",
        "value": moddets / (ms_graph / 1e3), "unit": "modular dets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph,
        "ms_per_step_median": ms_med, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 (mod p < 2^30)", "data": "synthetic (seeded)",
        "config": {"workload": f"{len(mats)} matrices, n 4..24, 2-3 variables, degree 1-4 per "
                               "variable, 10-40% zero entries, coefficients U[-4096,4096]",
                   "matrices": len(mats), "modular_dets": moddets, "elimination_updates": updates,
                   "workspace_bytes": infos[0]["workspace_bytes"]},
        "exact_dets_per_s": len(mats) / (ms_graph / 1e3),
        "batched": {"graph_ms_mean": ms_graph, "graph_ms_median": ms_med,
                    "graph_ms_all": per, "eager_ms_median": statistics.median(per_eager),
                    "eager_steps": args.eager_steps},
        "plain": {"ms_median": ms_plain, "ms_mean": statistics.fmean(per_plain),
                  "ms_all": per_plain, "steps": args.plain_steps},
        "plain_ms_per_step": ms_plain,
        "batched_over_plain": ms_plain / ms_med,
        "stage_ms_batched": stage_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "T elimination-updates/s", "frac": achieved / peak,
                     "frac_elimination_only": achieved / (alu_peak_updates_elimination_only(mix) / 1e12),
                     "frac_of_single_step_peak": achieved / (SINGLE_STEP_PEAK_UPDATES / 1e12),
                     "traffic": None,
                     "kernel": "det_fused(_pair)_batch_kernel<n,lanes>: every elimination "
                               "launch of one batched solve (order 24, 4 lanes, two terms per "
                               "lane: det_fused_pair_kernel<24,4,2> once per matrix)",
                     "work_per_launch": updates, "avg_ms": det_ms,
                     "avg_ms_source": "HIP events before and after each elimination launch of "
                                      "one batched solve (sum)"},
        "plan_seconds": plan_s,
        "batched_one_stream_eager_ms_median": statistics.median(per_serial),
    }
    if not args.no_extras:
        progress("small-matrix subset")
        line["small_subset"] = bench_small_subset(mats, args)
    if not args.no_extras:
        progress("batch done; 12x12 trivariate roofline")
        c2, (arr2, info2) = config2_roofline()
        line["roofline_config2"] = c2
        progress("the 4x4 bivariate and 22x22 Sylvester matrices")
        line["single_matrix"] = {w: single_summary(w) for w in ("config1", "config3")}
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        line["cpu_baseline"] = cpu_baseline_batch(mats, infos, args.cpu_budget)
    print(json.dumps(line), flush=True)


def plan_batch_streams(pdm, mats, streams):
    """A batched plan on `streams` streams: 1 runs every launch on the caller's stream, 2
    (the default) runs consecutive chunks side by side (the library reads
    POLYDET_BATCH_STREAMS when the plan is made)."""
    old = os.environ.get("POLYDET_BATCH_STREAMS")
    os.environ["POLYDET_BATCH_STREAMS"] = str(streams)
    try:
        return pdm.plan_batch(mats)
    finally:
        if old is None:
            del os.environ["POLYDET_BATCH_STREAMS"]
        else:
            os.environ["POLYDET_BATCH_STREAMS"] = old


def bench_small_subset(mats, args, max_n=12):
    """Batched against plain on the matrices of order <= max_n alone (launch-bound work: few
    determinants per matrix), both replayed from captured graphs, median of --steps solves."""
    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    sub = [a for a in mats if a.shape[0] <= max_n]
    pl = pdm.plan_batch(sub)
    plain = pdm.plan_batch(sub, flags=pdm.BATCH_PLAIN)
    co, oo = [], []
    c = o = 0
    for a, info in zip(sub, pl.infos):
        co.append(c)
        oo.append(o)
        c += a.size
        o += info["ncoeff"] * info["limbs"]
    dev = torch.device("cuda:0")
    d_coeffs = torch.from_numpy(np.concatenate([a.reshape(-1) for a in sub])).to(dev)
    d_out = torch.empty(o, dtype=torch.int32, device=dev)
    ws = torch.empty(max(pl.infos[0]["workspace_bytes"], plain.infos[0]["workspace_bytes"]),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(stream):
        for name, p in (("batched", pl), ("plain", plain)):
            def solve(p=p):
                pdm.solve_batch_device(p, d_coeffs, co, d_out, oo, workspace=ws, stream=stream)
            for _ in range(2):
                solve()
            stream.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                solve()
            _, per = timed_each(graph.replay, max(5, args.steps), stream)
            res[name] = statistics.median(per)
            if name == "batched":
                ref = d_out.clone()
            else:
                assert torch.equal(d_out, ref), "plain differs from batched on the subset"
    moddets = sum(i["pn"] * i["G"] for i in pl.infos)
    return {"workload": f"the {len(sub)} matrices of order <= {max_n} of the batch",
            "matrices": len(sub), "modular_dets": moddets,
            "batched_ms_median": res["batched"], "plain_ms_median": res["plain"],
            "batched_over_plain": res["plain"] / res["batched"],
            "value_batched": moddets / (res["batched"] / 1e3)}


# The single-matrix workloads: generator name in workloads/ and description.
SINGLE_WORKLOADS = {
    "config1": ("config1", "4x4 bivariate degree-2 matrix, coefficients U[-10,10], dense, "
                           "16^2 grid, 1 prime"),
    "config2": ("config2", "12x12 trivariate degree-3 matrix, coefficients U[-1000,1000], 30% "
                           "zero entries, 64^3 grid, 7 primes"),
    "config3": ("config3a", "22x22 Sylvester matrix of two polynomials of degree 12 and 10 in x "
                            "whose coefficients are dense bivariate degree-4 polynomials with "
                            "coefficients U[-32768,32768], 128^2 grid, 15 primes"),
}


def graph_replay_ms(pl, d, out, ws, reps):
    """ms per solve of `reps` replays of one solve captured in a HIP graph (no host launch
    overhead), between one pair of events; the replays equal the eager solve."""
    import torch

    import paper_2010_12117_amd as pdm
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pdm.solve_device(pl, d, out, ws, stream=stream)
    stream.synchronize()
    want = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        pdm.solve_device(pl, d, out, ws, stream=stream)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
        total = timed_total(g.replay, reps, stream)
    if not torch.equal(out, want):
        raise RuntimeError("graph replay differs from the eager solve")
    return total / reps


def bench_single(args):
    """One matrix alone: the 4 x 4 bivariate (config1), 12 x 12 trivariate (config2) or 22 x 22
    Sylvester (config3) workload; prints its JSON line."""
    print(json.dumps(single_line(args)), flush=True)


def single_summary(workload, steps=50):
    """The main figures of a single-matrix workload's line (no CPU baseline), for the batch
    line."""
    import types
    a = types.SimpleNamespace(workload=workload, det_lanes=None, det_form="auto",
                              calibrate_copy=False, warmup=5, steps=steps, no_cpu_baseline=True)
    d = single_line(a)
    return {"workload": d["config"]["workload"], "solves": steps,
            "ms_per_solve": d["ms_per_step"], "ms_per_solve_median": d["ms_per_step_median"],
            "ms_per_solve_graph": d["ms_per_step_graph"], "modular_dets_per_s": d["value"],
            "exact_dets_per_s": d["exact_dets_per_s"], "stage_kernel_ms": d["stage_kernel_ms"],
            "roofline_frac": d["roofline"]["frac"], "det_kernel": d["roofline"]["kernel"]}


def single_line(args):
    """The JSON line of one single-matrix workload (bench_single)."""
    import numpy as np
    import torch

    import paper_2010_12117_amd as pdm
    import workloads as W
    from oracle import plan as PL

    gen, description = SINGLE_WORKLOADS[args.workload]
    arr = getattr(W, gen)()
    n = arr.shape[0]
    deg = tuple(x - 1 for x in arr.shape[2:])
    flags = 0
    if args.det_lanes:
        flags |= pdm.DET_LANES_LOG2(args.det_lanes.bit_length() - 1)
    flags |= {"auto": 0, "left-looking": pdm.DET_LEFT_LOOKING,
              "exchange": pdm.DET_EXCHANGE}[args.det_form]
    pl = pdm.plan(n, deg, host_coeffs=arr, flags=flags)
    info = pl.info
    pn, G = info["pn"], info["G"]
    dev = torch.device("cuda:0")
    d = torch.from_numpy(np.ascontiguousarray(arr)).to(dev)
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
        pdm.solve_device(pl, d, out, ws)
    # the timed region: K solves between one pair of events; then K more with an event after
    # each for the median
    total = timed_total(lambda: pdm.solve_device(pl, d, out, ws), args.steps, stream)
    ms = total / args.steps
    _, per = timed_each(lambda: pdm.solve_device(pl, d, out, ws), args.steps, stream)
    graph_ms = graph_replay_ms(pl, d, out, ws, args.steps)
    stage = stage_kernel_ms(pl, d, out, ws, args.steps, stream)
    nnz = int(np.count_nonzero(np.abs(arr).reshape(n * n, -1).sum(axis=1)))
    work = pn * G * det_updates(n)
    achieved = work / (stage["determinants"] / 1e3) / 1e12
    mix = [(n, pn * G, nnz, deg[0] + 1)]
    peak = alu_peak_updates(mix) / 1e12
    traffic = (DET_TRAFFIC["bytes"]
               if args.workload == "config2"
               and kernel_sources_hash() == DET_TRAFFIC["sources_sha256_16"] else None)
    eval_bytes = expand_bytes(pn, nnz, [x + 1 for x in deg], list(info["N"]))
    line = {
        "metric": "modular dets/sec (prime x point), exact poly det end to end, 1 GPU",
        "value": pn * G / (ms / 1e3), "unit": "modular dets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "ms_per_step_median": statistics.median(per), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 (mod p < 2^30)",
        "data": "synthetic (seeded)",
        "config": {"workload": description,
                   "n": n, "nvars": len(deg), "deg": list(deg), "grid": list(info["N"]),
                   "primes": pn, "nonzero_entries": nnz},
        "exact_dets_per_s": 1e3 / ms,
        "ms_per_step_graph": graph_ms,
        "stage_kernel_ms": stage,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "T elimination-updates/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": det_kernel_name(info),
                     "work_per_launch": work, "avg_ms": stage["determinants"],
                     "frac_elimination_only": achieved / (alu_peak_updates_elimination_only(mix) / 1e12),
                     "frac_of_single_step_peak": achieved / (SINGLE_STEP_PEAK_UPDATES / 1e12)},
    }
    if eval_bytes and stage["evaluate"] > 0:
        gbs = eval_bytes / (stage["evaluate"] / 1e3) / 1e9
        line["roofline_other"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                                  "kernel": "expand_kernel (evaluation passes)",
                                  "bytes_per_solve": eval_bytes, "avg_ms": stage["evaluate"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_single(arr, PL.det_degree_bound_from_shape(n, deg),
                                                   pn, G)
    return line


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
        srv = S.Server(memory_budget=budget, slots=args.slots, policy=args.policy)
        arr = S.poisson_arrivals(np.random.default_rng(77), len(jobs), rate) if rate else None
        t0 = time.perf_counter()
        last = t0
        futs = []

        def tick():
            nonlocal last
            now = time.perf_counter()
            if now - last > 15:
                done = sum(f.done() for f in futs)
                progress(f"serving: {label}: {len(futs)} submitted, {done} done, {now - t0:.0f} s")
                last = now

        for i, a in enumerate(jobs):
            if arr is not None:
                wait = arr[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            futs.append(srv.submit(a))
            tick()
        for f in futs:
            while True:
                try:
                    f.result(timeout=5)
                    break
                except FutureTimeout:
                    tick()
        makespan = time.perf_counter() - t0
        srv.close()
        st = srv.stats()
        st["makespan_s"] = makespan
        st["jobs_per_s"] = len(jobs) / makespan
        return st

    run(0, "warm-up")  # plans, kernels, allocator
    torch.cuda.synchronize()
    progress("serving: warm-up done")
    cap = run(0, "capacity")
    capacity = cap["jobs_per_s"]
    progress(f"serving: capacity {capacity:.1f} jobs/s")
    out = {"capacity": cap}
    for rho in (0.5, 0.8):
        out[f"rho_{rho}"] = run(rho * capacity, f"rho {rho}")
        progress(f"serving: rho {rho} done")
    line = {
        "metric": "serving: p50/p99 latency and throughput of exact determinant jobs, 1 GPU",
        "value": out["rho_0.8"]["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic (seeded)",
        "config": {"workload": f"{len(jobs)} Poisson-arriving jobs, n 4..32, 2-3 variables, "
                               f"degree 1-5, coefficients U[-2^16,2^16], {large} of them "
                               "32x32 trivariate degree 5",
                   "slots": args.slots, "memory_budget_gb": args.serve_budget_gb,
                   "policy": args.policy},
        "results": out,
    }
    print(json.dumps(line), flush=True)


def cpu_single_core(args):
    """The oracle (pointwise integer Bareiss + exact interpolation) in one process, on the
    single-matrix workloads: the 4x4 bivariate matrix, the 12x12 trivariate one and the 22x22
    Sylvester matrix, whole; one JSON line with the seconds of each and their modular
    determinants per second in the GPU metric's unit."""
    import workloads as W
    from oracle import det as OD
    from oracle import plan as PL
    cores, model = host_cpu()
    out = {}
    for name, make in (("4x4 bivariate degree 2", W.config1),
                       ("12x12 trivariate degree 3", W.config2),
                       ("22x22 Sylvester, bivariate degree 4 entries", W.config3a)):
        arr = make()
        n = arr.shape[0]
        deg = [x - 1 for x in arr.shape[2:]]
        D = PL.det_degree_bound_from_shape(n, deg)
        t0 = time.perf_counter()
        OD.det_pointwise(arr, D)
        t = time.perf_counter() - t0
        import paper_2010_12117_amd as pdm
        info = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY).info
        out[name] = {"seconds": t, "modular_dets_per_s_equivalent": info["pn"] * info["G"] / t,
                     "pn": info["pn"], "G": info["G"]}
        progress(f"oracle, one core: {name}: {t:.1f} s")
    print(json.dumps({"metric": "oracle on one host core (exact determinant, whole matrix)",
                      "cores_used": 1, "host_cores": cores, "cpu": model, "results": out}),
          flush=True)


def calibrate_alu(args):
    """Vector-ALU throughput probes (include/polydet_calibrate.h) and the elimination update's
    peak derived from the published rates, beside the measured update rate."""
    import ctypes

    import torch

    import paper_2010_12117_amd as pdm
    lib = pdm.load_library()
    lib.polydet_calibrate_alu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    lib.polydet_calibrate_alu.restype = ctypes.c_int
    names = ["mad_u64_u32", "mul_lo_u32", "add_u32", "elimination_update", "fma_f64", "fma_f32",
             "two_step_update", "update_64bit"]
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    out = {}
    for probe, name in enumerate(names):
        best = 0.0
        for _ in range(3):
            r = ctypes.c_double()
            st = lib.polydet_calibrate_alu(probe, args.probe_blocks, args.probe_iters,
                                           ctypes.byref(r), ctypes.c_void_p(stream.cuda_stream))
            if st != 0:
                raise RuntimeError(f"probe {name}: status {st}")
            best = max(best, r.value)
        out[name] = {"ops_per_s": best, "per_clk_per_cu": best / (CU * CLOCK_HZ)}
        progress(f"{name}: {best / 1e12:.2f} T/s")
    mad, mul = out["mad_u64_u32"]["per_clk_per_cu"], out["mul_lo_u32"]["per_clk_per_cu"]
    add = out["add_u32"]["per_clk_per_cu"]
    mix = 1.0 / (3 / mad + 1 / mul + 1 / add)  # updates per clock per CU from the measured rates
    line = {"metric": "vector-ALU throughput probes", "unit": "ops/s", "probes": out,
            "blocks": args.probe_blocks, "iters_per_thread": args.probe_iters,
            "update_peak_derived": SINGLE_STEP_PEAK_UPDATES,
            "two_step_update_peak_derived": CU * CLOCK_HZ / (5 * MULT_CLK + 2 * PLAIN_CLK),
            "update_peak_from_measured_instruction_rates": mix * CU * CLOCK_HZ,
            "update_measured": out["elimination_update"]["ops_per_s"],
            "clock_assumed_hz": CLOCK_HZ, "cus": CU}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 5 batch solves; 200 for a single matrix)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 1 batch solve; 20 for a single matrix)")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="timed solves of the plain per-matrix path (default: --steps)")
    ap.add_argument("--eager-steps", type=int, default=2,
                    help="timed eager (not graph-replayed) batched solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="batch workload: only the batched and plain solves and the stage-timed "
                         "pass (no 4-stream, subset or single-matrix figures; for kernel traces)")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of the oracle on the host (batch workload)")
    ap.add_argument("--workload", default="config4",
                    choices=["config4", "config1", "config2", "config3", "config5"],
                    help="config4: the batch of 4096 uneven matrices, batched against plain "
                         "(default); config2: the 12x12 trivariate matrix; config5: serving")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--jobs", type=int, default=2000, help="serving: number of jobs")
    ap.add_argument("--slots", type=int, default=4, help="serving: jobs in flight")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0,
                    help="serving: device memory for jobs in flight")
    ap.add_argument("--policy", default="sjf", choices=["sjf", "fifo"],
                    help="serving: admission order")
    ap.add_argument("--det-lanes", type=int, default=0,
                    help="config2: lanes per determinant (1, 2, 4, 8, 16); 0 = the plan's choice")
    ap.add_argument("--det-form", default="auto", choices=["auto", "left-looking", "exchange"],
                    help="config2: elimination form of the determinant kernel")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="config2: copy 1 GiB device to device once first (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--calibrate-alu", action="store_true",
                    help="run the vector-ALU throughput probes instead of a workload")
    ap.add_argument("--cpu-single-core", action="store_true",
                    help="time the oracle in one process on the single-matrix workloads")
    ap.add_argument("--probe-blocks", type=int, default=8192)
    ap.add_argument("--probe-iters", type=int, default=4096)
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the determinant path is a single-GPU "
              "kernel pipeline, and no figure at several GPUs is measured", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_alu:
        calibrate_alu(args)
        return
    if args.cpu_single_core:
        cpu_single_core(args)
        return
    single = args.workload in SINGLE_WORKLOADS
    if args.steps is None:
        args.steps = 200 if single else 5
    if args.warmup is None:
        args.warmup = 20 if single else 1
    if args.plain_steps is None:
        args.plain_steps = args.steps
    if args.workload == "config4":
        bench_batch(args)
    elif args.workload == "config5":
        bench_serving(args)
    else:
        bench_single(args)


if __name__ == "__main__":
    main()
