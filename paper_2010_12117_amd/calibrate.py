"""Measures the rates of the running-time prediction (polydet_rates in include/polydet.h).

For every matrix order n in 2..32 and class (a first variable with 2..4 coefficients, whose
evaluation is paired with two terms per lane, or any other), a probe matrix with at least `min_dets` modular
determinants per solve is solved once; then each stage is run again `reps` times by itself on
the finished workspace (polydet_solve_stages) between two HIP events, which gives the stage's
kernel time without events between its kernels. The elimination's rate is the probe's
elimination updates over its determinants-stage time. The other stages' rates and the cost of
one launch are fitted by least squares to every probe's stage times and stage work (the terms
listed with polydet_rates). The result is written as the table that binding.py installs at
load time (rates_gfx950.json next to this file).

Usage (on the GPU): python -m paper_2010_12117_amd.calibrate --out FILE [--orders 2-32]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import binding as B

CLASSES = ("paired", "other")


def probe_matrix(n: int, cls: str, min_dets: int, rng: np.random.Generator) -> np.ndarray:
    """Random n x n matrix of the class with at least min_dets modular dets per solve: a first
    variable with 4 coefficients (class "paired") or 6 (class "other": paired with three
    terms per lane), a quarter of the entries zero."""
    first = 3 if cls == "paired" else 5
    arr = None
    for deg in ((first, 1), (first, 2), (first, 1, 1), (first, 2, 1), (first, 2, 2),
                (first, 3, 2), (first, 3, 3), (first, 4, 3), (first, 4, 4)):
        arr = rng.integers(-64, 65, size=(n, n) + tuple(d + 1 for d in deg), dtype=np.int64)
        arr[rng.random((n, n)) < 0.25] = 0
        info = B.plan(n, deg, host_coeffs=arr, flags=B.HOST_ONLY).info
        if info["pn"] * info["G"] >= min_dets:
            return arr
    return arr


def stage_work(info: dict) -> dict:
    """The work terms of each stage, as the prediction counts them (predict.cpp)."""
    pn, ns, k = info["pn"], info["nslots"], info["nvars"]
    T = int(np.prod([d + 1 for d in info["deg"]])) if k else 1
    m = [d + 1 for d in info["deg"]]
    N, D = list(info["N"]), list(info["D"])
    red = 8.0 * ns * T + 4.0 * pn * ns * T
    box, ev, ev_l = float(T), 0.0, 0
    for v in range(k - 1, 0, -1):  # fused: the first variable is evaluated in the elimination
        out = box / m[v] * N[v]
        ev += 4.0 * pn * ns * (box + out)
        box = out
        ev_l += 1
    it, it_l, cur = 0.0, 0, float(info["G"])
    for v in range(k):
        out = cur / N[v] * (D[v] + 1)
        it += 4.0 * pn * (cur + out + (cur if v == 0 else 0.0))
        cur = out
        it_l += 1
    L = info["limbs"]
    ga = info["ncoeff"] * (pn * (pn + 1) / 2 + pn * L)
    n = info["n"]
    upd = pn * info["G"] * (n - 1) * n * (2 * n - 1) / 6
    return {"reduce": (red, 1), "evaluate": (ev, ev_l), "interpolate": (it, it_l),
            "reconstruct": (ga, 1), "determinants": (upd, 1)}


def stage_ms(arr: np.ndarray, reps: int) -> tuple:
    import torch
    n, deg = B.shape_of(arr)
    pl = B.plan(n, deg, host_coeffs=arr)
    d = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    out, ws = B.solve_device(pl, d)
    stream = torch.cuda.current_stream()
    res = {}
    for s, name in enumerate(B.STAGES):
        B.solve_stages_device(pl, s, s + 1, d, out, ws)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            B.solve_stages_device(pl, s, s + 1, d, out, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    return pl.info, res


def calibrate(orders=range(2, 33), reps: int = 3, min_dets: int = 4_000_000,
              seed: int = 11) -> dict:
    rng = np.random.default_rng(seed)
    t0 = time.time()
    det = {cls: {} for cls in CLASSES}
    rows, rhs = [], []  # least squares: launches * launch_s + work_s / rate_s = time
    keys = ("reduce", "evaluate", "interpolate", "reconstruct")
    for cls in CLASSES:
        for n in orders:
            arr = probe_matrix(n, cls, min_dets, rng)
            info, ms = stage_ms(arr, reps)
            w = stage_work(info)
            det[cls][str(n)] = w["determinants"][0] / (ms["determinants"] / 1e3)
            for i, key in enumerate(keys):
                work, launches = w[key]
                if launches == 0:
                    continue
                row = [0.0] * (1 + len(keys))
                row[0] = launches
                row[1 + i] = work
                rows.append(row)
                rhs.append(ms[key] / 1e3)
            print(f"{cls} n={n}: {det[cls][str(n)] / 1e12:.2f} T updates/s, "
                  f"{time.time() - t0:.0f} s", file=sys.stderr, flush=True)
    A, b = np.array(rows), np.array(rhs)
    scale = A.max(axis=0)
    x, *_ = np.linalg.lstsq(A / scale, b, rcond=None)
    x = np.maximum(x / scale, 1e-30)
    table = {"det_updates_per_s": det, "launch_us": float(x[0] * 1e6),
             "reduce_bytes_per_s": float(1 / x[1]), "eval_bytes_per_s": float(1 / x[2]),
             "intt_bytes_per_s": float(1 / x[3]), "garner_ops_per_s": float(1 / x[4])}
    fit = A @ x
    table["_measured"] = {
        "seconds": round(time.time() - t0, 1), "reps": reps, "min_dets": min_dets,
        "fit_relative_error_median": float(np.median(np.abs(fit - b) / b)),
        "device": _device_name()}
    return table


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:  # pragma: no cover
        return "unknown"


def _parse_orders(s: str):
    lo, _, hi = s.partition("-")
    return range(int(lo), int(hi or lo) + 1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--orders", default="2-32")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--min-dets", type=int, default=4_000_000)
    args = ap.parse_args(argv)
    B.load_library()
    table = calibrate(_parse_orders(args.orders), args.reps, args.min_dets)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps({k: v for k, v in table.items() if k != "det_updates_per_s"}), flush=True)


if __name__ == "__main__":
    main()
