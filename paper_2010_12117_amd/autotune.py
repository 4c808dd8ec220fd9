"""Autotuner of the elimination kernel's launch mapping (polydet_tuning in include/polydet.h).

For every matrix order n and class (first variable with 2..4 coefficients, whose evaluation is
paired across the wave's halves with two terms per lane, or any other; its probe has 5
coefficients, paired with three terms per lane), it times the candidate mappings on the GPU:
* lanes per matrix: every count the build compiles for n;
* points per LDS tile (Q): 4, 8, 16;
* elimination form: the exchanging kernel, and for n <= 16 the left-looking pass + repair.
Each candidate is installed as the table entry, a plan is built from it, and the elimination
stage's device time (POLYDET_STAGE_TIMING), the best mean over interleaved rounds of a few
solves each, decides. The winners form the table
that binding.py installs at load time (tuning_gfx950.json next to this file).

The probe matrix of each (n, class) has random coefficients with a quarter of the entries zero
and enough variables and degree that one solve holds at least `min_dets` modular determinants,
so that the kernel fills the GPU as it does in real workloads. No choice changes a result.

Usage (on the GPU): python -m paper_2010_12117_amd.autotune --out FILE [--orders 2-32]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import binding as B

CLASSES = ("paired", "other")
LANES = (1, 2, 4, 8, 16)
TILE_POINTS = (4, 8, 16)
LL_MAX_N = 16


def supported_lanes(n: int):
    """The (order, lanes) pairs the library compiles (det_config_supported)."""
    ok = {1: n <= 12, 2: 2 <= n <= 16, 4: 4 <= n <= 24, 8: n >= 8, 16: n >= 16}
    return [g for g in LANES if ok[g]]


def probe_matrix(n: int, cls: str, min_dets: int, rng: np.random.Generator) -> np.ndarray:
    """Random n x n matrix of the class with at least min_dets modular dets per solve."""
    first = 3 if cls == "paired" else 4  # 4 or 5 coefficients in the first variable
    for deg in ((first, 1), (first, 2), (first, 1, 1), (first, 2, 1), (first, 2, 2),
                (first, 3, 2), (first, 3, 3), (first, 4, 3), (first, 4, 4)):
        arr = rng.integers(-64, 65, size=(n, n) + tuple(d + 1 for d in deg), dtype=np.int64)
        arr[rng.random((n, n)) < 0.25] = 0
        info = B.plan(n, deg, host_coeffs=arr, flags=B.HOST_ONLY).info
        if info["pn"] * info["G"] >= min_dets:
            return arr
    return arr


def time_candidate(arr: np.ndarray, reps: int) -> float:
    """Mean device ms of the elimination stage over `reps` solves (one warm-up)."""
    import torch
    n, deg = B.shape_of(arr)
    pl = B.plan(n, deg, host_coeffs=arr, flags=B.STAGE_TIMING)
    d = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    out = torch.empty((pl.info["ncoeff"], pl.info["limbs"]), dtype=torch.int32, device="cuda")
    ws = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    B.solve_device(pl, d, out, ws)
    torch.cuda.synchronize()
    pl.stage_times()
    for _ in range(reps):
        B.solve_device(pl, d, out, ws)
    torch.cuda.synchronize()
    ms, solves = pl.stage_times()
    return ms["determinants"] / max(1, solves)


def _entry(table: dict, cls: str, n: int, lanes: int, ll: int, q: int) -> dict:
    t = json.loads(json.dumps(table))
    for field, v in (("lanes", lanes), ("left_looking", ll), ("tile_points", q)):
        t.setdefault(field, {}).setdefault(cls, {})[str(n)] = v
    return t


def tune(orders=range(2, 33), reps: int = 5, min_dets: int = 4_000_000, seed: int = 7,
         rounds: int = 2, log=sys.stderr) -> dict:
    """Measure every candidate; returns the table (set_tuning's form) and the timings."""
    rng = np.random.default_rng(seed)
    table = {"lanes": {c: {} for c in CLASSES}, "left_looking": {c: {} for c in CLASSES},
             "tile_points": {c: {} for c in CLASSES}}
    timings = {c: {} for c in CLASSES}
    for cls in CLASSES:
        for n in orders:
            arr = probe_matrix(n, cls, min_dets, rng)
            cands = []
            for lanes in supported_lanes(n):
                for q in TILE_POINTS:
                    forms = (2, 1) if (n <= LL_MAX_N and lanes == supported_lanes(n)[0]) else (2,)
                    cands += [(lanes, ll, q) for ll in forms]
            best = {c: float("inf") for c in cands}
            for _ in range(rounds):  # interleaved rounds; each candidate keeps its best mean
                for c in cands:
                    B.set_tuning(_entry(table, cls, n, *c))
                    best[c] = min(best[c], time_candidate(arr, reps))
            results = sorted((ms, *c) for c, ms in best.items())
            ms, lanes, ll, q = results[0]
            for field, v in (("lanes", lanes), ("left_looking", ll), ("tile_points", q)):
                table[field][cls][str(n)] = v
            timings[cls][str(n)] = [[round(r[0], 4), r[1], r[2], r[3]] for r in results]
            print(f"autotune: {cls} n={n}: lanes {lanes}, "
                  f"{'left-looking' if ll == 1 else 'exchange'}, Q {q}: {ms:.4f} ms "
                  f"(worst {results[-1][0]:.4f})", file=log, flush=True)
    B.set_tuning(table)
    return {"table": table, "timings": timings}


def parse_orders(text: str):
    lo, _, hi = text.partition("-")
    return range(int(lo), int(hi or lo) + 1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True, help="table file to write (JSON)")
    ap.add_argument("--orders", default="2-32")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--min-dets", type=int, default=4_000_000)
    args = ap.parse_args(argv)
    B.set_tuning(None)  # measure from the built-in choices
    t0 = time.time()
    res = tune(parse_orders(args.orders), args.reps, args.min_dets, rounds=args.rounds)
    out = dict(res["table"])
    out["_measured"] = {"device": _device_name(), "seconds": round(time.time() - t0, 1),
                        "timings_ms_lanes_form_q": res["timings"]}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(f"autotune: wrote {args.out}", file=sys.stderr)


def _device_name():
    import torch
    return torch.cuda.get_device_name(0)


if __name__ == "__main__":
    main()
