"""Write config4_oracle_digests.json: the oracle's exact determinant of each of the cheapest
matrices of the 4096-matrix batching workload, stored as a digest.

The workload is the seeded generator's (n uniform in [4, 24], 2-3 variables, per-variable
degree 1-4, coefficients uniform in [-2^12, 2^12], 10-40% zero entries). Matrices are ranked by
the pointwise oracle's cost, prod_v (n d_v + 1) nodes times n^3, and the cheapest `--fraction`
of them are solved by the oracle's pointwise Bareiss (evaluation at integer nodes, integer
Bareiss per node, exact interpolation through the integer-scaled inverse Vandermonde
matrix). Each result is stored as the first 16 hex digits of the SHA-256 of its canonical
text (see `canonical_text`), which does not depend on the box the coefficients are laid out
in.

Only the oracle and the seeded input generator are used. Usage:
    python tests/golden/make_config4_digests.py [--fraction 0.75] [--workers 7]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import det as OD, plan as PL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_oracle_digests.json")


def oracle_cost(n, deg):
    return int(np.prod([n * d + 1 for d in deg])) * n ** 3


def canonical_text(box) -> str:
    """Nonzero coefficients as 'e1.e2..:value' sorted by exponent tuple, joined by ';'."""
    box = np.asarray(box, dtype=object)
    items = []
    for idx in np.ndindex(box.shape):
        v = int(box[idx])
        if v:
            items.append((tuple(int(x) for x in idx), v))
    items.sort()
    return ";".join(".".join(str(e) for e in k) + ":" + str(v) for k, v in items)


def digest(box) -> str:
    return hashlib.sha256(canonical_text(box).encode()).hexdigest()[:16]


def ranked_indices(fraction: float):
    shapes, _ = W.config4_shapes()
    order = sorted(range(len(shapes)), key=lambda i: (oracle_cost(shapes[i][0], shapes[i][1]), i))
    return order[:int(len(order) * fraction)], shapes


def _solve(args):
    i, a = args
    n = a.shape[0]
    deg = [a.shape[2 + v] - 1 for v in range(a.ndim - 2)]
    box = OD.det_pointwise(a, PL.det_degree_bound_from_shape(n, deg))
    return i, digest(box)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fraction", type=float, default=0.75)
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    idx, shapes = ranked_indices(args.fraction)
    mats = W.config4()
    # the most expensive first, so that the pool ends evenly
    work = [(i, mats[i]) for i in sorted(idx, key=lambda i: -oracle_cost(*shapes[i][:2]))]
    t0 = time.time()
    out = {}
    with Pool(args.workers) as pool:
        for done, (i, d) in enumerate(pool.imap_unordered(_solve, work, chunksize=1), 1):
            out[i] = d
            if done % 256 == 0:
                print(f"{done}/{len(work)} in {time.time() - t0:.0f} s", flush=True)
    doc = {
        "workload": "4096-matrix batching workload of the seeded generator (workloads.config4)",
        "selection": f"cheapest {args.fraction:.2f} by prod_v (n d_v + 1) * n^3",
        "digest": "sha256 of canonical_text, first 16 hex digits",
        "oracle": "oracle.det.det_pointwise with the degree bound from the shape",
        "digests": {str(i): out[i] for i in sorted(out)},
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {len(out)} digests in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
