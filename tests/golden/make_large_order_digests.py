"""Write large_order_oracle_digests.json: the oracle's exact determinant of matrices of order
25-32 whose first variable has 1 or 5-7 coefficients.

These shapes take the elimination kernels with 8 or 16 lanes per matrix whose first-variable
evaluation is paired with three terms per lane (5 or 6 coefficients, as in the 32 x 32
trivariate degree-5 serving job) or term by term (1 or 7 coefficients). Coefficients are drawn like the serving jobs'
(uniform in [-2^16, 2^16], dense), so the prime count reaches 20-25 and the reconstruction
runs its widest form.

Each matrix comes from the seeded generator (`case_matrix`); the oracle's pointwise Bareiss
(integer nodes, integer Bareiss per node, exact interpolation) gives its determinant, stored
as the digest of make_config4_digests.digest. Only the oracle and the seeded generator are
used. Usage:
    python tests/golden/make_large_order_digests.py [--workers 7]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import workloads as W  # noqa: E402
from make_config4_digests import digest  # noqa: E402
from oracle import det as OD, plan as PL  # noqa: E402

OUT = os.path.join(HERE, "large_order_oracle_digests.json")

# (n, per-variable degree, seed): first-variable coefficient counts 6, 5, 6, 6, 7 and 1
CASES = [
    (25, (5,), 25051),
    (26, (4,), 26041),
    (32, (5,), 32051),
    (28, (5, 1), 28511),
    (32, (5, 1), 32511),
    (29, (6, 1), 29611),
    (27, (0, 3), 27031),
]


def case_key(n, deg, seed) -> str:
    return f"{n}:{'.'.join(str(d) for d in deg)}:{seed}"


def case_matrix(n, deg, seed) -> np.ndarray:
    return W.random_matrix(np.random.default_rng(seed), n, deg, -65536, 65536)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    t0 = time.time()
    out = {}
    with Pool(args.workers) as pool:
        for n, deg, seed in CASES:
            a = case_matrix(n, deg, seed)
            box = OD.det_pointwise(a, PL.det_degree_bound_from_shape(n, deg), pool=pool)
            out[case_key(n, deg, seed)] = digest(box)
            print(f"{n} {deg}: {time.time() - t0:.0f} s", flush=True)
    doc = {
        "workload": "seeded dense matrices of order 25-32, coefficients U[-2^16, 2^16]",
        "digest": "sha256 of make_config4_digests.canonical_text, first 16 hex digits",
        "oracle": "oracle.det.det_pointwise with the degree bound from the shape",
        "digests": out,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {len(out)} digests in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
