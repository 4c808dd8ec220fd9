"""The serving workload's large job: a 32 x 32 matrix of trivariate polynomials of degree 5 per
variable, coefficients in [-2^16, 2^16] (16.8 M grid points, 25+ primes). The oracle cannot
solve it in a test's time (about 45 core-hours), so the result is checked by identities that
hold for the exact determinant only with high probability (Schwartz-Zippel), never as oracle
parity:

* at three seeded integer points a in [-2^20, 2^20]^3, the output polynomial evaluated with
  Python integers equals det M(a) from the oracle's integer Bareiss (a false pass has
  probability at most (sum_v D_v / 2^21) per point);
* at two seeded points of F_q^3 for a prime q not of the library's form, the output reduced
  mod q and evaluated on the device equals det M(point) mod q from the oracle's modular
  elimination (probability at most sum_v D_v / q per point).
"""
import numpy as np
import pytest

import paper_2010_12117_amd as pdm
import workloads as W
from oracle import det as OD
from oracle import modular as OM

from helpers import Q31, device_values_at_point

pytestmark = pytest.mark.gpu


def large_job():
    return W.random_matrix(np.random.default_rng(5032), 32, (5, 5, 5), -65536, 65536)


def limb_rows_to_ints(limbs):
    """Little-endian two's-complement uint32 rows -> Python ints (one from_bytes per row)."""
    limbs = np.ascontiguousarray(np.asarray(limbs).view(np.uint32))
    C, L = limbs.shape
    raw = limbs.tobytes()
    w = 4 * L
    return [int.from_bytes(raw[i * w:(i + 1) * w], "little", signed=True) for i in range(C)]


def horner_box(box, point):
    """sum_e box[e] prod_v point_v^{e_v} with Python integers, innermost variable first."""
    for v in range(box.ndim - 1, -1, -1):
        acc = np.zeros(box.shape[:-1], dtype=object)
        for e in range(box.shape[-1] - 1, -1, -1):
            acc = acc * point[v] + box[..., e]
        box = acc
    return int(box[()]) if isinstance(box, np.ndarray) else int(box)


@pytest.fixture(scope="module")
def solved():
    import torch
    a = large_job()
    pl = pdm.plan(32, (5, 5, 5), host_coeffs=a)
    out, ws = pdm.solve_device(pl, torch.from_numpy(a).cuda())
    torch.cuda.synchronize()
    del ws
    return a, pl, out


def test_large_job_shape_and_kernel(solved):
    a, pl, out = solved
    info = pl.info
    assert info["N"] == (256, 256, 256) and info["D"] == (160, 160, 160)
    assert info["pn"] >= 25 and info["det_lanes"] in (8, 16)
    # six coefficients in the first variable: the paired evaluation with three terms per lane
    assert info["deg"][0] + 1 == 6


def test_large_job_exact_integer_points(solved):
    a, pl, out = solved
    info = pl.info
    box_shape = tuple(d + 1 for d in info["D"])
    vals = limb_rows_to_ints(out.cpu().numpy())
    box = np.empty(len(vals), dtype=object)
    box[:] = vals
    box = box.reshape(box_shape)
    rng = np.random.default_rng(16032)
    for _ in range(3):
        point = [int(x) for x in rng.integers(-(1 << 20), (1 << 20) + 1, size=3)]
        M = [[horner_box(a[r, c].astype(object), point) for c in range(32)] for r in range(32)]
        assert horner_box(box, point) == OD.det_bareiss_int(M)


def test_large_job_independent_prime(solved):
    a, pl, out = solved
    info = pl.info
    box_shape = tuple(d + 1 for d in info["D"])
    rng = np.random.default_rng(26032)
    flat = out.view(-1)
    for _ in range(2):
        point = [int(x) for x in rng.integers(1, Q31, size=3)]
        got = device_values_at_point(flat, 0, info["ncoeff"], info["limbs"], box_shape, point,
                                     Q31)
        M = [[horner_box((a[r, c] % Q31).astype(object), point) % Q31 for c in range(32)]
             for r in range(32)]
        assert got == OM.det_mod(M, Q31)
