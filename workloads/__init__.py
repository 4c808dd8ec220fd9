"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays them out; it holds none of the
determinant method's arithmetic. A matrix is an int64 array of shape
(n, n, d1+1, ..., dk+1): entry (i, j) is the dense coefficient box of a polynomial in
x1..xk, first variable slowest, the encoding of the paper's Section 2 (the worked example
F = 1 + 2x + 3xy + 4x^2 + 5y^2 -> [1, 0, 5, 2, 3, 0, 4, 0, 0]).

The paper gives no input matrices (only coefficient range [-100, 100] and degree vectors,
Section 4); every input here is synthetic and stands in for the paper's random matrices:

config 1  n=4, k=2, per-variable degree 2, coefficients U{-10..10}, dense.
config 2  n=12, k=3, degree 3, coefficients U{-1000..1000}, exactly 43 zero entries.
config 3a Sylvester matrix (22 x 22) of f, g in Z[x, y, z] with deg_x 12 and 10, every
          x-coefficient a dense degree-(4,4) polynomial in (y, z), U{-32768..32768},
          leading coefficients nonzero; rows of f first, descending powers of x.
config 3b the same shape from factored f = prod (a_i x - b_i), g = prod (c_j x - d_j).
config 4  4096 matrices, n ~ U{4..24}, k ~ U{2,3}, degree U{1..4} per variable, zero
          fraction U[0.10, 0.40] (Bernoulli per entry), coefficients U{-4096..4096}.
config 5  serving jobs: n ~ U{4..32}, k ~ U{2,3}, degree U{1..5}, U{-65536..65536},
          dense; with probability 1/100 a 32 x 32, k=3, degree (5,5,5) job.

Seeds are 1211700 + config number; draws are made in the order shape, mask, coefficients.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

SEED_BASE = 1211700


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config + 1000 * salt)


def random_matrix(rng: np.random.Generator, n: int, deg: Sequence[int], lo: int, hi: int,
                  zero_entries: int = 0, zero_prob: float = 0.0) -> np.ndarray:
    """Dense random polynomial matrix; coefficients U{lo..hi} inclusive. Either exactly
    `zero_entries` entries (chosen uniformly) or each entry with probability `zero_prob`
    is set to the zero polynomial."""
    box = tuple(int(d) + 1 for d in deg)
    mask = np.ones((n, n), dtype=bool)
    if zero_entries:
        idx = rng.choice(n * n, size=zero_entries, replace=False)
        mask.reshape(-1)[idx] = False
    elif zero_prob > 0:
        mask = rng.random((n, n)) >= zero_prob
    coeffs = rng.integers(lo, hi, size=(n, n) + box, endpoint=True, dtype=np.int64)
    coeffs[~mask] = 0
    return coeffs


def config1(seed_salt: int = 0) -> np.ndarray:
    rng = rng_for(1, seed_salt)
    return random_matrix(rng, 4, (2, 2), -10, 10)


def config2(seed_salt: int = 0, n: int = 12, deg=(3, 3, 3), zeros: int | None = None) -> np.ndarray:
    rng = rng_for(2, seed_salt)
    if zeros is None:
        zeros = int(round(0.3 * n * n))
    return random_matrix(rng, n, deg, -1000, 1000, zero_entries=zeros)


def poly_mul_box(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product of two dense coefficient boxes (object ints), used only to expand the
    factored inputs of config 3b."""
    a = np.asarray(a, dtype=object)
    b = np.asarray(b, dtype=object)
    shape = tuple(x + y - 1 for x, y in zip(a.shape, b.shape))
    out = np.zeros(shape, dtype=object)
    for ia in np.ndindex(a.shape):
        ca = a[ia]
        if ca == 0:
            continue
        for ib in np.ndindex(b.shape):
            cb = b[ib]
            if cb:
                out[tuple(x + y for x, y in zip(ia, ib))] += ca * cb
    return out


def sylvester(f: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Sylvester matrix of f, g in x with coefficients in Z[y, z].

    f has shape (m+1, ...): f[i] is the coefficient box of x^i (likewise g, degree l). The
    result has shape (m+l, m+l, ...): the first l rows hold f's coefficients in descending
    powers of x shifted one column per row, the next m rows hold g's."""
    m = f.shape[0] - 1
    l = g.shape[0] - 1
    inner = np.broadcast_shapes(f.shape[1:], g.shape[1:])
    size = m + l
    S = np.zeros((size, size) + inner, dtype=np.int64)
    for r in range(l):
        for i in range(m + 1):
            S[r, r + i] = f[m - i]
    for r in range(m):
        for j in range(l + 1):
            S[l + r, r + j] = g[l - j]
    return S


def config3a(seed_salt: int = 0, mdeg: int = 12, ldeg: int = 10, inner=(4, 4)) -> np.ndarray:
    rng = rng_for(3, seed_salt)
    box = tuple(d + 1 for d in inner)
    f = rng.integers(-32768, 32768, size=(mdeg + 1,) + box, endpoint=True, dtype=np.int64)
    g = rng.integers(-32768, 32768, size=(ldeg + 1,) + box, endpoint=True, dtype=np.int64)
    for h in (f, g):
        while not np.any(h[-1]):
            h[-1] = rng.integers(-32768, 32768, size=box, endpoint=True, dtype=np.int64)
    return sylvester(f, g)


def factored_linear(rng: np.random.Generator, count: int, n_var: int,
                    var_factors: int, inner_box) -> List[Tuple[np.ndarray, np.ndarray]]:
    """`count` linear factors (a, b) meaning a*x - b with a, b in Z[y, z] as boxes of shape
    `inner_box`. The first `var_factors` have a = alpha + beta*y, b = gamma + delta*z with
    alpha..delta in U{-3..3}, alpha != 0; the rest have integer a != 0 and b in U{-3..3}."""
    out = []
    for t in range(count):
        a = np.zeros(inner_box, dtype=np.int64)
        b = np.zeros(inner_box, dtype=np.int64)
        alpha = 0
        while alpha == 0:
            alpha = int(rng.integers(-3, 3, endpoint=True))
        a[0, 0] = alpha
        if t < var_factors:
            a[1, 0] = int(rng.integers(-3, 3, endpoint=True))
            b[0, 0] = int(rng.integers(-3, 3, endpoint=True))
            b[0, 1] = int(rng.integers(-3, 3, endpoint=True))
        else:
            b[0, 0] = int(rng.integers(-3, 3, endpoint=True))
        out.append((a, b))
    return out


def expand_linear_product(factors, inner_box) -> np.ndarray:
    """Coefficients in x (descending index = power) of prod (a_i x - b_i), each an inner
    box, returned with shape (count+1,) + inner_box; raises if the inner degree exceeds
    the box."""
    poly = [np.zeros((1, 1), dtype=object)]
    poly[0][0, 0] = 1
    for a, b in factors:
        new = [None] * (len(poly) + 1)
        for i, c in enumerate(poly):
            ta = poly_mul_box(c, a)
            tb = -poly_mul_box(c, b)
            new[i + 1] = ta if new[i + 1] is None else _add_box(new[i + 1], ta)
            new[i] = tb if new[i] is None else _add_box(new[i], tb)
        poly = new
    out = np.zeros((len(poly),) + tuple(inner_box), dtype=np.int64)
    for i, c in enumerate(poly):
        for idx in np.ndindex(c.shape):
            if c[idx] != 0:
                if any(x >= s for x, s in zip(idx, inner_box)):
                    raise ValueError("inner degree exceeds the box")
                if abs(int(c[idx])) > 2 ** 15:
                    raise ValueError("coefficient exceeds 2^15")
                out[(i,) + idx] = int(c[idx])
    return out


def _add_box(a, b):
    shape = tuple(max(x, y) for x, y in zip(a.shape, b.shape))
    out = np.zeros(shape, dtype=object)
    out[tuple(slice(0, s) for s in a.shape)] += a
    out[tuple(slice(0, s) for s in b.shape)] += b
    return out


def config3b(seed_salt: int = 0, mdeg: int = 12, ldeg: int = 10, var_factors: int = 4,
             inner=(4, 4)):
    """Returns (Sylvester matrix, f factors, g factors). Resamples until every coefficient
    fits the (y, z) box and |c| <= 2^15."""
    rng = rng_for(3, 100 + seed_salt)
    box = tuple(d + 1 for d in inner)
    while True:
        ff = factored_linear(rng, mdeg, 2, var_factors, (2, 2))
        gf = factored_linear(rng, ldeg, 2, var_factors, (2, 2))
        try:
            f = expand_linear_product(ff, box)
            g = expand_linear_product(gf, box)
        except ValueError:
            continue
        return sylvester(f, g), ff, gf


def config4_shapes(count: int = 4096, seed_salt: int = 0):
    rng = rng_for(4, seed_salt)
    shapes = []
    for _ in range(count):
        n = int(rng.integers(4, 24, endpoint=True))
        k = int(rng.integers(2, 3, endpoint=True))
        deg = tuple(int(x) for x in rng.integers(1, 4, size=k, endpoint=True))
        z = float(rng.uniform(0.10, 0.40))
        shapes.append((n, deg, z))
    return shapes, rng


def config4(count: int = 4096, seed_salt: int = 0) -> List[np.ndarray]:
    shapes, rng = config4_shapes(count, seed_salt)
    return [random_matrix(rng, n, deg, -4096, 4096, zero_prob=z) for n, deg, z in shapes]


def config5_job(rng: np.random.Generator) -> np.ndarray:
    if rng.random() < 0.01:
        return random_matrix(rng, 32, (5, 5, 5), -65536, 65536)
    n = int(rng.integers(4, 32, endpoint=True))
    k = int(rng.integers(2, 3, endpoint=True))
    deg = tuple(int(x) for x in rng.integers(1, 5, size=k, endpoint=True))
    return random_matrix(rng, n, deg, -65536, 65536)


def small_random(rng: np.random.Generator, n: int, deg: Sequence[int], amp: int = 5,
                 zero_prob: float = 0.0) -> np.ndarray:
    return random_matrix(rng, n, deg, -amp, amp, zero_prob=zero_prob)
