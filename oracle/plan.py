"""Plan quantities of the modular method (oracle; test infrastructure only).

Section 2 (after Algorithm 1) fixes what the plan must provide:
* a bound on the determinant's coefficients and the least number of primes whose product
  reaches it (the paper says the bound is easily computed but does not define it; the
  reading used here is Hadamard's inequality applied to 1-norms of the entries, see
  `hadamard_bound_sq`);
* per-variable degrees enlarged to powers of two (the example (15, 7, 9) -> (16, 8, 16),
  largest 2^q_max with q_max = 4);
* primes of the form p = c * 2^q + 1 (equation "primes") so that Z/pZ holds a principal
  2^q-th root of unity (Section 2, DFT over Z/pZ), with "9-digit" (about 2^30) primes.

Readings taken where the paper is silent:
* the number of interpolation nodes per variable must exceed the determinant's degree in
  that variable (Theorem 1 of Section 3.3 needs deg + 1 distinct nodes), so the grid is
  N_v = next_pow2(D_v + 1) with D_v a bound on the determinant's degree in x_v;
* coefficients are recovered in the symmetric range, so the primes' product M must satisfy
  M > 2B, checked exactly as M^2 > 4 B^2;
* the primes are those in (2^29, 2^30) with p = 1 mod 2^16, in descending order: the
  "9-digit" primes c * 2^q + 1 of Section 2, about 10^9.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import poly as P

PRIME_LO = 1 << 29
PRIME_HI = 1 << 30
PRIME_TWO_ADICITY = 16


def next_pow2(x: int) -> int:
    """Smallest power of two >= x (x >= 1)."""
    p = 1
    while p < x:
        p *= 2
    return p


def enlarge_degrees(d: Sequence[int]) -> List[int]:
    """The paper's degree enlargement, read as: each degree rounded up to a power of two
    (so that (15, 7, 9) becomes (16, 8, 16))."""
    return [next_pow2(x) for x in d]


def entry_degrees(arr: np.ndarray) -> np.ndarray:
    """deg[i, j, v]: the degree of entry (i, j) in variable v, -1 for a zero entry, read
    from the dense box (shape (n, n, d1+1, ..., dk+1))."""
    arr = np.asarray(arr)
    n = arr.shape[0]
    k = arr.ndim - 2
    out = np.full((n, n, k), -1, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            box = arr[i, j]
            for v in range(k):
                other = tuple(a for a in range(k) if a != v)
                nz = np.any(box != 0, axis=other) if other else (box != 0)
                idx = np.nonzero(nz)[0]
                out[i, j, v] = int(idx[-1]) if len(idx) else -1
    return out


def det_degree_bound_from_shape(n: int, deg: Sequence[int]) -> List[int]:
    """D_v for a matrix whose entries all fit in the box deg: the determinant is a sum of
    products of n entries, so its degree in x_v is at most n * deg_v."""
    return [n * int(d) for d in deg]


def det_degree_bound(arr: np.ndarray) -> List[int]:
    """Tighter data-dependent D_v = min(sum_i max_j deg_v a_ij, sum_j max_i deg_v a_ij)
    (every Leibniz term takes one entry per row and one per column)."""
    deg = entry_degrees(arr)
    n = deg.shape[0]
    k = deg.shape[2]
    out = []
    for v in range(k):
        rows = sum(max(0, int(deg[i, :, v].max())) for i in range(n))
        cols = sum(max(0, int(deg[:, j, v].max())) for j in range(n))
        out.append(min(rows, cols))
    return out


def grid_sizes(D: Sequence[int]) -> List[int]:
    """N_v = next_pow2(D_v + 1): enough distinct roots of unity to interpolate."""
    return [next_pow2(int(x) + 1) for x in D]


def hadamard_bound_sq(arr: np.ndarray) -> int:
    """B^2 = min(prod_i sum_j |a_ij|_1^2, prod_j sum_i |a_ij|_1^2) (exact integer).

    Every coefficient of det M is at most its 2-norm; by Parseval on the unit torus and
    Hadamard's inequality the 2-norm is at most sqrt(prod_i sum_j sup|a_ij|^2), and the
    supremum of |a_ij| on the torus is at most its 1-norm. The same holds by columns."""
    arr = np.asarray(arr)
    n = arr.shape[0]
    k = arr.ndim - 2
    norms = [[P.norm1(P.from_box(arr[i, j], k)) for j in range(n)] for i in range(n)]
    rows = 1
    for i in range(n):
        rows *= sum(norms[i][j] ** 2 for j in range(n))
    cols = 1
    for j in range(n):
        cols *= sum(norms[i][j] ** 2 for i in range(n))
    return min(rows, cols)


def is_prime(m: int) -> bool:
    """Trial division (plain and obviously correct; m < 2^31 here)."""
    if m < 2:
        return False
    if m % 2 == 0:
        return m == 2
    f = 3
    while f * f <= m:
        if m % f == 0:
            return False
        f += 2
    return True


def ntt_primes(count: int) -> List[int]:
    """The first `count` primes p in (2^29, 2^30) with p = 1 mod 2^16, descending."""
    out = []
    step = 1 << PRIME_TWO_ADICITY
    c = (PRIME_HI - 1) // step
    while len(out) < count:
        p = c * step + 1
        if p <= PRIME_LO:
            raise ValueError("ran out of primes")
        if p < PRIME_HI and is_prime(p):
            out.append(p)
        c -= 1
    return out


def num_primes(bound_sq: int, primes: Sequence[int] | None = None) -> int:
    """Least t with (p_0 ... p_{t-1})^2 > 4 B^2 (at least one prime)."""
    t = 0
    prod = 1
    while True:
        if primes is not None and t >= len(primes):
            raise ValueError("not enough primes")
        p = primes[t] if primes is not None else ntt_primes(t + 1)[t]
        prod *= p
        t += 1
        if prod * prod > 4 * bound_sq:
            return t


def prime_factors(m: int) -> List[int]:
    out = []
    f = 2
    while f * f <= m:
        if m % f == 0:
            out.append(f)
            while m % f == 0:
                m //= f
        f += 1
    if m > 1:
        out.append(m)
    return out


def primitive_root(p: int) -> int:
    """Smallest generator of the multiplicative group of Z/pZ."""
    qs = prime_factors(p - 1)
    g = 2
    while any(pow(g, (p - 1) // q, p) == 1 for q in qs):
        g += 1
    return g


def root_of_unity(p: int, N: int) -> int:
    """Principal N-th root of unity g^((p-1)/N) with g the smallest primitive root."""
    assert (p - 1) % N == 0
    return pow(primitive_root(p), (p - 1) // N, p)


def limbs_for(M: int) -> int:
    """32-bit limbs that hold every integer in [-(M-1)/2, (M-1)/2] in two's complement."""
    return max(1, (M.bit_length() + 31) // 32)
