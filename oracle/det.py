"""Exact determinants over Z and Z[x1..xk] (oracle; test infrastructure only).

The quantity the paper's method computes (Algorithm 1; Section 2, "Problem" and the
modular-method rationale) is det M in Z[x1..xk] for an n x n matrix M of integer
polynomials, with no loss of accuracy. This module computes it in three independent ways:

* `det_leibniz`      the definition: sum over permutations of sign * product of entries.
* `det_bareiss_poly` "oracle A": fraction-free (Bareiss) elimination directly over
                     Z[x1..xk] with exact polynomial division.
* `det_pointwise`    "oracle B": the integer determinant (Bareiss over Z) at every node of
                     the integer grid {0..D1} x ... x {0..Dk}, then exact interpolation on
                     that grid. Interpolation is unique on D_v + 1 distinct nodes per
                     variable (Theorem 1 of Section 3.3, the Vandermonde argument).

plus `det_fraction` (Gaussian elimination over Q with `fractions.Fraction`) as a textbook
special case for integer matrices (k = 0). None of these shares code with the GPU path.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import factorial
from typing import List, Sequence

import numpy as np

from . import poly as P


def _perm_sign(perm: Sequence[int]) -> int:
    sign = 1
    seen = [False] * len(perm)
    for i in range(len(perm)):
        if seen[i]:
            continue
        j, length = i, 0
        while not seen[j]:
            seen[j] = True
            j = perm[j]
            length += 1
        if length % 2 == 0:
            sign = -sign
    return sign


def det_leibniz(M, k: int | None = None):
    """Permutation expansion. Entries are ints (k is None) or dict polynomials in k vars."""
    n = len(M)
    if k is None:
        total = 0
        for perm in itertools.permutations(range(n)):
            t = _perm_sign(perm)
            for i in range(n):
                t *= M[i][perm[i]]
                if t == 0:
                    break
            total += t
        return total
    total: P.Poly = {}
    for perm in itertools.permutations(range(n)):
        t = P.const(_perm_sign(perm), k)
        for i in range(n):
            t = P.mul(t, M[i][perm[i]])
            if not t:
                break
        total = P.add(total, t)
    return total


def det_bareiss_int(M: List[List[int]]) -> int:
    """Fraction-free Bareiss elimination over Z with row exchanges.

    At step s every entry of the trailing block becomes the s+1 order leading minor
    expansion (a_ss a_ij - a_is a_sj) / a_{s-1,s-1}, an exact integer division (Sylvester's
    identity). A zero pivot is replaced by the first lower row with a nonzero entry in the
    pivot column, flipping the sign; if there is none the determinant is 0."""
    n = len(M)
    if n == 0:
        return 1
    A = [list(map(int, row)) for row in M]
    sign = 1
    prev = 1
    for s in range(n - 1):
        if A[s][s] == 0:
            r = next((r for r in range(s + 1, n) if A[r][s] != 0), None)
            if r is None:
                return 0
            A[s], A[r] = A[r], A[s]
            sign = -sign
        piv = A[s][s]
        for i in range(s + 1, n):
            ais = A[i][s]
            row_i = A[i]
            row_s = A[s]
            for j in range(s + 1, n):
                num = piv * row_i[j] - ais * row_s[j]
                q, rem = divmod(num, prev)
                if rem:
                    raise ArithmeticError("Bareiss division not exact")
                row_i[j] = q
            row_i[s] = 0
        prev = piv
    return sign * A[n - 1][n - 1]


def det_bareiss_poly(M, k: int) -> P.Poly:
    """Oracle A: Bareiss elimination over Z[x1..xk] with exact polynomial division and
    row exchanges (the same recurrence as `det_bareiss_int`, on dict polynomials)."""
    n = len(M)
    if n == 0:
        return P.const(1, k)
    A = [[dict(e) for e in row] for row in M]
    sign = 1
    prev = P.const(1, k)
    for s in range(n - 1):
        if not A[s][s]:
            r = next((r for r in range(s + 1, n) if A[r][s]), None)
            if r is None:
                return {}
            A[s], A[r] = A[r], A[s]
            sign = -sign
        piv = A[s][s]
        for i in range(s + 1, n):
            ais = A[i][s]
            for j in range(s + 1, n):
                num = P.sub(P.mul(piv, A[i][j]), P.mul(ais, A[s][j]))
                A[i][j] = P.divexact(num, prev)
            A[i][s] = {}
        prev = piv
    return P.scale(A[n - 1][n - 1], sign)


def det_fraction(M: List[List[int]]) -> int:
    """Gaussian elimination over Q with exact fractions (first nonzero pivot, sign per
    swap); the product of the pivots is the determinant. For integer matrices."""
    n = len(M)
    A = [[Fraction(int(x)) for x in row] for row in M]
    det = Fraction(1)
    for s in range(n):
        r = next((r for r in range(s, n) if A[r][s] != 0), None)
        if r is None:
            return 0
        if r != s:
            A[s], A[r] = A[r], A[s]
            det = -det
        det *= A[s][s]
        for i in range(s + 1, n):
            f = A[i][s] / A[s][s]
            if f:
                for j in range(s, n):
                    A[i][j] -= f * A[s][j]
    assert det.denominator == 1
    return int(det)


# ---------------------------------------------------------------------------------------
# Oracle B: pointwise integer determinants on the integer grid, exact interpolation.
# ---------------------------------------------------------------------------------------

def vandermonde_int(D: int) -> np.ndarray:
    """V[t, e] = t**e for integer nodes t = 0..D and exponents e = 0..D (object ints)."""
    V = np.empty((D + 1, D + 1), dtype=object)
    for t in range(D + 1):
        for e in range(D + 1):
            V[t, e] = t ** e
    return V


def scaled_inverse_vandermonde(D: int) -> np.ndarray:
    """W = D! * V^{-1} for the nodes 0..D, as exact integers.

    V^{-1} maps values at the nodes to monomial coefficients. Its entries are Lagrange-basis
    coefficients with denominators i!(D-i)!, which divide D!, so W is integral. Computed by
    Gauss-Jordan elimination over Q."""
    n = D + 1
    V = vandermonde_int(D)
    A = [[Fraction(int(V[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        r = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[r] = A[r], A[c]
        inv = 1 / A[c][c]
        A[c] = [x * inv for x in A[c]]
        for i in range(n):
            if i != c and A[i][c] != 0:
                f = A[i][c]
                A[i] = [x - f * y for x, y in zip(A[i], A[c])]
    fD = factorial(D)
    W = np.empty((n, n), dtype=object)
    for i in range(n):
        for j in range(n):
            w = A[i][n + j] * fD
            assert w.denominator == 1
            W[i, j] = int(w.numerator)
    return W


def _apply_along(arr: np.ndarray, mat: np.ndarray, axis: int) -> np.ndarray:
    """out[..., i, ...] = sum_j mat[i, j] * arr[..., j, ...] along `axis` (exact ints)."""
    moved = np.moveaxis(arr, axis, -1)
    out = np.tensordot(moved, mat.T, axes=([moved.ndim - 1], [0]))
    return np.moveaxis(out, -1, axis)


def evaluate_on_grid(box: np.ndarray, D: Sequence[int]) -> np.ndarray:
    """Exact values of one entry (dense coefficient box, first variable slowest) at every
    integer node of {0..D1} x ... x {0..Dk}, one variable at a time."""
    vals = np.asarray(box, dtype=object)
    for v, Dv in enumerate(D):
        m = vals.shape[v]
        V = np.empty((Dv + 1, m), dtype=object)
        for t in range(Dv + 1):
            for e in range(m):
                V[t, e] = t ** e
        vals = _apply_along(vals, V, v)
    return vals


def interpolate_grid(values: np.ndarray, D: Sequence[int]) -> np.ndarray:
    """Exact monomial coefficients of the unique polynomial with per-variable degree <= D_v
    taking the given integer values on {0..D1} x ... x {0..Dk}; raises if not integral."""
    out = np.asarray(values, dtype=object)
    denom = 1
    for v, Dv in enumerate(D):
        out = _apply_along(out, scaled_inverse_vandermonde(Dv), v)
        denom *= factorial(Dv)
    flat = out.reshape(-1)
    res = np.empty(flat.shape, dtype=object)
    for i, x in enumerate(flat):
        q, r = divmod(int(x), denom)
        if r:
            raise ArithmeticError("interpolated coefficient is not an integer")
        res[i] = q
    return res.reshape(out.shape)


def node_matrices(arr: np.ndarray, D: Sequence[int]) -> np.ndarray:
    """Object array of shape (D1+1, ..., Dk+1, n, n): the integer matrix at every node."""
    n = arr.shape[0]
    k = arr.ndim - 2
    grid = tuple(d + 1 for d in D)
    out = np.empty(grid + (n, n), dtype=object)
    for i in range(n):
        for j in range(n):
            out[(Ellipsis, i, j)] = evaluate_on_grid(np.asarray(arr[i, j], dtype=object), D)
    assert k == len(D)
    return out


def _det_rows(mats):
    return [det_bareiss_int(m) for m in mats]


def det_pointwise(arr, D: Sequence[int], pool=None) -> np.ndarray:
    """Oracle B. `arr` has shape (n, n, d1+1, ..., dk+1) (int64 or object); `D` bounds the
    determinant's degree per variable. Returns the dense coefficient box of det M with
    shape (D1+1, ..., Dk+1) as Python ints (object array).

    `pool` (optional, a multiprocessing pool) spreads the node determinants over workers;
    the arithmetic is the same either way."""
    arr = np.asarray(arr, dtype=object)
    n = arr.shape[0]
    D = [int(d) for d in D]
    if n == 0:
        raise ValueError("empty matrix")
    mats = node_matrices(arr, D)
    grid = mats.shape[:-2]
    flat = mats.reshape((-1, n, n))
    rows = [[[int(x) for x in r] for r in m] for m in flat]
    if pool is None:
        dets = _det_rows(rows)
    else:
        chunk = max(1, len(rows) // (64 * max(1, getattr(pool, "_processes", 1))))
        parts = [rows[i:i + chunk] for i in range(0, len(rows), chunk)]
        dets = [d for part in pool.map(_det_rows, parts) for d in part]
    values = np.empty(len(dets), dtype=object)
    for i, d in enumerate(dets):
        values[i] = d
    values = values.reshape(grid)
    return interpolate_grid(values, D)
