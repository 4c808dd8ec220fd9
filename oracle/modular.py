"""The modular method step by step, for small inputs (oracle; test infrastructure only).

Algorithm 1 of the paper: for each prime p_i, evaluate every entry on the interpolation
nodes (FFT), take a numeric determinant at every node (DET), interpolate the determinant
polynomial mod p_i (IFFT); then recover the integer coefficients by the Chinese remainder
theorem in mixed-radix form (CRT, Section 3.4 and Algorithm 4). Each step here is the plain
definition (direct sums rather than fast transforms), in the paper's order:

* `reduce_mod`        integer coefficients -> residues in [0, p).
* `evaluate_at_node`  entry polynomial at the node (w_1^j_1, ..., w_k^j_k), the DFT over
                      Z/pZ at a principal root of unity (Section 2, DFT paragraph).
* `det_mod`           determinant of a matrix over Z/pZ by elimination with the first
                      nonzero pivot, each row exchange flipping the sign (the role of
                      Algorithm 3; its printed update is garbled, so the plain elimination is
                      used: the determinant mod p is unique).
* `interpolate_mod`   inverse DFT: opposite sign in the exponent and a 1/N factor
                      (Section 3.3, last paragraph), separably over the variables.
* `garner`            mixed-radix digits alpha_i with alpha_0 = x_0 and
                      alpha_i = (x_i - sum_{j<i} alpha_j m_j) c_i mod p_i, m_j = p_0..p_{j-1},
                      c_i = (p_0..p_{i-1})^{-1} mod p_i (Section 3.4, read with the index
                      fixes listed below), X = sum alpha_i m_i, then the symmetric range.
* `crt_naive`         the textbook CRT sum, to cross-check `garner`.

Readings of garbled formulas (Section 3.4): m_j is the product of the primes before p_j
(not up to p_{n-1}); the Horner form multiplies by p_i; the digit loop runs i = 1..pn-1.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np

from . import plan as PL
from . import poly as P


def reduce_mod(c: int, p: int) -> int:
    return int(c) % p


def evaluate_at_node(entry: P.Poly, p: int, omegas: Sequence[int], j: Sequence[int]) -> int:
    """sum_e c_e prod_v (w_v^{j_v})^{e_v} mod p."""
    point = [pow(w, jj, p) for w, jj in zip(omegas, j)]
    return P.evaluate({e: c % p for e, c in entry.items()}, point, p)


def det_mod(A: List[List[int]], p: int) -> int:
    """Determinant over Z/pZ: Gaussian elimination, first nonzero pivot scanning down the
    column, sign flip per exchange, inverse by Fermat's little theorem."""
    n = len(A)
    A = [[int(x) % p for x in row] for row in A]
    det = 1
    for s in range(n):
        r = next((r for r in range(s, n) if A[r][s] != 0), None)
        if r is None:
            return 0
        if r != s:
            A[s], A[r] = A[r], A[s]
            det = -det
        piv = A[s][s]
        det = det * piv % p
        inv = pow(piv, p - 2, p)
        for i in range(s + 1, n):
            f = A[i][s] * inv % p
            if f:
                for j in range(s, n):
                    A[i][j] = (A[i][j] - f * A[s][j]) % p
    return det % p


def interpolate_mod(values: np.ndarray, p: int, omegas: Sequence[int]) -> np.ndarray:
    """Coefficients a_e = prod_v N_v^{-1} * sum_j values[j] * prod_v w_v^{-j_v e_v} mod p.

    `values` is indexed by the node exponents (j_1, ..., j_k) in natural order; the result
    has the same shape, indexed by exponents."""
    out = np.asarray(np.asarray(values, dtype=object) % p, dtype=object)
    for v, w in enumerate(omegas):
        N = out.shape[v]
        winv = pow(w, p - 2, p)
        Ninv = pow(N, p - 2, p)
        T = np.empty((N, N), dtype=object)
        for e in range(N):
            for jj in range(N):
                T[e, jj] = pow(winv, e * jj, p) * Ninv % p
        moved = np.moveaxis(out, v, -1)
        res = np.tensordot(moved, T.T, axes=([moved.ndim - 1], [0]))
        out = np.moveaxis(res, -1, v) % p
    return np.asarray(out, dtype=object)


def garner(residues: Sequence[int], primes: Sequence[int]) -> int:
    """Mixed-radix conversion followed by the symmetric range (-(M-1)/2 .. (M-1)/2)."""
    pn = len(primes)
    alphas = []
    for i in range(pn):
        pi = primes[i]
        acc = 0
        mj = 1
        for j in range(i):
            acc = (acc + alphas[j] * (mj % pi)) % pi
            mj *= primes[j]
        ci = pow(mj % pi, pi - 2, pi) if i else 1
        alphas.append((residues[i] - acc) * ci % pi)
    X = 0
    for i in reversed(range(pn)):
        X = X * primes[i] + alphas[i]
    M = 1
    for p in primes:
        M *= p
    return X - M if X > (M - 1) // 2 else X


def crt_naive(residues: Sequence[int], primes: Sequence[int]) -> int:
    """Textbook CRT: X = sum r_i M_i (M_i^{-1} mod p_i) mod M, then the symmetric range."""
    M = 1
    for p in primes:
        M *= p
    X = 0
    for r, p in zip(residues, primes):
        Mi = M // p
        X += r * Mi * pow(Mi % p, p - 2, p)
    X %= M
    return X - M if X > (M - 1) // 2 else X


def modular_determinant(arr: np.ndarray, D: Sequence[int] | None = None,
                        extra_primes: int = 0, primes: Sequence[int] | None = None):
    """Algorithm 1 with every step done by its definition. Small inputs only.

    Returns (coefficient box of det M as an object array of shape (D1+1, ..., Dk+1),
    dict with the plan quantities and the per-prime intermediates)."""
    arr = np.asarray(arr)
    n = arr.shape[0]
    k = arr.ndim - 2
    deg = [arr.shape[2 + v] - 1 for v in range(k)]
    if D is None:
        D = PL.det_degree_bound_from_shape(n, deg)
    N = PL.grid_sizes(D)
    B2 = PL.hadamard_bound_sq(arr)
    if primes is None:
        pn = PL.num_primes(B2) + extra_primes
        primes = PL.ntt_primes(pn)
    pn = len(primes)
    M = [[P.from_box(arr[i, j], k) for j in range(n)] for i in range(n)]
    per_prime = []
    for p in primes:
        omegas = [PL.root_of_unity(p, Nv) for Nv in N]
        dets = np.empty(tuple(N), dtype=object)
        for j in itertools.product(*[range(Nv) for Nv in N]):
            A = [[evaluate_at_node(M[r][c], p, omegas, j) for c in range(n)] for r in range(n)]
            dets[j] = det_mod(A, p)
        coefs = interpolate_mod(dets, p, omegas)
        per_prime.append(dict(p=p, omegas=omegas, dets=dets, coefs=coefs))
    box = tuple(d + 1 for d in D)
    out = np.empty(box, dtype=object)
    for e in itertools.product(*[range(b) for b in box]):
        out[e] = garner([pp["coefs"][e] for pp in per_prime], primes)
    # coefficients beyond D must vanish mod every prime (the grid is larger than the box)
    for pp in per_prime:
        c = pp["coefs"]
        for e in itertools.product(*[range(Nv) for Nv in N]):
            if any(ev > dv for ev, dv in zip(e, D)):
                assert c[e] == 0, "nonzero coefficient beyond the degree bound"
    info = dict(D=list(D), N=N, B2=B2, primes=list(primes), pn=pn, per_prime=per_prime)
    return out, info
