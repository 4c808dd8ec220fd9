"""Planted mistakes in the oracle are caught by its pins (CPU only).

Each case replaces one oracle function, in this process only, by a version with a plausible
mistake (a dropped sign, a wrong index, an off-by-one, a transposed operand, a wrong root or
scale), then runs the pins of tests/test_oracle.py until one fails. A mistake that no pin
catches fails this test. The oracle's files are not modified."""
import inspect
import itertools
import random

import numpy as np
import pytest

import test_oracle as T
from oracle import det as OD
from oracle import modular as OM
from oracle import plan as PL
from oracle import poly as P


def _pin_calls():
    """(name, zero-argument callable) for every pin of test_oracle, parametrized cases
    expanded; pins that need pytest fixtures are left out."""
    out = []
    for name, fn in inspect.getmembers(T, inspect.isfunction):
        if not name.startswith("test_") or fn.__module__ != T.__name__:
            continue
        params = list(inspect.signature(fn).parameters)
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not params:
            out.append((name, fn))
            continue
        if len(marks) != 1:
            continue
        argnames, values = marks[0].args[0], marks[0].args[1]
        argnames = [a.strip() for a in argnames.split(",")] if isinstance(argnames, str) else list(argnames)
        if sorted(argnames) != sorted(params):
            continue
        for v in values:
            v = v if len(argnames) > 1 else (v,)
            out.append((f"{name}{v}", (lambda f, kw: (lambda: f(**kw)))(fn, dict(zip(argnames, v)))))
    return out


def _caught(monkeypatch, target, attr, replacement):
    monkeypatch.setattr(target, attr, replacement)
    for name, call in _pin_calls():
        try:
            call()
        except Exception:
            return name
    return None


# --- the planted mistakes ----------------------------------------------------------------

def leibniz_no_sign(M, k=None):
    n = len(M)
    if k is None:
        total = 0
        for perm in itertools.permutations(range(n)):
            t = 1
            for i in range(n):
                t *= M[i][perm[i]]
            total += t
        return total
    total = {}
    for perm in itertools.permutations(range(n)):
        t = P.const(1, k)
        for i in range(n):
            t = P.mul(t, M[i][perm[i]])
        total = P.add(total, t)
    return total


def bareiss_int_no_swap_sign(M):
    n = len(M)
    A = [list(map(int, r)) for r in M]
    prev = 1
    for s in range(n - 1):
        if A[s][s] == 0:
            r = next((r for r in range(s + 1, n) if A[r][s] != 0), None)
            if r is None:
                return 0
            A[s], A[r] = A[r], A[s]
        for i in range(s + 1, n):
            for j in range(s + 1, n):
                A[i][j] = (A[s][s] * A[i][j] - A[i][s] * A[s][j]) // prev
        prev = A[s][s]
    return A[n - 1][n - 1] if n else 1


def bareiss_int_wrong_divisor(M):
    n = len(M)
    A = [list(map(int, r)) for r in M]
    sign = 1
    for s in range(n - 1):
        if A[s][s] == 0:
            r = next((r for r in range(s + 1, n) if A[r][s] != 0), None)
            if r is None:
                return 0
            A[s], A[r] = A[r], A[s]
            sign = -sign
        for i in range(s + 1, n):
            for j in range(s + 1, n):
                A[i][j] = A[s][s] * A[i][j] - A[i][s] * A[s][j]  # never divided
    return sign * A[n - 1][n - 1] if n else 1


def det_mod_no_swap_sign(A, p):
    n = len(A)
    A = [[int(x) % p for x in r] for r in A]
    det = 1
    for s in range(n):
        r = next((r for r in range(s, n) if A[r][s] != 0), None)
        if r is None:
            return 0
        A[s], A[r] = A[r], A[s]
        det = det * A[s][s] % p
        inv = pow(A[s][s], p - 2, p)
        for i in range(s + 1, n):
            f = A[i][s] * inv % p
            for j in range(s, n):
                A[i][j] = (A[i][j] - f * A[s][j]) % p
    return det


_orig_eval = OM.evaluate_at_node
_orig_interp = OM.interpolate_mod
_orig_garner = OM.garner
_orig_root = PL.root_of_unity
_orig_svand = OD.scaled_inverse_vandermonde
_orig_grid = PL.grid_sizes
_orig_bound = PL.det_degree_bound
_orig_primes = PL.ntt_primes


def eval_conjugate(entry, p, omegas, j):
    return _orig_eval(entry, p, [pow(w, p - 2, p) for w in omegas], j)


def interp_no_scale(values, p, omegas):
    out = _orig_interp(values, p, omegas)
    scale = 1
    for N in np.asarray(values).shape:
        scale = scale * N % p
    return np.asarray(out * scale % p, dtype=object)


def garner_unreduced_weight(residues, primes):
    pn = len(primes)
    alphas = []
    for i in range(pn):
        pi = primes[i]
        acc = 0
        mj = 1
        for j in range(i):
            acc = (acc + alphas[j] * mj) % pi
            mj *= primes[j]
        ci = pow(mj % pi, pi - 2, pi) if i else 1
        alphas.append((residues[i] - acc) * ci % pi)
    X = 0
    for i in reversed(range(pn)):
        X = X * primes[i] + alphas[i]
    M = 1
    for p in primes:
        M *= p
    return X - M if X >= (M - 1) // 2 else X  # and the boundary compared with >=


def garner_no_symmetric_range(residues, primes):
    out = _orig_garner(residues, primes)
    M = 1
    for p in primes:
        M *= p
    return out % M


def root_not_principal(p, N):
    return pow(2, (p - 1) // N, p)


def svand_transposed(D):
    return _orig_svand(D).T.copy()


def grid_too_small(D):
    return [PL.next_pow2(max(1, int(x))) for x in D]


def degree_bound_rows_only(arr):
    deg = PL.entry_degrees(arr)
    n, k = deg.shape[0], deg.shape[2]
    return [sum(max(0, int(deg[i, :, v].max())) for i in range(n)) - (1 if n > 1 else 0)
            for v in range(k)]


def primes_wrong_form(count):
    out = []
    c = ((1 << 30) - 1) >> 15
    while len(out) < count:
        q = c * (1 << 15) + 1
        if q < (1 << 30) and PL.is_prime(q):
            out.append(q)
        c -= 1
    return out


def num_primes_one_short(bound_sq, primes=None):
    t = 0
    prod = 1
    while True:
        p = primes[t] if primes is not None else _orig_primes(t + 1)[t]
        prod *= p
        t += 1
        if prod > bound_sq:  # compared with B^2 instead of 4 B^2 and without squaring M
            return t


def limbs_one_short(M):
    return max(1, M.bit_length() // 32)


def hadamard_rows_only_max(arr):
    arr = np.asarray(arr)
    n, k = arr.shape[0], arr.ndim - 2
    norms = [[P.norm1(P.from_box(arr[i, j], k)) for j in range(n)] for i in range(n)]
    out = 1
    for i in range(n):
        out *= max(x for x in norms[i]) ** 2
    return out


def poly_mul_dropped_term(a, b):
    out = {}
    items = sorted(b.items())
    for ea, ca in a.items():
        for eb, cb in items[1:] if len(items) > 2 else items:
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c}


MUTATIONS = [
    ("leibniz without permutation sign", OD, "det_leibniz", leibniz_no_sign),
    ("integer Bareiss without the sign of a row exchange", OD, "det_bareiss_int", bareiss_int_no_swap_sign),
    ("integer Bareiss without the exact division", OD, "det_bareiss_int", bareiss_int_wrong_divisor),
    ("determinant mod p without the sign of a row exchange", OM, "det_mod", det_mod_no_swap_sign),
    ("evaluation at conjugate nodes (w^-j)", OM, "evaluate_at_node", eval_conjugate),
    ("interpolation without the 1/N factor", OM, "interpolate_mod", interp_no_scale),
    ("Garner with unreduced weights and a shifted range boundary", OM, "garner", garner_unreduced_weight),
    ("Garner without the symmetric range", OM, "garner", garner_no_symmetric_range),
    ("root of unity from a non-generator", PL, "root_of_unity", root_not_principal),
    ("transposed inverse Vandermonde", OD, "scaled_inverse_vandermonde", svand_transposed),
    ("grid of next_pow2(D) points instead of next_pow2(D + 1)", PL, "grid_sizes", grid_too_small),
    ("degree bound from the rows only, one short", PL, "det_degree_bound", degree_bound_rows_only),
    ("primes 1 mod 2^15 instead of 1 mod 2^16", PL, "ntt_primes", primes_wrong_form),
    ("prime count from M > B^2 instead of M^2 > 4 B^2", PL, "num_primes", num_primes_one_short),
    ("one limb short", PL, "limbs_for", limbs_one_short),
    ("bound from the largest entry of each row only", PL, "hadamard_bound_sq", hadamard_rows_only_max),
    ("polynomial product dropping a term", P, "mul", poly_mul_dropped_term),
]


@pytest.mark.parametrize("label,target,attr,replacement", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, label, target, attr, replacement):
    random.seed(0)
    assert _caught(monkeypatch, target, attr, replacement) is not None, label


def test_unmutated_oracle_passes_the_same_pins():
    failed = []
    for name, call in _pin_calls():
        try:
            call()
        except Exception as e:  # pragma: no cover - reported below
            failed.append((name, repr(e)))
    assert not failed
