"""Dense multivariate integer polynomials as dicts (oracle; test infrastructure only).

A polynomial in k variables x1..xk is a dict {(e1, ..., ek): c} with c a nonzero Python
int. The zero polynomial is {}. The paper's input encoding (Section 2, FFT paragraph, the
worked example F = 1 + 2x + 3xy + 4x^2 + 5y^2 encoded as [1, 0, 5, 2, 3, 0, 4, 0, 0]) is a
dense box of coefficients in row-major order with the first variable slowest;
`from_box` / `to_box` convert between that box and the dict form.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Sequence, Tuple

Poly = Dict[Tuple[int, ...], int]


def from_box(box, k: int) -> Poly:
    """Dense coefficient box (nested sequences or numpy array, first variable slowest,
    index along axis v = exponent of x_v) -> dict polynomial. `k` is the number of axes."""
    out: Poly = {}
    if k == 0:
        c = int(box)
        return {(): c} if c else {}
    shape = []
    b = box
    for _ in range(k):
        shape.append(len(b))
        b = b[0]
    for e in itertools.product(*[range(s) for s in shape]):
        b = box
        for i in e:
            b = b[i]
        c = int(b)
        if c:
            out[tuple(e)] = c
    return out


def to_box(p: Poly, shape: Sequence[int]) -> list:
    """Dict polynomial -> flat list of the dense box of the given per-axis sizes, first
    variable slowest. Raises if a term does not fit in the box."""
    k = len(shape)
    size = 1
    for s in shape:
        size *= s
    flat = [0] * size
    for e, c in p.items():
        if len(e) != k or any(ei >= si for ei, si in zip(e, shape)):
            raise ValueError(f"term {e} outside box {tuple(shape)}")
        idx = 0
        for ei, si in zip(e, shape):
            idx = idx * si + ei
        flat[idx] = c
    return flat


def const(c: int, k: int) -> Poly:
    return {(0,) * k: c} if c else {}


def add(a: Poly, b: Poly) -> Poly:
    out = dict(a)
    for e, c in b.items():
        v = out.get(e, 0) + c
        if v:
            out[e] = v
        else:
            out.pop(e, None)
    return out


def neg(a: Poly) -> Poly:
    return {e: -c for e, c in a.items()}


def sub(a: Poly, b: Poly) -> Poly:
    return add(a, neg(b))


def mul(a: Poly, b: Poly) -> Poly:
    out: Poly = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c}


def scale(a: Poly, s: int) -> Poly:
    return {e: c * s for e, c in a.items()} if s else {}


def _lead(a: Poly) -> Tuple[int, ...]:
    # lexicographic order on exponent tuples: x1 > x2 > ... > xk
    return max(a)


def divexact(a: Poly, b: Poly) -> Poly:
    """Exact division a / b in Z[x1..xk] by multivariate long division in lex order.

    If b divides a, every step's leading term of the running remainder is divisible by the
    leading term of b (leading terms multiply in a monomial order), so the loop ends with a
    zero remainder. Raises ArithmeticError if the division is not exact."""
    if not b:
        raise ZeroDivisionError("division by the zero polynomial")
    lb = _lead(b)
    cb = b[lb]
    r = dict(a)
    q: Poly = {}
    while r:
        lr = _lead(r)
        cr = r[lr]
        if any(x < y for x, y in zip(lr, lb)) or cr % cb:
            raise ArithmeticError("polynomial division is not exact")
        e = tuple(x - y for x, y in zip(lr, lb))
        c = cr // cb
        q[e] = c
        r = sub(r, mul({e: c}, b))
    return q


def evaluate(a: Poly, point: Sequence[int], modulus: int | None = None) -> int:
    """Value of the polynomial at an integer point, exactly or modulo `modulus`."""
    total = 0
    for e, c in a.items():
        t = c
        for x, ei in zip(point, e):
            t = t * (pow(x, ei, modulus) if modulus else x ** ei)
            if modulus:
                t %= modulus
        total += t
    return total % modulus if modulus else total


def degree(a: Poly, v: int) -> int:
    """Degree in variable v (0-based); -1 for the zero polynomial."""
    return max((e[v] for e in a), default=-1)


def max_abs_coeff(a: Poly) -> int:
    return max((abs(c) for c in a.values()), default=0)


def norm1(a: Poly) -> int:
    return sum(abs(c) for c in a.values())


def matrix_from_array(arr, n: int, k: int):
    """n x n nested list of dict polynomials from a coefficient array of shape
    (n, n, d1+1, ..., dk+1) (numpy array or nested lists)."""
    return [[from_box(arr[i][j], k) for j in range(n)] for i in range(n)]


def matmul(A, B, k: int):
    """Product of two square matrices of dict polynomials."""
    n = len(A)
    out = []
    for i in range(n):
        row = []
        for j in range(n):
            s: Poly = {}
            for t in range(n):
                s = add(s, mul(A[i][t], B[t][j]))
            row.append(s)
        out.append(row)
    return out


def monomials(shape: Iterable[int]):
    return itertools.product(*[range(s) for s in shape])
