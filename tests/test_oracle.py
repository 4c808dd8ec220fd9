"""Pins for the oracle: each check ties the oracle to something other than itself (the
paper's worked examples, closed forms, an independent library routine, brute force on tiny
inputs, identities of the determinant). CPU only."""
import itertools
import json
import os
import random
from fractions import Fraction

import numpy as np
import pytest
import sympy

import workloads as W
from oracle import det as OD
from oracle import modular as OM
from oracle import plan as PL
from oracle import poly as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def rand_poly(rng, k, deg, amp=4, density=1.0):
    out = {}
    for e in itertools.product(*[range(d + 1) for d in deg]):
        if rng.random() < density:
            c = rng.randint(-amp, amp)
            if c:
                out[e] = c
    return out


def rand_matrix(rng, n, k, deg, amp=4, zero_prob=0.0):
    return [[{} if rng.random() < zero_prob else rand_poly(rng, k, deg, amp) for _ in range(n)]
            for _ in range(n)]


def to_sympy(p, syms):
    return sum((c * sympy.Mul(*[s ** e for s, e in zip(syms, ex)]) for ex, c in p.items()),
               sympy.Integer(0))


def from_sympy(expr, syms):
    if expr == 0:
        return {}
    poly = sympy.Poly(sympy.expand(expr), *syms)
    return {tuple(m): int(c) for m, c in zip(poly.monoms(), poly.coeffs())}


def matrix_to_array(M, n, k, deg):
    box = tuple(d + 1 for d in deg)
    arr = np.zeros((n, n) + box, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            flat = P.to_box(M[i][j], box)
            arr[i, j] = np.array(flat, dtype=np.int64).reshape(box)
    return arr


def box_to_poly(box):
    box = np.asarray(box, dtype=object)
    return {tuple(int(x) for x in idx): int(box[idx]) for idx in np.ndindex(box.shape)
            if box[idx] != 0}


# ---------------------------------------------------------------------------------------
# The paper's worked examples
# ---------------------------------------------------------------------------------------

def test_encoding_example_from_paper():
    g = golden()["encoding"]
    F = {tuple(e): c for e, c in g["terms"]}
    assert P.to_box(F, g["box"]) == g["vector"]
    back = P.from_box(np.array(g["vector"]).reshape(g["box"]), 2)
    assert back == F


def test_degree_enlargement_example_from_paper():
    g = golden()["degree_enlargement"]
    assert PL.enlarge_degrees(g["degrees"]) == g["enlarged"]
    assert max(g["enlarged"]) == 2 ** g["q_max"]


# ---------------------------------------------------------------------------------------
# Determinant by definition against an independent library and brute force
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,k", [(1, 2), (2, 1), (3, 2), (4, 2), (3, 3)])
def test_leibniz_matches_sympy(n, k):
    rng = random.Random(100 + 10 * n + k)
    syms = sympy.symbols(f"x0:{k}")
    M = rand_matrix(rng, n, k, [2] * k, amp=5, zero_prob=0.2)
    mine = OD.det_leibniz(M, k)
    ref = from_sympy(sympy.Matrix([[to_sympy(e, syms) for e in row] for row in M]).det(
        method="berkowitz"), syms)
    assert mine == ref


@pytest.mark.parametrize("n,k,deg,zp", [(1, 2, (2, 2), 0.0), (2, 2, (1, 2), 0.0),
                                        (3, 1, (3,), 0.3), (4, 2, (2, 1), 0.3),
                                        (5, 2, (1, 1), 0.4), (4, 3, (1, 1, 1), 0.0),
                                        (5, 1, (2,), 0.5)])
def test_bareiss_poly_matches_leibniz(n, k, deg, zp):
    rng = random.Random(7 * n + k)
    M = rand_matrix(rng, n, k, list(deg), amp=6, zero_prob=zp)
    assert OD.det_bareiss_poly(M, k) == OD.det_leibniz(M, k)


def test_bareiss_poly_needs_pivoting():
    # zero leading entries force row exchanges at every step
    k = 1
    x = {(1,): 1}
    one = {(0,): 1}
    M = [[{}, x, one], [one, {}, x], [x, one, {}]]
    assert OD.det_bareiss_poly(M, k) == OD.det_leibniz(M, k)
    # a column that vanishes below the pivot after elimination -> singular
    S = [[x, x], [x, x]]
    assert OD.det_bareiss_poly(S, k) == {}


@pytest.mark.parametrize("n,k,deg", [(1, 2, (3, 1)), (2, 2, (2, 2)), (3, 2, (2, 1)),
                                     (4, 2, (1, 2)), (3, 3, (1, 1, 2)), (5, 1, (2,)),
                                     (4, 0, ())])
def test_pointwise_matches_bareiss_poly(n, k, deg):
    rng = random.Random(11 * n + 3 * k)
    M = rand_matrix(rng, n, k, list(deg), amp=7, zero_prob=0.25)
    arr = matrix_to_array(M, n, k, deg)
    D = PL.det_degree_bound_from_shape(n, deg)
    boxB = OD.det_pointwise(arr, D)
    A = OD.det_bareiss_poly(M, k)
    assert box_to_poly(boxB) == A


def test_config1_oracles_agree():
    arr = W.config1()
    n, k = 4, 2
    M = P.matrix_from_array(arr, n, k)
    A = OD.det_bareiss_poly(M, k)
    D = PL.det_degree_bound_from_shape(n, [2, 2])
    B = OD.det_pointwise(arr, D)
    assert box_to_poly(B) == A
    assert A  # a random dense 4x4 has a nonzero determinant


def test_config2_shape_downscaled_oracles_agree():
    # same structure as the 12 x 12 trivariate case (30% zero entries), n = 5
    arr = W.config2(n=5, deg=(1, 1, 1))
    M = P.matrix_from_array(arr, 5, 3)
    A = OD.det_bareiss_poly(M, 3)
    B = OD.det_pointwise(arr, PL.det_degree_bound_from_shape(5, (1, 1, 1)))
    assert box_to_poly(B) == A


def test_config4_digest_file_agrees_with_bareiss_over_polynomials():
    """The stored digests of the batching workload (written from the pointwise oracle) match,
    for the 24 cheapest matrices, the fraction-free Bareiss elimination over Z[x1..xk]: the
    other realisation of the oracle, which shares no evaluation or interpolation code."""
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_config4_digests as MD
    import hashlib
    stored = json.load(open(MD.OUT))["digests"]
    idx, shapes = MD.ranked_indices(0.75)
    assert sorted(int(i) for i in stored) == sorted(idx)
    mats = W.config4()
    for i in idx[:24]:
        a = mats[i]
        n, k = a.shape[0], a.ndim - 2
        A = OD.det_bareiss_poly(P.matrix_from_array(a, n, k), k)
        text = ";".join(".".join(str(e) for e in key) + ":" + str(A[key]) for key in sorted(A))
        assert hashlib.sha256(text.encode()).hexdigest()[:16] == stored[str(i)], i


# ---------------------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------------------

def test_vandermonde_closed_form():
    # Theorem 1's Vandermonde matrix with polynomial nodes t_i: det = prod_{i<j} (t_j - t_i)
    rng = random.Random(5)
    k, n = 2, 4
    ts = [rand_poly(rng, k, [1, 1], amp=3) for _ in range(n)]
    V = []
    for i in range(n):
        row = [P.const(1, k)]
        for _ in range(1, n):
            row.append(P.mul(row[-1], ts[i]))
        V.append(row)
    expect = P.const(1, k)
    for i in range(n):
        for j in range(i + 1, n):
            expect = P.mul(expect, P.sub(ts[j], ts[i]))
    assert OD.det_bareiss_poly(V, k) == expect
    deg = [max(P.degree(V[i][j], v) for i in range(n) for j in range(n)) for v in range(k)]
    arr = matrix_to_array(V, n, k, deg)
    assert box_to_poly(OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, deg))) == expect


def _factor_poly(a_box):
    return box_to_poly(a_box)


def test_sylvester_resultant_closed_form_small():
    # f = prod (a_i x - b_i), g = prod (c_j x - d_j): Res_x(f, g) = prod_{i,j} (b_i c_j - a_i d_j)
    rng = np.random.default_rng(77)
    ff = W.factored_linear(rng, 3, 2, 2, (2, 2))
    gf = W.factored_linear(rng, 2, 2, 1, (2, 2))
    box = (5, 5)
    f = W.expand_linear_product(ff, box)
    g = W.expand_linear_product(gf, box)
    S = W.sylvester(f, g)
    n = S.shape[0]
    expect = P.const(1, 2)
    for a, b in ff:
        for c, d in gf:
            term = P.sub(P.mul(_factor_poly(b), _factor_poly(c)), P.mul(_factor_poly(a), _factor_poly(d)))
            expect = P.mul(expect, term)
    M = P.matrix_from_array(S, n, 2)
    assert OD.det_bareiss_poly(M, 2) == expect
    # and an independent library routine: sympy's resultant of the expanded polynomials
    x, y, z = sympy.symbols("x y z")
    fx = sum(to_sympy(box_to_poly(f[i]), (y, z)) * x ** i for i in range(f.shape[0]))
    gx = sum(to_sympy(box_to_poly(g[i]), (y, z)) * x ** i for i in range(g.shape[0]))
    assert from_sympy(sympy.resultant(fx, gx, x), (y, z)) == expect


def test_triangular_is_product_of_diagonal():
    rng = random.Random(9)
    k, n = 2, 5
    M = [[rand_poly(rng, k, [2, 1]) if j >= i else {} for j in range(n)] for i in range(n)]
    expect = P.const(1, k)
    for i in range(n):
        expect = P.mul(expect, M[i][i])
    assert OD.det_bareiss_poly(M, k) == expect
    arr = matrix_to_array(M, n, k, (2, 1))
    assert box_to_poly(OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, (2, 1)))) == expect


def test_det_of_product():
    rng = random.Random(13)
    k, n = 2, 3
    A = rand_matrix(rng, n, k, [1, 1], amp=4)
    B = rand_matrix(rng, n, k, [1, 1], amp=4)
    AB = P.matmul(A, B, k)
    lhs = OD.det_bareiss_poly(AB, k)
    rhs = P.mul(OD.det_bareiss_poly(A, k), OD.det_bareiss_poly(B, k))
    assert lhs == rhs
    arr = matrix_to_array(AB, n, k, (2, 2))
    assert box_to_poly(OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, (2, 2)))) == rhs


def test_integer_matrices_k0():
    rng = random.Random(21)
    for n in range(1, 7):
        for _ in range(5):
            M = [[rng.randint(-50, 50) if rng.random() > 0.3 else 0 for _ in range(n)]
                 for _ in range(n)]
            f = OD.det_fraction(M)
            assert OD.det_bareiss_int(M) == f
            assert OD.det_leibniz(M) == f
            assert int(sympy.Matrix(M).det()) == f


def test_singular_and_extreme_integer_matrices():
    big = 2 ** 63 - 1
    M = [[big, -big - 1], [-(2 ** 62), 2 ** 62]]
    assert OD.det_bareiss_int(M) == big * 2 ** 62 - (big + 1) * 2 ** 62
    assert OD.det_bareiss_int([[1, 2, 3], [2, 4, 6], [0, 1, 5]]) == 0
    assert OD.det_bareiss_int([[0, 0], [0, 0]]) == 0


def test_scaled_inverse_vandermonde():
    for D in range(0, 9):
        V = OD.vandermonde_int(D)
        W_ = OD.scaled_inverse_vandermonde(D)
        prod = V.dot(W_)
        fD = 1
        for i in range(2, D + 1):
            fD *= i
        for i in range(D + 1):
            for j in range(D + 1):
                assert prod[i, j] == (fD if i == j else 0)


# ---------------------------------------------------------------------------------------
# Plan quantities
# ---------------------------------------------------------------------------------------

def test_ntt_primes_against_sympy():
    ps = PL.ntt_primes(40)
    assert ps == sorted(ps, reverse=True)
    assert len(set(ps)) == 40
    for p in ps:
        assert sympy.isprime(p)
        assert (p - 1) % (1 << 16) == 0
        assert (1 << 29) < p < (1 << 30)
    # no prime of that form is skipped between the first and the last
    lo, hi = ps[-1], ps[0]
    step = 1 << 16
    expect = [c * step + 1 for c in range(hi // step, lo // step - 1, -1)
              if lo <= c * step + 1 <= hi and sympy.isprime(c * step + 1)]
    assert expect == ps


def test_prime_supply_count():
    # how many primes of the form c * 2^16 + 1 exist in (2^29, 2^30)
    step = 1 << 16
    count = sum(1 for c in range((1 << 29) // step, (1 << 30) // step)
                if c * step + 1 > (1 << 29) and sympy.isprime(c * step + 1))
    assert count == 784
    assert PL.ntt_primes(1) == [1073479681]
    assert PL.is_prime(1073479681) and not PL.is_prime(1073479681 + step)


@pytest.mark.parametrize("N", [1, 2, 4, 16, 64, 1024, 65536])
def test_roots_of_unity(N):
    for p in PL.ntt_primes(3):
        w = PL.root_of_unity(p, N)
        assert pow(w, N, p) == 1
        if N > 1:
            assert pow(w, N // 2, p) == p - 1
        g = PL.primitive_root(p)
        assert sympy.is_primitive_root(g, p)
        assert all(not sympy.is_primitive_root(h, p) for h in range(2, g))


def test_grid_rule_and_degree_bounds():
    assert PL.grid_sizes([8, 8]) == [16, 16]
    assert PL.grid_sizes([36, 36, 36]) == [64, 64, 64]
    assert PL.grid_sizes([88, 88]) == [128, 128]
    assert PL.grid_sizes([0, 15, 16]) == [1, 16, 32]
    assert PL.det_degree_bound_from_shape(12, (3, 3, 3)) == [36, 36, 36]
    rng = random.Random(3)
    for _ in range(20):
        n = rng.randint(1, 4)
        k = rng.randint(1, 2)
        deg = [rng.randint(0, 2) for _ in range(k)]
        M = rand_matrix(rng, n, k, deg, zero_prob=0.3)
        arr = matrix_to_array(M, n, k, deg)
        d = OD.det_leibniz(M, k)
        bound = PL.det_degree_bound(arr)
        for v in range(k):
            assert P.degree(d, v) <= bound[v] <= n * deg[v]


def test_hadamard_bound_holds():
    rng = random.Random(17)
    worst = 0.0
    for _ in range(30):
        n = rng.randint(1, 5)
        k = rng.randint(0, 2)
        deg = [rng.randint(0, 2) for _ in range(k)]
        M = rand_matrix(rng, n, k, deg, amp=rng.choice([1, 10, 1000]), zero_prob=0.2)
        arr = matrix_to_array(M, n, k, deg)
        B2 = PL.hadamard_bound_sq(arr)
        d = OD.det_leibniz(M, k)
        c = P.max_abs_coeff(d)
        assert c * c <= B2
        if B2:
            worst = max(worst, c * c / B2)
    assert worst <= 1.0


def test_num_primes_is_minimal():
    ps = PL.ntt_primes(10)
    for B2 in [0, 1, 2 ** 60, 2 ** 61, 2 ** 200, 3 ** 300]:
        t = PL.num_primes(B2, ps)
        prod = 1
        for p in ps[:t]:
            prod *= p
        assert prod * prod > 4 * B2
        prod_less = prod // ps[t - 1]
        assert t == 1 or prod_less * prod_less <= 4 * B2


# ---------------------------------------------------------------------------------------
# Modular steps
# ---------------------------------------------------------------------------------------

def test_garner_matches_naive_crt_and_roundtrips():
    rng = random.Random(23)
    for pn in [1, 2, 3, 7, 15, 27]:
        ps = PL.ntt_primes(pn)
        M = 1
        for p in ps:
            M *= p
        half = (M - 1) // 2
        for x in [0, 1, -1, half, -half, half - 1, -half + 1] + [rng.randint(-half, half)
                                                                 for _ in range(20)]:
            res = [x % p for p in ps]
            assert OM.garner(res, ps) == x
            assert OM.crt_naive(res, ps) == x
        for _ in range(10):
            res = [rng.randrange(p) for p in ps]
            assert OM.garner(res, ps) == OM.crt_naive(res, ps)


def test_det_mod_matches_leibniz_mod_p():
    rng = random.Random(29)
    p = PL.ntt_primes(1)[0]
    for n in range(1, 7):
        for _ in range(5):
            A = [[rng.randrange(p) if rng.random() > 0.3 else 0 for _ in range(n)] for _ in range(n)]
            assert OM.det_mod(A, p) == OD.det_leibniz(A) % p
    # adversarial: all p-1, permutation matrices, rank deficient
    assert OM.det_mod([[p - 1] * 3] * 3, p) == 0
    perm = [[0, 1, 0], [0, 0, 1], [1, 0, 0]]
    assert OM.det_mod(perm, p) == 1
    perm2 = [[0, 1, 0], [1, 0, 0], [0, 0, 1]]
    assert OM.det_mod(perm2, p) == p - 1


def test_interpolation_inverts_evaluation():
    rng = random.Random(31)
    p = PL.ntt_primes(1)[0]
    N = [4, 8]
    omegas = [PL.root_of_unity(p, x) for x in N]
    f = {(i, j): rng.randrange(p) for i in range(4) for j in range(8)}
    vals = np.empty(tuple(N), dtype=object)
    for j in itertools.product(range(4), range(8)):
        vals[j] = OM.evaluate_at_node(f, p, omegas, j)
    back = OM.interpolate_mod(vals, p, omegas)
    for e in itertools.product(range(4), range(8)):
        assert back[e] == f.get(e, 0)


def test_modular_method_matches_bareiss():
    rng = random.Random(37)
    for n, k, deg in [(3, 2, (1, 1)), (2, 1, (3,)), (3, 0, ()), (1, 2, (2, 1))]:
        M = rand_matrix(rng, n, k, list(deg), amp=9, zero_prob=0.2)
        arr = matrix_to_array(M, n, k, deg)
        box, info = OM.modular_determinant(arr)
        assert box_to_poly(box) == OD.det_bareiss_poly(M, k)
        # extra primes and a disjoint prime set do not change the result
        box2, _ = OM.modular_determinant(arr, extra_primes=2)
        assert box_to_poly(box2) == box_to_poly(box)
        box3, _ = OM.modular_determinant(arr, primes=PL.ntt_primes(info["pn"] + 3)[info["pn"]:])
        assert box_to_poly(box3) == box_to_poly(box)


def test_modular_stage_values_match_oracle_polynomial():
    # the determinant mod p at each node equals the exact determinant polynomial reduced
    # mod p and evaluated at that node
    rng = random.Random(41)
    M = rand_matrix(rng, 3, 2, [1, 1], amp=9)
    arr = matrix_to_array(M, 3, 2, (1, 1))
    _, info = OM.modular_determinant(arr)
    exact = OD.det_bareiss_poly(M, 2)
    for pp in info["per_prime"]:
        p = pp["p"]
        for j in itertools.product(*[range(x) for x in info["N"]]):
            assert pp["dets"][j] == OM.evaluate_at_node(exact, p, pp["omegas"], j)


def test_evaluation_exponent_sign_and_root_against_sympy_ntt():
    # the node j of variable v is w_v^{+j}: evaluating x alone at node 1 gives w itself, and a
    # dense univariate entry at every node equals sympy's number-theoretic transform (which
    # takes the same root, the least primitive root raised to (p-1)/N)
    from sympy.discrete.transforms import intt, ntt
    p = PL.ntt_primes(3)[2]
    for N in (4, 16):
        w = PL.root_of_unity(p, N)
        assert OM.evaluate_at_node({(1,): 1}, p, [w], [1]) == w
        assert OM.evaluate_at_node({(1,): 1}, p, [w], [3]) == pow(w, 3, p)
        rng = random.Random(N)
        coeffs = [rng.randrange(p) for _ in range(N)]
        f = {(e,): c for e, c in enumerate(coeffs)}
        vals = [OM.evaluate_at_node(f, p, [w], [j]) for j in range(N)]
        assert vals == [int(x) for x in ntt(coeffs, p)]
        back = OM.interpolate_mod(np.array(vals, dtype=object), p, [w])
        assert [int(x) for x in back] == [int(x) for x in intt(vals, p)] == coeffs
    # bivariate: x y^2 at (j1, j2) is w1^j1 w2^(2 j2)
    w1, w2 = PL.root_of_unity(p, 8), PL.root_of_unity(p, 4)
    assert OM.evaluate_at_node({(1, 2): 1}, p, [w1, w2], [3, 1]) == pow(w1, 3, p) * pow(w2, 2, p) % p


def test_limbs_for_is_the_twos_complement_width():
    # L limbs hold every x with |x| <= (M-1)/2 as a two's-complement integer of 32 L bits, and
    # L - 1 limbs do not (Python's own signed encoding is the reference)
    ps = PL.ntt_primes(5)
    prods = [1]
    for p in ps:
        prods.append(prods[-1] * p)
    for M in [3, 2 ** 32 - 1, 2 ** 32 + 1, 2 ** 33 - 1, 2 ** 64 - 1, 2 ** 64 + 1, 2 ** 96 + 3] + prods[1:]:
        L = PL.limbs_for(M)
        half = (M - 1) // 2
        for x in (half, -half):
            x.to_bytes(4 * L, "little", signed=True)
        if L > 1:
            with pytest.raises(OverflowError):
                half.to_bytes(4 * (L - 1), "little", signed=True)
    assert PL.limbs_for(2 ** 32 - 1) == 1 and PL.limbs_for(2 ** 32 + 1) == 2
