"""Parity of the HIP path with the oracle (GPU). Every comparison is bit-exact: the path
computes exact integers.

Oracle A (Bareiss over Z[x]) covers small cases, oracle B (pointwise integer Bareiss with
exact interpolation) covers the larger ones; stage checks compare the workspace after a
solve with the oracle's modular steps at every or at sampled grid points."""
import itertools
import multiprocessing as mp
import random

import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W
from oracle import det as OD
from oracle import modular as OM
from oracle import plan as PL
from oracle import poly as P

from helpers import box_to_dict, mont_to_plain, node_index, supported_lanes

pytestmark = pytest.mark.gpu


def gpu_solve(arr, flags=0, use_coeffs=True):
    import torch
    arr = np.ascontiguousarray(arr, dtype=np.int64)
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr if use_coeffs else None,
                  coeff_bits=None if use_coeffs else B.coeff_bits_of(arr), flags=flags)
    d = torch.from_numpy(arr).cuda()
    out, ws = pdm.solve_device(pl, d)
    torch.cuda.synchronize()
    vals = B.limbs_to_ints(out.cpu().numpy())
    box = tuple(x + 1 for x in pl.info["D"])
    res = np.empty(len(vals), dtype=object)
    for i, v in enumerate(vals):
        res[i] = v
    return res.reshape(box) if box else res.reshape(()), pl, ws


def det_regions(pl, ws):
    """(numerators, denominators) per (prime, point), uint32 [pn][G] (Montgomery form)."""
    info = pl.info
    nb = 4 * info["pn"] * info["G"]
    w = ws.cpu().numpy()
    num = w[info["off_detv"]:info["off_detv"] + nb].view(np.uint32).reshape(info["pn"], info["G"])
    den = w[info["off_den"]:info["off_den"] + nb].view(np.uint32).reshape(info["pn"], info["G"])
    return num, den


def assert_same_fractions(pla, wsa, plb, wsb):
    """Both solves left the same determinant num / den mod p at every (prime, point), and no
    zero denominator. (The two-column condensation and the left-looking pass reach the same
    quotient through different numerators and denominators, so the pairs are compared by
    cross-multiplication: num_a den_b = num_b den_a mod p; the Montgomery factors cancel.)"""
    na, da = det_regions(pla, wsa)
    nb, db = det_regions(plb, wsb)
    assert pla.info["primes"] == plb.info["primes"]
    assert da.all() and db.all()
    for q, p in enumerate(pla.info["primes"]):
        lhs = na[q].astype(np.uint64) * db[q].astype(np.uint64) % np.uint64(p)
        rhs = nb[q].astype(np.uint64) * da[q].astype(np.uint64) % np.uint64(p)
        assert np.array_equal(lhs, rhs)


def oracle_box(arr):
    n, deg = B.shape_of(arr)
    return OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, deg))


def oracle_poly(arr):
    n, deg = B.shape_of(arr)
    return OD.det_bareiss_poly(P.matrix_from_array(arr, n, len(deg)), len(deg))


@pytest.fixture(scope="module")
def pool():
    ctx = mp.get_context("spawn")
    p = ctx.Pool(min(16, mp.cpu_count()))
    yield p
    p.close()
    p.join()


def test_config1_bit_exact():
    arr = W.config1()
    got, pl, _ = gpu_solve(arr)
    assert box_to_dict(got) == oracle_poly(arr)
    assert box_to_dict(got) == box_to_dict(oracle_box(arr))


CASES = [
    # (n, deg, amp, zero_prob, seed)
    (1, (3, 2), 50, 0.0, 1), (2, (1, 1), 9, 0.0, 2), (3, (2,), 100, 0.3, 3),
    (4, (1, 1, 1), 7, 0.3, 4), (5, (2, 1), 1000, 0.4, 5), (6, (1, 1), 3, 0.5, 6),
    (3, (), 10 ** 6, 0.2, 7), (7, (1,), 2 ** 20, 0.2, 8), (4, (5, 3), 30, 0.1, 9),
    (2, (7, 1, 1, 1), 5, 0.0, 10), (3, (1, 1, 1, 1, 1), 4, 0.0, 11), (8, (1, 1), 2, 0.6, 12),
]


@pytest.mark.parametrize("n,deg,amp,zp,seed", CASES)
def test_small_random_cases(n, deg, amp, zp, seed):
    rng = np.random.default_rng(seed)
    arr = W.random_matrix(rng, n, deg, -amp, amp, zero_prob=zp)
    got, _, _ = gpu_solve(arr)
    expect = oracle_poly(arr) if n <= 5 else box_to_dict(oracle_box(arr))
    assert box_to_dict(got) == expect


@pytest.mark.parametrize("n", list(range(1, 33)))
def test_every_order_default_lanes(n):
    rng = np.random.default_rng(1000 + n)
    arr = W.random_matrix(rng, n, (1,), -20, 20, zero_prob=0.2)
    got, _, _ = gpu_solve(arr)
    assert box_to_dict(got) == box_to_dict(oracle_box(arr))


LANE_CASES = [(n, gl) for n in (2, 4, 7, 8, 12, 13, 16, 17, 22, 24, 25, 31, 32)
              for gl in supported_lanes(n)]

# first variable of degree 4 or 5 (5 or 6 coefficients): the paired evaluation with three terms
# per lane, at every lane mapping of these orders
PAIR3_ORDERS = {3: 4, 8: 5, 12: 4, 13: 5, 16: 4, 17: 5, 24: 4, 25: 5, 32: 5}
PAIR3_CASES = [(n, gl) for n in PAIR3_ORDERS for gl in supported_lanes(n)]
_pair3_oracle = {}


@pytest.mark.parametrize("n,lanes", LANE_CASES)
def test_every_lane_mapping(n, lanes):
    rng = np.random.default_rng(2000 + 40 * n + lanes)
    arr = W.random_matrix(rng, n, (1,), -9, 9, zero_prob=0.35)
    log2 = {1: 0, 2: 1, 4: 2, 8: 3, 16: 4}[lanes]
    got, pl, _ = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2) | pdm.DET_EXCHANGE)
    assert pl.info["det_lanes"] == lanes
    assert box_to_dict(got) == box_to_dict(oracle_box(arr))


@pytest.mark.parametrize("n,lanes", PAIR3_CASES)
def test_three_term_pairing_every_lane_mapping(n, lanes):
    rng = np.random.default_rng(2500 + n)
    arr = W.random_matrix(rng, n, (PAIR3_ORDERS[n],), -9, 9, zero_prob=0.3)
    log2 = {1: 0, 2: 1, 4: 2, 8: 3, 16: 4}[lanes]
    got, pl, _ = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2) | pdm.DET_EXCHANGE)
    assert pl.info["det_lanes"] == lanes
    if n not in _pair3_oracle:
        _pair3_oracle[n] = box_to_dict(oracle_box(arr))
    assert box_to_dict(got) == _pair3_oracle[n]


def vanishing_pivots(rng, n, deg, kind):
    """Random matrix whose elimination meets a zero pivot at some grid points whatever row
    order is taken. kind 0: column 0 is (x1 - 1, x1 + 1, 0, ..., 0), so the first pivot
    vanishes at x1 = 1 or at x1 = -1 (both on every grid). kind 1: the leading 2 x 2 block
    is [[1, x1], [1, 1]] with zeros below it in columns 0 and 1, so the second pivot is
    1 - x1 or x1 - 1."""
    a = W.random_matrix(rng, n, deg, -20, 20, zero_prob=0.2)
    one = np.zeros(a.shape[2:], dtype=np.int64)
    one[(0,) * len(deg)] = 1
    x1 = np.zeros_like(one)
    x1[(1,) + (0,) * (len(deg) - 1)] = 1
    a[:, 0] = 0
    if kind == 0:
        a[0, 0] = x1 - one
        if n > 1:
            a[1, 0] = x1 + one
    else:
        a[:, 1] = 0
        a[0, 0], a[0, 1], a[1, 0], a[1, 1] = one, x1, one, one
    return a


LL_CASES = [(n, kind) for n in (2, 3, 5, 8, 11, 12, 13, 16) for kind in (0, 1)]


@pytest.mark.parametrize("n,kind", LL_CASES)
def test_left_looking_repairs_zero_pivots(n, kind):
    # the left-looking pass cannot exchange rows: points where a pivot vanishes mod p are
    # recomputed by the exchanging kernel, and the result equals the exchanging kernel's
    # at every grid point
    rng = np.random.default_rng(700 + 2 * n + kind)
    arr = vanishing_pivots(rng, n, (2, 1), kind)
    a, pla, wsa = gpu_solve(arr, flags=pdm.DET_LEFT_LOOKING)
    b, plb, wsb = gpu_solve(arr, flags=pdm.DET_EXCHANGE)
    assert pla.info["det_left_looking"] == 1 and plb.info["det_left_looking"] == 0
    assert box_to_dict(a) == box_to_dict(b) == box_to_dict(oracle_box(arr))
    assert_same_fractions(pla, wsa, plb, wsb)


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_left_looking_every_order(n):
    rng = np.random.default_rng(800 + n)
    arr = W.random_matrix(rng, n, (3, 1), -30, 30, zero_prob=0.3)
    a, _, _ = gpu_solve(arr, flags=pdm.DET_LEFT_LOOKING)
    b, _, _ = gpu_solve(arr, flags=pdm.DET_EXCHANGE)
    assert box_to_dict(a) == box_to_dict(b) == box_to_dict(oracle_box(arr))


def test_integer_matrices_extreme_values():
    # k = 0: the plain integer determinant, with int64 extremes
    rng = random.Random(5)
    for n in [1, 2, 3, 5, 8, 12]:
        M = [[rng.choice([0, 1, -1, 2 ** 63 - 1, -(2 ** 63), rng.randint(-2 ** 62, 2 ** 62)])
              for _ in range(n)] for _ in range(n)]
        arr = np.array(M, dtype=np.int64)
        got, _, _ = gpu_solve(arr)
        assert int(got[()]) == OD.det_bareiss_int(M)
    for n in [20, 32]:
        M = [[rng.randint(-2 ** 20, 2 ** 20) for _ in range(n)] for _ in range(n)]
        got, _, _ = gpu_solve(np.array(M, dtype=np.int64))
        assert int(got[()]) == OD.det_bareiss_int(M)


def test_singular_and_structured():
    rng = np.random.default_rng(44)
    # duplicated row -> 0
    a = W.random_matrix(rng, 6, (2, 1), -30, 30)
    a[3] = a[1]
    got, _, _ = gpu_solve(a)
    assert box_to_dict(got) == {}
    # zero matrix and zero column
    z = np.zeros((5, 5, 2, 2), dtype=np.int64)
    got, _, _ = gpu_solve(z)
    assert box_to_dict(got) == {}
    b = W.random_matrix(rng, 5, (1, 1), -5, 5)
    b[:, 2] = 0
    got, _, _ = gpu_solve(b)
    assert box_to_dict(got) == {}
    # permutation matrix of constants (every pivot needs an exchange)
    perm = [3, 0, 4, 1, 2]
    c = np.zeros((5, 5, 1), dtype=np.int64)
    for i, j in enumerate(perm):
        c[i, j, 0] = 1
    got, _, _ = gpu_solve(c)
    assert box_to_dict(got) == oracle_poly(c)
    # triangular with polynomial diagonal
    t = np.triu(np.ones((6, 6), dtype=np.int64))[:, :, None, None] * \
        W.random_matrix(rng, 6, (1, 2), -4, 4)
    got, _, _ = gpu_solve(t)
    assert box_to_dict(got) == box_to_dict(oracle_box(t))


def test_invariance_to_primes_and_bound():
    arr = W.random_matrix(np.random.default_rng(8), 6, (2, 2), -500, 500, zero_prob=0.3)
    base, pl, _ = gpu_solve(arr)
    pn = pl.info["pn"]
    more, _, _ = gpu_solve(arr, flags=pdm.FORCE_PN(pn + 2))
    disjoint, _, _ = gpu_solve(arr, flags=pdm.PRIME_OFFSET(pn + 5))
    worst, plw, _ = gpu_solve(arr, use_coeffs=False)
    assert plw.info["pn"] >= pn
    for other in (more, disjoint, worst):
        assert box_to_dict(other) == box_to_dict(base)


def test_stages_against_oracle_steps():
    # S2 values at every node, S3 determinants at every node, S4 coefficients mod p
    import torch
    arr = W.random_matrix(np.random.default_rng(9), 3, (2, 1), -40, 40, zero_prob=0.2)
    arr[0, 0] = 0  # a structurally zero pivot: the plan reorders the rows
    got, pl, ws = gpu_solve(arr, flags=pdm.FORCE_PN(2) | pdm.UNFUSED_EVAL)
    assert pl.info["row_order"][0] != 0 and pl.info["det_sign"] == -1
    info = pl.info
    n, k = 3, 2
    N = info["N"]
    G = info["G"]
    w = ws.cpu().numpy()
    ev = w[info["off_eval"]:info["off_eval"] + 4 * info["pn"] * n * n * G].view(np.uint32)
    ev = ev.reshape(info["pn"], n * n, G)
    num, den = det_regions(pl, ws)
    cf = w[info["off_coef"]:info["off_coef"] + 4 * info["pn"] * info["ncoeff"]].view(np.uint32)
    cf = cf.reshape(info["pn"], info["ncoeff"])
    M = P.matrix_from_array(arr, n, k)
    exact = oracle_poly(arr)
    box = tuple(d + 1 for d in info["D"])
    order = info["row_order"]
    assert sorted(order) == list(range(n))
    for q, p in enumerate(info["primes"]):
        omegas = [PL.root_of_unity(p, x) for x in N]
        for j in itertools.product(*[range(x) for x in N]):
            idx = node_index(j, N)
            A = [[OM.evaluate_at_node(M[r][c], p, omegas, j) for c in range(n)] for r in range(n)]
            for r in range(n):
                for c in range(n):
                    # row r of the eliminated matrix is input row order[r]
                    assert mont_to_plain(ev[q, r * n + c, idx], p) == A[order[r]][c]
            d = mont_to_plain(num[q, idx], p) * pow(mont_to_plain(den[q, idx], p), p - 2, p)
            assert d % p == info["det_sign"] * OM.det_mod(A, p) % p
        for e in itertools.product(*[range(b) for b in box]):
            ci = node_index(e, box)
            # the interpolation leaves the factor G (and the row-order sign) for the
            # reconstruction
            assert mont_to_plain(cf[q, ci], p) == info["det_sign"] * exact.get(e, 0) * G % p


# first-variable coefficient counts: 2-4 (paired, two terms per lane), 5-6 (paired, three),
# 1 and 7 (term by term)
FUSE_CASES = [(3, (2, 1), 1), (12, (3, 3, 3), 1), (13, (1, 2), 2), (22, (2, 1), 4),
              (17, (1, 1, 1), 8), (30, (1, 2), 16), (9, (4,), 1), (5, (2, 0, 1), 2),
              (14, (5, 1), 2), (20, (4, 1), 4), (11, (5, 1, 1), 1), (19, (6,), 4),
              (10, (0, 2), 1), (26, (4, 1), 8)]


@pytest.mark.parametrize("n,deg,lanes", FUSE_CASES)
def test_fused_matches_unfused_and_stage_values(n, deg, lanes):
    # the fused first-variable evaluation gives the same determinant at every grid point as
    # the full evaluation tensor, including padded columns of the last lane slot
    rng = np.random.default_rng(300 + n)
    arr = W.random_matrix(rng, n, deg, -99, 99, zero_prob=0.3)
    log2 = {1: 0, 2: 1, 4: 2, 8: 3, 16: 4}[lanes]
    a, pla, wsa = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2))
    b, plb, wsb = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2) | pdm.UNFUSED_EVAL)
    assert box_to_dict(a) == box_to_dict(b)
    assert_same_fractions(pla, wsa, plb, wsb)


def test_config2_bit_exact(pool):
    arr = W.config2()
    got, pl, _ = gpu_solve(arr)
    assert pl.info["pn"] == 7 and pl.info["N"] == (64, 64, 64)
    expect = OD.det_pointwise(arr, PL.det_degree_bound_from_shape(12, (3, 3, 3)), pool=pool)
    assert box_to_dict(got) == box_to_dict(expect)


def test_config3a_sylvester_bit_exact(pool):
    arr = W.config3a()
    got, pl, _ = gpu_solve(arr)
    assert pl.info["N"] == (128, 128)
    expect = OD.det_pointwise(arr, PL.det_degree_bound_from_shape(22, (4, 4)), pool=pool)
    assert box_to_dict(got) == box_to_dict(expect)


def test_config3b_resultant_closed_form():
    S, ff, gf = W.config3b()
    got, _, _ = gpu_solve(S)
    expect = P.const(1, 2)
    for a, b in ff:
        for c, d in gf:
            term = P.sub(P.mul(box_to_dict(b), box_to_dict(c)), P.mul(box_to_dict(a), box_to_dict(d)))
            expect = P.mul(expect, term)
    assert box_to_dict(got) == expect


# shapes for the reduction folded into the first evaluation pass and the reconstruction folded
# into the last interpolation pass: last variables of degree 0, a 1 x 1 grid, three variables,
# the reconstruction's 16- and 32-prime forms (10 primes from the bound, 20 forced)
FOLD_CASES = [(4, (2, 0), 10 ** 6, 31, 0), (3, (0, 0), 10 ** 6, 32, 0),
              (5, (1, 0, 2), 10 ** 3, 33, 0), (6, (3, 1), 2 ** 45, 34, 0), (4, (2, 1), 10, 35, 20)]


def check_against_stages(arr, pl, ref):
    """The plan run one stage at a time (separate reduction, interpolation passes and
    reconstruction) gives the solve's limbs `ref`."""
    import torch
    d = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    ws = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    out = torch.full_like(ref, -1)
    for s in range(6):
        pdm.solve_stages_device(pl, s, s + 1, d if s == 0 else None, out if s == 5 else None, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


@pytest.mark.parametrize("n,deg,amp,seed,force", FOLD_CASES)
def test_folded_reduction_and_reconstruction(n, deg, amp, seed, force):
    # the solve (folded launches) against the oracle and against the same plan stage by stage
    import torch
    arr = W.random_matrix(np.random.default_rng(seed), n, deg, -amp, amp, zero_prob=0.2)
    got, pl, _ = gpu_solve(arr, flags=pdm.FORCE_PN(force) if force else 0)
    if force:
        assert pl.info["pn"] == force
    assert box_to_dict(got) == box_to_dict(oracle_box(arr))
    ref, _ = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    check_against_stages(arr, pl, ref)


# interpolation passes in registers: 32 points over 32 lines (the 4 x 8 form), 128 points over
# 64 (16 x 8, with a first variable of 14 coefficients: the term-by-term evaluation), 64
# points over 512 followed by a 32-point pass over 16 lines (LDS-staged)
REG_CASES = [(6, (4, 3), 51), (5, (13, 8), 52), (4, (9, 4, 2), 53)]


@pytest.mark.parametrize("n,deg,seed", REG_CASES)
def test_register_form_interpolation_lengths(n, deg, seed):
    arr = W.random_matrix(np.random.default_rng(seed), n, deg, -50, 50, zero_prob=0.2)
    got, pl, _ = gpu_solve(arr)
    assert box_to_dict(got) == box_to_dict(oracle_box(arr))


def test_reconstruction_tiles_beyond_lds():
    # 28 primes over a last-variable grid of 256: the folded pass's tiles (28 x 384 words) do
    # not fit its LDS, so the last pass and the reconstruction run as separate launches; the
    # result equals the folded solve with 8 primes (the primes beyond the bound's need change
    # nothing) and the stage-by-stage run
    import torch
    arr = W.random_matrix(np.random.default_rng(44), 5, (1, 31), -10, 10, zero_prob=0.2)
    a, pla, _ = gpu_solve(arr, flags=pdm.FORCE_PN(28))
    b, plb, _ = gpu_solve(arr, flags=pdm.FORCE_PN(8))
    assert pla.info["N"][-1] == 256 and 28 * (256 + 128) * 4 > 40 * 1024 >= 8 * (256 + 128) * 4
    assert box_to_dict(a) == box_to_dict(b)
    ref, _ = pdm.solve_device(pla, torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    check_against_stages(arr, pla, ref)


def _large_order_cases():
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_large_order_digests as LG
    return LG


@pytest.mark.parametrize("idx", range(7))
def test_large_orders_against_oracle_digests(idx):
    # orders 25-32 whose first variable has 5 or 6 coefficients (the paired evaluation with
    # three terms per lane) or 1 or 7 (the term-by-term evaluation), with 8 and 16 lanes per
    # matrix and the default mapping, against the oracle's exact determinant (stored digests
    # written by tests/golden/make_large_order_digests.py from the pointwise oracle)
    import json
    LG = _large_order_cases()
    from make_config4_digests import digest
    n, deg, seed = LG.CASES[idx]
    want = json.load(open(LG.OUT))["digests"][LG.case_key(n, deg, seed)]
    arr = LG.case_matrix(n, deg, seed)
    assert not (2 <= deg[0] + 1 <= 4)  # not the two-term paired form
    for flags in (pdm.DET_LANES_LOG2(3), pdm.DET_LANES_LOG2(4), 0):
        got, pl, _ = gpu_solve(arr, flags=flags | pdm.DET_EXCHANGE)
        assert pl.info["pn"] >= 15
        assert digest(got) == want, (n, deg, pl.info["det_lanes"])


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_repeated_entries_are_evaluated_once(lanes):
    # a block matrix whose entries repeat (and some are zero), solved with one slot per
    # distinct entry, equals the solve that evaluates every entry (the full evaluation tensor)
    # and the oracle
    rng = np.random.default_rng(400 + lanes)
    base = W.random_matrix(rng, 3, (2, 1, 1), -40, 40, zero_prob=0.2)
    arr = np.concatenate([np.concatenate([base, base[::-1]], axis=1),
                          np.concatenate([base[:, ::-1], base], axis=1)], axis=0)
    arr[0, 5] = arr[4, 1]
    log2 = {1: 0, 2: 1, 4: 2}[lanes]
    got, pl, _ = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2))
    ref, plu, _ = gpu_solve(arr, flags=pdm.DET_LANES_LOG2(log2) | pdm.UNFUSED_EVAL)
    assert pl.info["nslots"] < 18 and plu.info["nslots"] == 36
    assert box_to_dict(got) == box_to_dict(ref) == box_to_dict(oracle_box(arr))
