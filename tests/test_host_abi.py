"""CPU checks of the C-ABI library: it loads, exports every declared entry point, and its
host-side plan (degree bound, grid, prime choice, limbs, errors) agrees with the oracle's
plan quantities. No GPU work is launched here."""
import ctypes

import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W
from oracle import plan as PL

from helpers import declared_functions


def test_library_exports_every_declared_symbol():
    lib = pdm.load_library()
    names = declared_functions()
    assert "polydet_solve_batch" in names and "polydet_plan" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings_and_limits():
    lib = pdm.load_library()
    for st in range(6):
        assert lib.polydet_status_string(st)
    lim = pdm.limits()
    assert lim["max_n"] >= 32 and lim["max_vars"] == 8 and lim["max_primes"] >= 27


def _oracle_pn(arr):
    return PL.num_primes(PL.hadamard_bound_sq(arr))


@pytest.mark.parametrize("which", ["c1", "c2", "c3a", "c3b", "k0", "n1"])
def test_host_plan_matches_oracle_plan(which):
    if which == "c1":
        arr = W.config1()
    elif which == "c2":
        arr = W.config2()
    elif which == "c3a":
        arr = W.config3a()
    elif which == "c3b":
        arr = W.config3b()[0]
    elif which == "k0":
        arr = np.array([[2 ** 62, -(2 ** 62)], [3, 2 ** 61]], dtype=np.int64)
    else:
        arr = np.arange(1, 10, dtype=np.int64).reshape(1, 1, 9)
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY)
    info = pl.info
    D = PL.det_degree_bound_from_shape(n, deg)
    assert list(info["D"]) == D
    assert list(info["N"]) == PL.grid_sizes(D)
    assert info["G"] == int(np.prod(PL.grid_sizes(D))) if D else info["G"] == 1
    pn0 = _oracle_pn(arr)
    # the library's bound carries a margin of at most one extra prime
    assert pn0 <= info["pn"] <= pn0 + 1
    assert info["primes"] == PL.ntt_primes(info["pn"])
    M = 1
    for p in info["primes"]:
        M *= p
    assert info["limbs"] == PL.limbs_for(M)


def test_workload_plan_sizes():
    # sizes of the paper-shaped workloads (grid, primes)
    c2 = pdm.plan(12, (3, 3, 3), host_coeffs=W.config2(), flags=pdm.HOST_ONLY).info
    assert c2["N"] == (64, 64, 64) and c2["pn"] == 7 and c2["ncoeff"] == 37 ** 3
    c3 = pdm.plan(22, (4, 4), host_coeffs=W.config3a(), flags=pdm.HOST_ONLY).info
    assert c3["N"] == (128, 128) and c3["pn"] == 15
    c1 = pdm.plan(4, (2, 2), host_coeffs=W.config1(), flags=pdm.HOST_ONLY).info
    assert c1["N"] == (16, 16) and c1["pn"] == 1


def test_worst_case_bound_dominates_data_bound():
    rng = np.random.default_rng(3)
    for _ in range(10):
        n = int(rng.integers(1, 20))
        k = int(rng.integers(0, 4))
        deg = tuple(int(x) for x in rng.integers(0, 4, size=k))
        arr = W.random_matrix(rng, n, deg, -1000, 1000)
        a = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY).info
        b = pdm.plan(n, deg, coeff_bits=10, flags=pdm.HOST_ONLY).info
        assert b["pn"] >= a["pn"]
        assert a["D"] == b["D"] and a["G"] == b["G"]


def test_forced_prime_count_and_offset():
    arr = W.config1()
    base = pdm.plan(4, (2, 2), host_coeffs=arr, flags=pdm.HOST_ONLY).info
    forced = pdm.plan(4, (2, 2), host_coeffs=arr, flags=pdm.HOST_ONLY | pdm.FORCE_PN(5)).info
    assert forced["pn"] == 5 and forced["primes"] == PL.ntt_primes(5)
    off = pdm.plan(4, (2, 2), host_coeffs=arr,
                   flags=pdm.HOST_ONLY | pdm.PRIME_OFFSET(3)).info
    assert off["primes"] == PL.ntt_primes(3 + off["pn"])[3:]
    big = W.config2()
    with pytest.raises(pdm.PolydetError) as e:
        pdm.plan(12, (3, 3, 3), host_coeffs=big, flags=pdm.HOST_ONLY | pdm.FORCE_PN(2))
    assert e.value.status == B.EINVAL


@pytest.mark.parametrize("n,deg,status", [
    (0, (1,), B.EINVAL), (-3, (), B.EINVAL), (3, (1,) * 9, B.EINVAL), (3, (-1, 2), B.EINVAL),
    (33, (1,), B.EUNSUPPORTED), (3, (32,), B.EUNSUPPORTED)])
def test_plan_errors(n, deg, status):
    lib = pdm.load_library()
    s = B.Shape()
    s.n = n
    s.nvars = len(deg)
    for v, d in enumerate(deg[:8]):
        s.deg[v] = d
    s.coeff_bits = 10
    h = ctypes.c_void_p()
    st = lib.polydet_plan(ctypes.byref(s), None, pdm.HOST_ONLY, ctypes.byref(h))
    assert st == status
    assert not h.value
    assert lib.polydet_last_error()


def test_bad_coeff_bits_and_null_arguments():
    lib = pdm.load_library()
    s = B.make_shape(3, (1,), 64)
    h = ctypes.c_void_p()
    assert lib.polydet_plan(ctypes.byref(s), None, pdm.HOST_ONLY, ctypes.byref(h)) == B.EINVAL
    assert lib.polydet_plan(None, None, pdm.HOST_ONLY, ctypes.byref(h)) == B.EINVAL
    assert lib.polydet_plan_query(None, 0, None) == B.EINVAL
    assert lib.polydet_plan_batch(None, 0, None, pdm.HOST_ONLY, ctypes.byref(h)) == B.EINVAL


def test_host_only_plan_cannot_be_solved():
    lib = pdm.load_library()
    pl = pdm.plan(4, (2, 2), coeff_bits=4, flags=pdm.HOST_ONLY)
    dummy = ctypes.c_void_p(256)
    st = lib.polydet_solve(pl.handle, dummy, dummy, dummy, pl.info["workspace_bytes"], None)
    assert st == B.EINVAL
    small = lib.polydet_solve(pl.handle, dummy, dummy, dummy, 16, None)
    assert small == B.EINVAL


def test_batch_plan_host_only():
    mats = W.config4(count=16)
    pl = pdm.plan_batch(mats, flags=pdm.HOST_ONLY)
    assert pl.count == 16
    for a, info in zip(mats, pl.infos):
        n, deg = B.shape_of(a)
        assert info["n"] == n and tuple(info["deg"]) == deg
        pn0 = _oracle_pn(a)
        assert pn0 <= info["pn"] <= pn0 + 1


def test_limb_decoding():
    vals = [0, 1, -1, 2 ** 31, -(2 ** 31), 2 ** 95 - 1, -(2 ** 95)]
    L = 3
    rows = []
    for v in vals:
        u = v % (1 << (32 * L))
        rows.append([(u >> (32 * l)) & 0xFFFFFFFF for l in range(L)])
    arr = np.array(rows, dtype=np.uint32)
    assert B.limbs_to_ints(arr) == vals


def test_structural_row_order():
    # the plan reorders rows so that symbolic elimination of the zero pattern meets no
    # structurally zero pivot; det_sign is the permutation's sign
    for arr in [W.config2(), W.config3a(), W.config3b()[0]] + W.config4(count=8):
        n, deg = B.shape_of(arr)
        info = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY).info
        order = list(info["row_order"])
        assert sorted(order) == list(range(n))
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if order[i] > order[j])
        assert info["det_sign"] == (-1) ** inv
        S = (np.abs(arr).reshape(n * n, -1).sum(axis=1) != 0).reshape(n, n)[order]
        S = S.copy()
        for k in range(n - 1):
            if S[k:, k].any():
                assert S[k, k]
            for i in range(k + 1, n):
                if S[i, k]:
                    S[i, k + 1:] |= S[k, k + 1:]
    # without coefficients the order is the identity
    info = pdm.plan(5, (1,), coeff_bits=3, flags=pdm.HOST_ONLY).info
    assert info["row_order"] == tuple(range(5)) and info["det_sign"] == 1


@pytest.fixture
def builtin_tuning():
    """The library's built-in launch mapping for the test, the installed table after it."""
    saved = pdm.get_tuning()
    pdm.set_tuning(None)
    yield
    pdm.set_tuning(saved)


def test_elimination_form_choice(builtin_tuning):
    # the exchanging kernel alone by default; a left-looking pass on request for orders up
    # to 16 when the first variable is evaluated inside the elimination kernel
    H = pdm.HOST_ONLY
    LL = pdm.DET_LEFT_LOOKING
    for n in (1, 5, 12, 13, 16):
        assert pdm.plan(n, (3, 3), coeff_bits=8, flags=H).info["det_left_looking"] == 0
        assert pdm.plan(n, (3, 3), coeff_bits=8, flags=H | LL).info["det_left_looking"] == 1
        assert pdm.plan(n, (3, 3), coeff_bits=8,
                        flags=H | LL | pdm.DET_EXCHANGE).info["det_left_looking"] == 0
        assert pdm.plan(n, (3, 3), coeff_bits=8,
                        flags=H | LL | pdm.UNFUSED_EVAL).info["det_left_looking"] == 0
    assert pdm.plan(17, (1,), coeff_bits=8, flags=H | LL).info["det_left_looking"] == 0
    assert pdm.plan(4, (), coeff_bits=8, flags=H | LL).info["det_left_looking"] == 0


def test_serving_jobs_compare_by_identity():
    # the server removes finished jobs from its running list; jobs hold arrays of any shape,
    # so equality must be identity
    from paper_2010_12117_amd import serving as S
    jobs = [S._Job(np.zeros((n, n, 2)), None, 0, None, 0.0) for n in (3, 4, 4)]
    running = list(jobs)
    running.remove(jobs[2])
    running.remove(jobs[0])
    assert running == [jobs[1]]


def test_tuning_table_round_trip_and_effect(builtin_tuning):
    H = pdm.HOST_ONLY
    table = {"lanes": {"paired": {"12": 2, "20": 8}, "other": {"12": 4}},
             "left_looking": {"paired": {"9": 1}, "other": {"12": 2}},
             "tile_points": {"paired": {"12": 4}, "other": {}}}
    pdm.set_tuning(table)
    got = pdm.get_tuning()
    assert got["lanes"] == {"paired": {12: 2, 20: 8}, "other": {12: 4}}
    assert got["left_looking"] == {"paired": {9: 1}, "other": {12: 2}}
    assert got["tile_points"] == {"paired": {12: 4}, "other": {}}
    # class "paired": 2..4 coefficients in the first variable; "other": everything else
    assert pdm.plan(12, (3, 2), coeff_bits=8, flags=H).info["det_lanes"] == 2
    assert pdm.plan(12, (4, 2), coeff_bits=8, flags=H).info["det_lanes"] == 4
    assert pdm.plan(12, (0, 2), coeff_bits=8, flags=H).info["det_lanes"] == 4
    assert pdm.plan(20, (1, 1), coeff_bits=8, flags=H).info["det_lanes"] == 8
    assert pdm.plan(11, (1, 1), coeff_bits=8, flags=H).info["det_lanes"] == 1  # no entry
    assert pdm.plan(9, (2,), coeff_bits=8, flags=H).info["det_left_looking"] == 1
    assert pdm.plan(9, (5,), coeff_bits=8, flags=H).info["det_left_looking"] == 0
    # flags override the table
    pl = pdm.plan(12, (3, 2), coeff_bits=8, flags=H | pdm.DET_LANES_LOG2(0))
    assert pl.info["det_lanes"] == 1
    assert pdm.plan(9, (2,), coeff_bits=8,
                    flags=H | pdm.DET_EXCHANGE).info["det_left_looking"] == 0
    pdm.set_tuning(None)
    assert pdm.get_tuning()["lanes"] == {"paired": {}, "other": {}}
    assert pdm.plan(12, (3, 2), coeff_bits=8, flags=H).info["det_lanes"] == 1


@pytest.mark.parametrize("bad", [
    {"lanes": {"paired": {"13": 1}}},          # one lane per matrix only up to n = 12
    {"lanes": {"other": {"4": 16}}},            # 16 lanes only from n = 16
    {"lanes": {"paired": {"8": 3}}},
    {"left_looking": {"paired": {"17": 1}}},    # left-looking only up to n = 16
    {"left_looking": {"other": {"5": 3}}},
    {"tile_points": {"paired": {"5": 3}}},
    {"tile_points": {"paired": {"5": 32}}},
    {"lanes": {"paired": {"0": 1}}},
])
def test_tuning_table_rejects_bad_entries(builtin_tuning, bad):
    before = pdm.get_tuning()
    with pytest.raises(pdm.PolydetError) as e:
        pdm.set_tuning(bad)
    assert e.value.status == B.EINVAL
    assert pdm.get_tuning() == before  # no change


def test_capped_plan_cuts_one_prime_into_grid_slabs():
    # below one prime's footprint the plan cuts each prime's grid into slabs along the second
    # variable: the least power of two that fits, at most half that variable's grid, and
    # never below what the determinants and the coefficient residues need whole
    H = pdm.HOST_ONLY
    arr = W.config2()
    one = None
    for cap in range(40 << 20, 4 << 20, -(1 << 19)):
        try:
            info = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H, max_workspace=cap).info
        except pdm.PolydetError as e:
            assert e.status == B.EUNSUPPORTED
            floor = cap
            break
        assert info["workspace_bytes"] <= cap
        if info["grid_slabs"] == 1:
            one = info["workspace_bytes"]  # the smallest footprint without slabs
            continue
        assert info["prime_group"] == 1 and info["workspace_bytes"] < one
        sl = info["grid_slabs"]
        assert sl & (sl - 1) == 0 and 2 <= sl <= info["N"][1] // 2
        assert info["det_left_looking"] == 0
        last = info
    assert one is not None and last["grid_slabs"] >= 8
    # the whole grid's determinants (numerators and denominators) and every prime's
    # coefficient residues stay in the workspace
    assert floor >= 2 * 4 * last["G"] + last["coef_bytes"]
    # slabs need a second variable
    one_var = W.random_matrix(np.random.default_rng(3), 6, (7,), -9, 9)
    info = pdm.plan(6, (7,), host_coeffs=one_var, flags=H).info
    with pytest.raises(pdm.PolydetError) as e:
        pdm.plan(6, (7,), host_coeffs=one_var, flags=H,
                 max_workspace=info["workspace_bytes"] // 2)
    assert e.value.status == B.EUNSUPPORTED
    # stage timing needs the whole grid at once
    with pytest.raises(pdm.PolydetError) as e:
        pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H | pdm.STAGE_TIMING,
                 max_workspace=last["workspace_bytes"])
    assert e.value.status == B.EINVAL


def test_capped_workspace_groups_primes():
    H = pdm.HOST_ONLY
    arr = W.config2()
    full = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H).info
    assert full["prime_group"] == full["pn"] == 7
    assert full["coef_bytes"] == 4 * full["pn"] * full["ncoeff"]
    seen = set()
    for frac in (0.9, 0.6, 0.4, 0.25):
        cap = int(full["workspace_bytes"] * frac)
        info = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H, max_workspace=cap).info
        assert info["workspace_bytes"] <= cap
        assert 1 <= info["prime_group"] < info["pn"]
        # the largest group that fits: one more prime would not
        seen.add(info["prime_group"])
        assert info["pn"] == full["pn"] and info["coef_bytes"] == full["coef_bytes"]
    assert len(seen) >= 3
    # no cap needed: the plan is the uncapped one
    info = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H,
                    max_workspace=full["workspace_bytes"]).info
    assert info["prime_group"] == 7 and info["workspace_bytes"] == full["workspace_bytes"]
    # below one prime's footprint
    with pytest.raises(pdm.PolydetError) as e:
        pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H, max_workspace=1 << 20)
    assert e.value.status == B.EUNSUPPORTED
    # stage timing needs all primes at once
    with pytest.raises(pdm.PolydetError) as e:
        pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=H | pdm.STAGE_TIMING,
                 max_workspace=full["workspace_bytes"] // 2)
    assert e.value.status == B.EINVAL
    # integer matrices are never split
    a = np.array([[3, 1], [2, 2 ** 40]], dtype=np.int64)
    info = pdm.plan(2, (), host_coeffs=a, flags=H).info
    with pytest.raises(pdm.PolydetError):
        pdm.plan(2, (), host_coeffs=a, flags=H, max_workspace=info["workspace_bytes"] - 256)


def test_prime_range_and_reconstruct_reject_bad_arguments():
    lib = pdm.load_library()
    pl = pdm.plan(4, (2, 2), coeff_bits=4, flags=pdm.HOST_ONLY)
    dummy = ctypes.c_void_p(256)
    ws = pl.info["workspace_bytes"]
    # a host-only plan, a bad range, a batch plan
    assert lib.polydet_solve_primes(pl.handle, dummy, 0, 1, dummy, ws, None) == B.EINVAL
    assert lib.polydet_reconstruct(pl.handle, dummy, ws, dummy, None) == B.EINVAL
    assert lib.polydet_solve_primes(None, dummy, 0, 1, dummy, ws, None) == B.EINVAL
    bp = pdm.plan_batch(W.config4(count=4), flags=pdm.HOST_ONLY)
    assert lib.polydet_solve_primes(bp.handle, dummy, 0, 1, dummy, 1 << 40, None) == B.EINVAL


def test_bench_algorithmic_figures():
    """bench.py's per-unit figures: elimination updates per determinant (sum of m^2 for
    m < n, 506 at n = 12, checked by counting the (n-k-1)^2 updates of each step) and the
    bytes of the evaluation passes at the 12x12 trivariate workload (7 primes, 101 nonzero
    entries): residues 4^3, pass over x3 writes 4^2 x 64 and the next reads it, the
    pre-tensor 4 x 64^2, 4 bytes each."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench_under_test", os.path.join(os.path.dirname(os.path.dirname(__file__)), "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for n in range(1, 33):
        assert bench.det_updates(n) == sum((n - k - 1) ** 2 for k in range(n))
    assert bench.det_updates(12) == 506
    assert bench.expand_bytes(7, 101, [4, 4, 4], [64, 64, 64]) == 4 * 7 * 101 * (64 + 2 * 1024 + 16384)
    assert bench.expand_bytes(3, 5, [2], [8]) == 0  # one variable: evaluated inside the elimination
    # issue cost of the two-column elimination (CU-clocks per lane): (m-2)^2 updates of
    # 5 multiply-class + 1 plain op and m-2 column-factor pairs of 8 + 7, then a 2x2 for even n
    upd, col, two = 5 / 64 + 1 / 128, 8 / 64 + 7 / 128, 4 / 64 + 2 / 128
    assert bench.det_issue_clk(1) == 0
    assert bench.det_issue_clk(2) == pytest.approx(two)
    assert bench.det_issue_clk(3) == pytest.approx(upd + col)
    assert bench.det_issue_clk(4) == pytest.approx(4 * upd + 2 * col + two)
    assert bench.det_issue_clk(5) == pytest.approx(9 * upd + 3 * col + upd + col)
    # first-variable evaluation per entry and point: paired (2..6 coefficients) one reduction
    # of two or three products and an addition; otherwise ceil(m0/2) two-product reductions
    # and the additions between them
    assert bench.eval_issue_clk(1) == 0
    assert bench.eval_issue_clk(4) == pytest.approx(two + 1 / 128)
    assert bench.eval_issue_clk(6) == pytest.approx(two + 1 / 64 + 1 / 128)
    assert bench.eval_issue_clk(8) == pytest.approx(4 * two + 3 * 3 / 128)
    # the peak of a launch counts both; elimination alone is faster
    mix = [(12, 1000, 101, 4)]
    assert bench.alu_peak_updates(mix) < bench.alu_peak_updates_elimination_only(mix)
    assert bench.alu_peak_updates_elimination_only(mix) == pytest.approx(
        506 / bench.det_issue_clk(12) * 256 * 2.4e9)


def test_plan_with_coefficients_is_specialised_to_their_zero_pattern():
    # the header's contract: a plan built from host coefficients skips their zero entries and
    # reorders rows around structurally zero pivots; without coefficients it does neither and
    # holds for every matrix of the shape within coeff_bits
    rng = np.random.default_rng(12)
    arr = W.random_matrix(rng, 5, (1, 1), -9, 9)
    arr[0, 0] = 0
    arr[1, 0] = 0
    spec = pdm.plan(5, (1, 1), host_coeffs=arr, flags=pdm.HOST_ONLY).info
    generic = pdm.plan(5, (1, 1), coeff_bits=4, flags=pdm.HOST_ONLY).info
    assert spec["row_order"][0] == 2 and spec["det_sign"] == -1
    assert generic["row_order"] == tuple(range(5)) and generic["det_sign"] == 1
    assert generic["pn"] >= spec["pn"]
    # the row order depends on the zero pattern, not on the values
    other = arr * 3
    assert pdm.plan(5, (1, 1), host_coeffs=other, flags=pdm.HOST_ONLY).info["row_order"] == \
        spec["row_order"]


def test_solve_stages_argument_errors():
    lib = pdm.load_library()
    arr = W.config1()
    host = pdm.plan(4, (2, 2), host_coeffs=arr, flags=pdm.HOST_ONLY)
    dummy = ctypes.c_void_p(256)
    for b, e in ((0, 0), (3, 2), (-1, 2), (0, 7)):
        assert lib.polydet_solve_stages(host.handle, b, e, dummy, dummy, dummy, 1 << 30,
                                        None) == B.EINVAL
    # a host-only plan cannot run even a valid range
    assert lib.polydet_solve_stages(host.handle, 0, 6, dummy, dummy, dummy, 1 << 30,
                                    None) == B.EINVAL
    batch = pdm.plan_batch([arr], flags=pdm.HOST_ONLY)
    assert lib.polydet_solve_stages(batch.handle, 0, 6, dummy, dummy, dummy, 1 << 30,
                                    None) == B.EINVAL


def _distinct_nonzero_entries(arr):
    n = arr.shape[0]
    boxes = {arr[i, j].tobytes() for i in range(n) for j in range(n) if np.any(arr[i, j])}
    return len(boxes)


@pytest.mark.parametrize("which", ["c2", "c3a", "c3b", "dup", "zero"])
def test_plan_evaluates_each_distinct_entry_once(which):
    # with the coefficients, entries with equal coefficient boxes are reduced and evaluated
    # once (a Sylvester matrix repeats each coefficient of f and g along a diagonal)
    if which == "c2":
        arr = W.config2()
    elif which == "c3a":
        arr = W.config3a()
    elif which == "c3b":
        arr = W.config3b()[0]
    elif which == "dup":
        rng = np.random.default_rng(5)
        base = W.random_matrix(rng, 3, (2, 1), -9, 9)
        arr = np.tile(base, (3, 3, 1, 1))  # 9 x 9 with each entry repeated 9 times
    else:
        arr = np.zeros((4, 4, 2, 3), dtype=np.int64)
    n, deg = B.shape_of(arr)
    info = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY).info
    assert info["nslots"] == _distinct_nonzero_entries(arr)
    if which == "c3a":
        assert info["nslots"] == 24 and _distinct_nonzero_entries(arr) == 24
    # without the coefficients, or with the full evaluation tensor, every entry is evaluated
    assert pdm.plan(n, deg, coeff_bits=16, flags=pdm.HOST_ONLY).info["nslots"] == n * n
    assert pdm.plan(n, deg, host_coeffs=arr,
                    flags=pdm.HOST_ONLY | pdm.UNFUSED_EVAL).info["nslots"] == n * n


def test_running_time_prediction_follows_its_rates():
    # the prediction is the sum of per-stage terms over the installed rates (polydet_rates):
    # doubling the elimination rate halves the elimination term, a larger grid predicts more
    saved = pdm.get_rates()
    try:
        pdm.set_rates(None)
        base = pdm.get_rates()
        arr = W.config2()
        p0 = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=pdm.HOST_ONLY).info
        assert p0["predicted_ms"] > 0
        det_term = p0["pn"] * p0["G"] * 506 / base["det_updates_per_s"]["paired"][12] * 1e3
        doubled = {"det_updates_per_s": {"paired": {12: 2 * base["det_updates_per_s"]["paired"][12]}}}
        pdm.set_rates(doubled)
        p1 = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=pdm.HOST_ONLY).info
        assert abs((p0["predicted_ms"] - p1["predicted_ms"]) - det_term / 2) < 1e-9 * det_term
        # built-in values stay where the table has zeros
        assert pdm.get_rates()["launch_us"] == base["launch_us"]
        small = pdm.plan(12, (1, 1, 1), host_coeffs=arr[..., :2, :2, :2], flags=pdm.HOST_ONLY).info
        assert small["predicted_ms"] < p1["predicted_ms"]
        with pytest.raises(pdm.PolydetError):
            pdm.set_rates({"launch_us": -1.0})
    finally:
        pdm.set_rates(None)
        pdm.set_rates({k: v for k, v in saved.items()})
