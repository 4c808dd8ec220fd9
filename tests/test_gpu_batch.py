"""Batched solves (polydet_solve_batch): thousands of matrices of uneven order, variable count
and degree in chunked persistent launches. Bit-exact against the plain per-matrix path,
single-matrix solves and the oracle; also across chunk boundaries, for matrices that fall
back to single solves, and on replays of a captured HIP graph."""
import os

import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W
from oracle import det as OD
from oracle import plan as PL

from helpers import Q31, box_to_dict, det_mod_q_stack, device_values_at_point

pytestmark = pytest.mark.gpu


def pack(mats, pl):
    import torch
    coeff_off, out_off = [], []
    c = o = 0
    for a, info in zip(mats, pl.infos):
        coeff_off.append(c)
        out_off.append(o)
        c += a.size
        o += info["ncoeff"] * info["limbs"]
    flat = np.concatenate([np.ascontiguousarray(a, dtype=np.int64).reshape(-1) for a in mats])
    d_coeffs = torch.from_numpy(flat).cuda()
    d_out = torch.zeros(max(o, 1), dtype=torch.int32, device="cuda")
    return d_coeffs, coeff_off, d_out, out_off


def unpack(pl, d_out, out_off):
    host = d_out.cpu().numpy()
    res = []
    for info, off in zip(pl.infos, out_off):
        L = info["limbs"]
        vals = B.limbs_to_ints(host[off:off + info["ncoeff"] * L].reshape(-1, L))
        box = tuple(d + 1 for d in info["D"])
        arr = np.empty(len(vals), dtype=object)
        for i, v in enumerate(vals):
            arr[i] = v
        res.append(arr.reshape(box) if box else arr.reshape(()))
    return res


def solve_batch(mats, flags=0):
    import torch
    pl = pdm.plan_batch(mats, flags=flags)
    d_coeffs, co, d_out, oo = pack(mats, pl)
    pdm.solve_batch_device(pl, d_coeffs, co, d_out, oo)
    torch.cuda.synchronize()
    return unpack(pl, d_out, oo), pl


def solve_single(a):
    import torch
    n, deg = B.shape_of(a)
    pl = pdm.plan(n, deg, host_coeffs=a)
    out, _ = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(a)).cuda())
    torch.cuda.synchronize()
    vals = B.limbs_to_ints(out.cpu().numpy())
    arr = np.empty(len(vals), dtype=object)
    for i, v in enumerate(vals):
        arr[i] = v
    box = tuple(d + 1 for d in pl.info["D"])
    return arr.reshape(box) if box else arr.reshape(())


def oracle_cost(a):
    n, deg = B.shape_of(a)
    return int(np.prod([n * d + 1 for d in deg])) * n ** 3


def mixed_batch(seed=0, count=40):
    rng = np.random.default_rng(500 + seed)
    mats = []
    for _ in range(count):
        n = int(rng.integers(1, 13))
        k = int(rng.integers(1, 4))
        deg = tuple(int(x) for x in rng.integers(0, 3, size=k))
        mats.append(W.random_matrix(rng, n, deg, -50, 50, zero_prob=float(rng.uniform(0, 0.4))))
    # kinds that take the single-matrix path inside a batch
    mats.append(np.array([[3, -7], [2 ** 40, 5]], dtype=np.int64))  # no variables
    mats.append(W.random_matrix(rng, 3, (9, 1), -5, 5))  # 10 coefficients in a later variable
    mats.append(W.random_matrix(rng, 3, (1, 9), -5, 5))
    mats.append(np.zeros((4, 4, 2, 2), dtype=np.int64))  # zero matrix
    # first pivot (x1 - 1 or x1 + 1) vanishes at grid points whatever the row order
    for n in (2, 6, 12):
        v = W.random_matrix(rng, n, (1, 1), -9, 9)
        v[:, 0] = 0
        v[0, 0, 0, 0], v[0, 0, 1, 0] = -1, 1
        v[1, 0, 0, 0], v[1, 0, 1, 0] = 1, 1
        mats.append(v)
    return mats


def test_batch_matches_plain_single_and_oracle():
    mats = mixed_batch()
    got, pl = solve_batch(mats)
    plain, _ = solve_batch(mats, flags=pdm.BATCH_PLAIN)
    for i, a in enumerate(mats):
        assert box_to_dict(got[i]) == box_to_dict(plain[i]), i
        n, deg = B.shape_of(a)
        expect = OD.det_pointwise(a, PL.det_degree_bound_from_shape(n, deg))
        assert box_to_dict(got[i]) == box_to_dict(expect), i


def test_batch_left_looking_and_exchanging_agree():
    mats = mixed_batch(seed=3)
    ll, _ = solve_batch(mats, flags=pdm.DET_LEFT_LOOKING)
    ex, _ = solve_batch(mats, flags=pdm.DET_EXCHANGE)
    for i in range(len(mats)):
        assert box_to_dict(ll[i]) == box_to_dict(ex[i]), i


def test_batch_across_chunks(monkeypatch):
    mats = W.config4(count=24)
    monkeypatch.setenv("POLYDET_BATCH_BUDGET_MB", "8")
    got, _ = solve_batch(mats)
    monkeypatch.delenv("POLYDET_BATCH_BUDGET_MB")
    whole, _ = solve_batch(mats)
    for i, a in enumerate(mats):
        assert box_to_dict(got[i]) == box_to_dict(whole[i]), i
    cheap = sorted(range(len(mats)), key=lambda i: oracle_cost(mats[i]))[:6]
    for i in cheap:
        assert box_to_dict(got[i]) == box_to_dict(solve_single(mats[i])), i
        n, deg = B.shape_of(mats[i])
        expect = OD.det_pointwise(mats[i], PL.det_degree_bound_from_shape(n, deg))
        assert box_to_dict(got[i]) == box_to_dict(expect), i


@pytest.mark.parametrize("streams", [1, 2])
def test_batch_graph_replay(streams, monkeypatch):
    # a captured batched solve replays bit-identically, with eager work between replays; with
    # 2 streams the odd chunks fork from and join back into the captured stream (a budget of
    # 1 MiB makes several chunks of this batch)
    monkeypatch.setenv("POLYDET_BATCH_BUDGET_MB", "1")
    import torch
    mats = mixed_batch(seed=1, count=24)
    monkeypatch.setenv("POLYDET_BATCH_STREAMS", str(streams))
    pl = pdm.plan_batch(mats)
    monkeypatch.delenv("POLYDET_BATCH_STREAMS")
    monkeypatch.delenv("POLYDET_BATCH_BUDGET_MB")
    ref = pdm.plan_batch(mats)
    d_coeffs, co, d_out, oo = pack(mats, pl)
    ws = torch.empty(max(pl.infos[0]["workspace_bytes"], ref.infos[0]["workspace_bytes"]),
                     dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pdm.solve_batch_device(pl, d_coeffs, co, d_out, oo, workspace=ws, stream=stream)
    stream.synchronize()
    eager = d_out.clone()
    with torch.cuda.stream(stream):
        pdm.solve_batch_device(ref, d_coeffs, co, d_out, oo, workspace=ws, stream=stream)
    stream.synchronize()
    assert torch.equal(d_out, eager)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        pdm.solve_batch_device(pl, d_coeffs, co, d_out, oo, workspace=ws, stream=stream)
    for _ in range(3):
        d_out.fill_(-1)
        junk = torch.randn(1 << 20, device="cuda") * 2
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(d_out, eager)
        del junk


def test_det_mod_q_stack_matches_oracle_steps():
    from oracle import modular as OM
    rng = np.random.default_rng(1)
    for n in [1, 2, 5, 9]:
        A = rng.integers(0, Q31, size=(20, n, n)).astype(np.uint64)
        A[rng.random((20, n, n)) < 0.4] = 0
        got = det_mod_q_stack(A, Q31)
        for t in range(20):
            assert int(got[t]) == OM.det_mod(A[t].astype(object).tolist(), Q31)


@pytest.fixture(scope="module")
def config4_solved():
    """The 4096-matrix workload solved once in one batched call."""
    import torch
    mats = W.config4()
    pl = pdm.plan_batch(mats)
    d_coeffs, co, d_out, oo = pack(mats, pl)
    pdm.solve_batch_device(pl, d_coeffs, co, d_out, oo)
    torch.cuda.synchronize()
    return mats, pl, d_out, oo


def test_config4_all_matrices_identity_and_cheap_oracle(config4_solved):
    """Every one of the 4096 matrices: the batched result, reduced mod an independent prime
    q and evaluated at a seeded random point, equals det M(point) mod q (a false pass has
    probability at most deg/q per matrix, Schwartz-Zippel). The cheapest matrices are also
    compared with the oracle exactly."""
    mats, pl, d_out, oo = config4_solved
    rng = np.random.default_rng(4242)
    q = Q31
    lhs, points = [], []
    for a, info, off in zip(mats, pl.infos, oo):
        n, deg = B.shape_of(a)
        point = [int(x) for x in rng.integers(1, q, size=len(deg))]
        points.append(point)
        box = tuple(d + 1 for d in info["D"])
        lhs.append(device_values_at_point(d_out, off, info["ncoeff"], info["limbs"], box, point, q))
    # det M(point) mod q, grouped by order
    by_n = {}
    for t, a in enumerate(mats):
        by_n.setdefault(a.shape[0], []).append(t)
    for n, ts in by_n.items():
        stack = np.zeros((len(ts), n, n), dtype=np.uint64)
        for s_, t in enumerate(ts):
            a = mats[t]
            k = a.ndim - 2
            vals = (a % q).astype(np.uint64)
            for v in range(k - 1, -1, -1):
                pw = np.array([pow(points[t][v], e, q) for e in range(a.shape[2 + v])],
                              dtype=np.uint64)
                vals = np.sum((vals * pw) % q, axis=-1, dtype=np.uint64) % q
            stack[s_] = vals
        dets = det_mod_q_stack(stack, q)
        for s_, t in enumerate(ts):
            assert lhs[t] == int(dets[s_]), t
    cheap = sorted(range(len(mats)), key=lambda i: oracle_cost(mats[i]))[:12]
    for i in cheap:
        info, off = pl.infos[i], oo[i]
        L = info["limbs"]
        vals = B.limbs_to_ints(d_out[off:off + info["ncoeff"] * L].cpu().numpy().reshape(-1, L))
        n, deg = B.shape_of(mats[i])
        expect = OD.det_pointwise(mats[i], PL.det_degree_bound_from_shape(n, deg)).reshape(-1)
        assert vals == [int(x) for x in expect], i


def test_config4_exact_integer_points_on_a_sample(config4_solved):
    """A seeded sample of 48 of the 4096 matrices: at a random integer point a with
    coordinates in [-2^20, 2^20], the batched result evaluated exactly (Python integers)
    equals det M(a) from the oracle's integer Bareiss. A probabilistic identity check
    (Schwartz-Zippel: a false pass has probability at most sum_v D_v / 2^21 per matrix), not
    parity with the oracle's polynomial."""
    mats, pl, d_out, oo = config4_solved
    rng = np.random.default_rng(777)
    small = [i for i, info in enumerate(pl.infos) if info["ncoeff"] <= 50000]
    sample = sorted(int(i) for i in rng.choice(small, size=48, replace=False))
    host = d_out.cpu().numpy()
    for i in sample:
        a, info, off = mats[i], pl.infos[i], oo[i]
        n, deg = B.shape_of(a)
        point = [int(x) for x in rng.integers(-(1 << 20), (1 << 20) + 1, size=len(deg))]
        L = info["limbs"]
        vals = B.limbs_to_ints(host[off:off + info["ncoeff"] * L].reshape(-1, L))
        box = np.empty(len(vals), dtype=object)
        box[:] = vals
        box = box.reshape(tuple(d + 1 for d in info["D"]))
        for v in range(len(deg) - 1, -1, -1):  # Horner along the last axis
            acc = np.zeros(box.shape[:-1], dtype=object)
            for e in range(box.shape[-1] - 1, -1, -1):
                acc = acc * point[v] + box[..., e]
            box = acc
        got = int(box[()]) if isinstance(box, np.ndarray) else int(box)
        M = []
        for r in range(n):
            row = []
            for c in range(n):
                ent = a[r, c].astype(object)
                for v in range(len(deg) - 1, -1, -1):
                    acc = np.zeros(ent.shape[:-1], dtype=object)
                    for e in range(ent.shape[-1] - 1, -1, -1):
                        acc = acc * point[v] + ent[..., e]
                    ent = acc
                row.append(int(ent[()]) if isinstance(ent, np.ndarray) else int(ent))
            M.append(row)
        assert got == OD.det_bareiss_int(M), i


def test_config4_bit_exact_against_stored_oracle_digests(config4_solved):
    """The cheapest three quarters of the 4096 matrices (by the pointwise oracle's cost): the
    batched result equals the oracle's determinant exactly, compared through the digests that
    tests/golden/make_config4_digests.py wrote from the oracle (canonical text of the nonzero
    coefficients, SHA-256)."""
    import json
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from make_config4_digests import OUT, digest
    stored = json.load(open(OUT))["digests"]
    assert len(stored) >= 3000
    mats, pl, d_out, oo = config4_solved
    host = d_out.cpu().numpy()
    bad = []
    for key, want in stored.items():
        i = int(key)
        info, off = pl.infos[i], oo[i]
        L = info["limbs"]
        vals = B.limbs_to_ints(host[off:off + info["ncoeff"] * L].reshape(-1, L))
        arr = np.empty(len(vals), dtype=object)
        arr[:] = vals
        box = tuple(d + 1 for d in info["D"])
        if digest(arr.reshape(box) if box else arr.reshape(())) != want:
            bad.append(i)
    assert not bad, f"{len(bad)} matrices differ from the oracle, first {bad[:10]}"
