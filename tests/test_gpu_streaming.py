"""Prime groups, prime ranges and checkpoint/resume (polydet_plan_capped, polydet_solve_primes,
polydet_reconstruct): every way of splitting the primes gives the coefficients of the one-shot
solve, bit for bit, and the coefficient region alone carries a solve across workspaces."""
import random

import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W
from oracle import det as OD
from oracle import plan as PL

from helpers import box_to_dict

pytestmark = pytest.mark.gpu


def one_shot(arr):
    import torch
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr)
    out, _ = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), pl


@pytest.mark.parametrize("frac", [0.8, 0.5, 0.3, 0.2])
def test_capped_plan_matches_one_shot(frac):
    import torch
    arr = W.config2()
    want, full = one_shot(arr)
    cap = int(full.info["workspace_bytes"] * frac)
    pl = pdm.plan(12, (3, 3, 3), host_coeffs=arr, max_workspace=cap)
    assert pl.info["prime_group"] < pl.info["pn"] and pl.info["workspace_bytes"] <= cap
    out, ws = pdm.solve_device(pl, torch.from_numpy(arr).cuda())
    torch.cuda.synchronize()
    assert ws.numel() <= cap
    assert np.array_equal(out.cpu().numpy(), want)


def test_capped_small_case_against_oracle():
    import torch
    rng = np.random.default_rng(61)
    arr = W.random_matrix(rng, 5, (2, 1, 2), -10 ** 6, 10 ** 6, zero_prob=0.2)
    n, deg = B.shape_of(arr)
    full = pdm.plan(n, deg, host_coeffs=arr).info
    assert full["pn"] >= 3
    pl = pdm.plan(n, deg, host_coeffs=arr, max_workspace=full["workspace_bytes"] // 2)
    assert pl.info["prime_group"] < full["pn"]
    out, _ = pdm.solve_device(pl, torch.from_numpy(arr).cuda())
    torch.cuda.synchronize()
    vals = B.limbs_to_ints(out.cpu().numpy())
    got = np.empty(len(vals), dtype=object)
    got[:] = vals
    got = got.reshape(tuple(d + 1 for d in pl.info["D"]))
    expect = OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, deg))
    assert box_to_dict(got) == box_to_dict(expect)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prime_ranges_in_any_split_and_order(seed):
    import torch
    arr = W.config2()
    want, pl = one_shot(arr)
    pn = pl.info["pn"]
    rng = random.Random(seed)
    cuts = sorted(rng.sample(range(1, pn), rng.randint(1, pn - 1)))
    ranges = list(zip([0] + cuts, cuts + [pn]))
    rng.shuffle(ranges)
    d = torch.from_numpy(arr).cuda()
    ws = torch.full((pl.info["workspace_bytes"],), 0xAB, dtype=torch.uint8, device="cuda")
    for b, e in ranges:
        pdm.solve_primes_device(pl, d, b, e, ws)
    out = pdm.reconstruct_device(pl, ws)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)


def test_checkpoint_and_resume_in_another_workspace():
    import torch
    arr = W.config2()
    want, pl = one_shot(arr)
    pn = pl.info["pn"]
    d = torch.from_numpy(arr).cuda()
    ws1 = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    pdm.solve_primes_device(pl, d, 0, 3, ws1)
    torch.cuda.synchronize()
    saved = pdm.coefficient_region(pl, ws1).cpu()  # the checkpoint: host copy of the state
    del ws1
    # a capped plan of the same matrix resumes it: its coefficient region has the same layout
    pl2 = pdm.plan(12, (3, 3, 3), host_coeffs=arr,
                   max_workspace=pl.info["workspace_bytes"] // 2)
    assert pl2.info["coef_bytes"] == pl.info["coef_bytes"]
    ws2 = torch.full((pl2.info["workspace_bytes"],), 0x5C, dtype=torch.uint8, device="cuda")
    pdm.coefficient_region(pl2, ws2).copy_(saved.cuda())
    pdm.solve_primes_device(pl2, d, 3, pn, ws2)
    out = pdm.reconstruct_device(pl2, ws2)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)


def test_integer_matrix_by_primes():
    import torch
    rng = np.random.default_rng(5)
    a = rng.integers(-2 ** 40, 2 ** 40, size=(9, 9), dtype=np.int64)
    want, pl = one_shot(a)
    pn = pl.info["pn"]
    assert pn >= 3
    d = torch.from_numpy(a).cuda()
    ws = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    for i in reversed(range(pn)):
        pdm.solve_primes_device(pl, d, i, i + 1, ws)
    out = pdm.reconstruct_device(pl, ws)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    assert int(B.limbs_to_ints(out.cpu().numpy())[0]) == OD.det_bareiss_int(a.tolist())


def capped_solve(arr, cap):
    import torch
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr, max_workspace=cap)
    out, ws = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    torch.cuda.synchronize()
    assert ws.numel() <= cap
    return out.cpu().numpy(), pl


@pytest.mark.parametrize("cap_mb", [9, 7, 6, 5.5])
def test_grid_slabs_match_one_shot(cap_mb):
    # a cap below one prime's footprint (11.8 MB): each prime's grid runs in 2 .. 16 slabs
    # along the second variable, bit-identical to the one-shot solve
    arr = W.config2()
    want, _ = one_shot(arr)
    got, pl = capped_solve(arr, int(cap_mb * (1 << 20)))
    print(f"cap {cap_mb} MB: {pl.info['grid_slabs']} slabs", flush=True)
    assert pl.info["prime_group"] == 1 and pl.info["grid_slabs"] >= 2
    assert np.array_equal(got, want)


@pytest.mark.parametrize("deg", [(5, 3), (2, 4, 1, 2), (3, 5, 2)])
def test_grid_slabs_other_shapes_against_oracle(deg):
    # two variables (the sliced pass reads the residues), four variables (two passes before
    # it), and a first variable of 6 coefficients (three terms per lane); half the smallest one-prime
    # footprint forces the most slabs that fit
    import torch
    rng = np.random.default_rng(90 + len(deg))
    arr = W.random_matrix(rng, 4, deg, -50, 50, zero_prob=0.2)
    n, _ = B.shape_of(arr)
    want, full = one_shot(arr)
    cap, info = full.info["workspace_bytes"], None
    while True:
        try:
            info = pdm.plan(n, deg, host_coeffs=arr, flags=pdm.HOST_ONLY,
                            max_workspace=cap).info
        except pdm.PolydetError:
            break
        if info["grid_slabs"] >= 4:
            break
        cap = int(cap * 0.8)
    got, pl = capped_solve(arr, max(cap, info["workspace_bytes"]))
    print(f"deg {deg}: {pl.info['grid_slabs']} slabs", flush=True)
    assert pl.info["grid_slabs"] >= 2
    assert np.array_equal(got, want)
    vals = B.limbs_to_ints(got)
    box = np.empty(len(vals), dtype=object)
    box[:] = vals
    box = box.reshape(tuple(d + 1 for d in pl.info["D"]))
    expect = OD.det_pointwise(arr, PL.det_degree_bound_from_shape(n, deg))
    assert box_to_dict(box) == box_to_dict(expect)


def test_grid_slabs_by_prime_ranges_and_resume():
    # prime ranges on a slabbed plan, with the coefficient region carried to a fresh workspace
    import torch
    arr = W.config2()
    want, _ = one_shot(arr)
    pl = pdm.plan(12, (3, 3, 3), host_coeffs=arr, max_workspace=6 << 20)
    assert pl.info["grid_slabs"] >= 4
    d = torch.from_numpy(arr).cuda()
    ws = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    pdm.solve_primes_device(pl, d, 0, 3, ws)
    saved = pdm.coefficient_region(pl, ws).clone()
    ws2 = torch.full_like(ws, 0x5C)
    pdm.coefficient_region(pl, ws2).copy_(saved)
    pdm.solve_primes_device(pl, d, 3, pl.info["pn"], ws2)
    out = pdm.reconstruct_device(pl, ws2)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
