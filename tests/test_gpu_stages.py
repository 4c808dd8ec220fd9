"""Stage ranges (polydet_solve_stages) and stage timing on the GPU: running the stages of a
solve in pieces, or running a stage again on the same workspace, gives exactly the solve's
result; stage events attribute time to the stages that ran, for single and batched plans."""
import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W

pytestmark = pytest.mark.gpu


def inputs():
    rng = np.random.default_rng(61)
    k3 = W.random_matrix(rng, 7, (2, 1, 1), -300, 300, zero_prob=0.3)
    k3[0, 0] = 0  # a structurally zero pivot: rows are reordered
    return [W.config1(), k3, np.array([[5, -2, 2 ** 50], [7, 1, 0], [3, 3, -9]], dtype=np.int64),
            W.random_matrix(rng, 13, (4,), -9, 9, zero_prob=0.2)]


@pytest.mark.parametrize("idx", range(4))
def test_stage_ranges_and_repeats_equal_the_solve(idx):
    import torch
    arr = inputs()[idx]
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr)
    d = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    ref, _ = pdm.solve_device(pl, d)
    ws = torch.empty(pl.info["workspace_bytes"], dtype=torch.uint8, device="cuda")
    for split in range(1, 6):
        out = torch.full_like(ref, -1)
        pdm.solve_stages_device(pl, 0, split, d, None, ws)
        pdm.solve_stages_device(pl, split, 6, None, out, ws)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), split
    # every stage again, some of them several times, on the finished workspace
    for s in (2, 2, 4, 4, 3, 1, 2, 4, 0):
        pdm.solve_stages_device(pl, s, s + 1, d, None, ws)
    out = torch.full_like(ref, -1)
    pdm.solve_stages_device(pl, 5, 6, None, out, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_stage_timing_of_a_single_stage():
    import torch
    arr = W.config2()
    pl = pdm.plan(12, (3, 3, 3), host_coeffs=arr, flags=pdm.STAGE_TIMING)
    d = torch.from_numpy(arr).cuda()
    out, ws = pdm.solve_device(pl, d)
    torch.cuda.synchronize()
    pl.stage_times()
    for _ in range(5):
        pdm.solve_stages_device(pl, 2, 3, None, None, ws)
    ms, solves = pl.stage_times()
    assert solves == 5 and ms["determinants"] > 0
    for s in ("reduce", "evaluate", "finalize", "interpolate", "reconstruct"):
        assert 0 <= ms[s] < 0.05 * ms["determinants"], s


def test_batch_stage_timing():
    import torch
    mats = W.config4(count=40)
    pl = pdm.plan_batch(mats, flags=pdm.STAGE_TIMING)
    co, oo, c, o = [], [], 0, 0
    for a, info in zip(mats, pl.infos):
        co.append(c)
        oo.append(o)
        c += a.size
        o += info["ncoeff"] * info["limbs"]
    d = torch.from_numpy(np.concatenate([a.reshape(-1) for a in mats])).cuda()
    out = torch.zeros(o, dtype=torch.int32, device="cuda")
    ref = torch.zeros_like(out)
    plain = pdm.plan_batch(mats, flags=pdm.BATCH_PLAIN)
    pdm.solve_batch_device(plain, d, co, ref, oo)
    for _ in range(3):
        pdm.solve_batch_device(pl, d, co, out, oo)
    ms, solves = pl.stage_times()
    assert solves == 3
    assert all(v >= 0 for v in ms.values()) and ms["determinants"] > 0
    assert ms["determinants"] > ms["reduce"]
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
