"""The launch-mapping autotuner on the GPU: it produces a valid table, and solves give the
same coefficients under any table (bit-exact)."""
import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import autotune as AT
from paper_2010_12117_amd import binding as B
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def keep_tuning():
    saved = pdm.get_tuning()
    yield
    pdm.set_tuning(saved)


def solve(arr):
    import torch
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr)
    out, _ = pdm.solve_device(pl, torch.from_numpy(np.ascontiguousarray(arr)).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), pl.info


def test_autotune_small_range(keep_tuning):
    res = AT.tune(orders=[4, 12], reps=1, min_dets=100_000, rounds=1)
    table = res["table"]
    for cls in AT.CLASSES:
        for n in ("4", "12"):
            lanes = table["lanes"][cls][n]
            assert lanes in AT.supported_lanes(int(n))
            assert table["left_looking"][cls][n] in (1, 2)
            assert table["tile_points"][cls][n] in AT.TILE_POINTS
            assert len(res["timings"][cls][n]) >= 3
    assert pdm.get_tuning()["lanes"]["paired"][12] == table["lanes"]["paired"]["12"]


def test_results_do_not_depend_on_the_table(keep_tuning):
    rng = np.random.default_rng(31)
    mats = [W.random_matrix(rng, 12, (3, 2), -99, 99, zero_prob=0.3),
            W.random_matrix(rng, 9, (2, 1, 1), -99, 99, zero_prob=0.2),
            W.random_matrix(rng, 14, (4, 1), -99, 99, zero_prob=0.2),
            W.random_matrix(rng, 20, (1, 2), -9, 9, zero_prob=0.3)]
    pdm.set_tuning(None)
    base = [solve(a)[0] for a in mats]
    other = {"lanes": {"paired": {"12": 2, "9": 4, "20": 8}, "other": {"14": 4}},
             "left_looking": {"paired": {"9": 1}, "other": {"14": 1}},
             "tile_points": {"paired": {"12": 4, "20": 8}, "other": {"14": 2}}}
    pdm.set_tuning(other)
    for a, want in zip(mats, base):
        got, info = solve(a)
        assert np.array_equal(got, want)
    assert solve(mats[0])[1]["det_lanes"] == 2
    assert solve(mats[1])[1]["det_left_looking"] == 1
