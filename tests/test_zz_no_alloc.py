"""polydet_solve_noalloc (the solve whose workspace is the library's own device array) against
polydet_solve with a caller's workspace, bit for bit, on two calls in a row: the 12 x 12
trivariate degree-3 matrix (a 70 MiB workspace), then the smaller 4 x 4 bivariate one, which
runs on the scratch the first call left behind. Also: a plan whose workspace exceeds the
scratch is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import paper_2010_12117_amd as pdm
from paper_2010_12117_amd import binding as B
import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc_c_abi(pl, d, out, torch):
    lib = pdm.load_library()
    st = lib.polydet_solve_noalloc(pl.handle, ctypes.c_void_p(d.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(arr, torch):
    n, deg = B.shape_of(arr)
    pl = pdm.plan(n, deg, host_coeffs=arr)
    assert pl.info["workspace_bytes"] <= B.NOALLOC_SCRATCH_BYTES
    print(f"noalloc case n={n} deg={deg} ws={pl.info['workspace_bytes']}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    ref, _ = pdm.solve_device(pl, d)
    out = torch.full_like(ref, -1)
    assert _noalloc_c_abi(pl, d, out, torch) == B.OK
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    return pl


def test_noalloc_matches_solve_on_two_calls_second_smaller():
    torch = pytest.importorskip("torch")
    big = W.config2()
    small = W.config1()
    _case(big, torch)
    _case(small, torch)


def test_noalloc_refuses_a_plan_beyond_its_scratch():
    torch = pytest.importorskip("torch")
    # the 32 x 32 trivariate degree-5 shape needs tens of GB of workspace
    pl = pdm.plan(32, (5, 5, 5), coeff_bits=16)
    assert pl.info["workspace_bytes"] > B.NOALLOC_SCRATCH_BYTES
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert _noalloc_c_abi(pl, d, out, torch) == B.EINVAL
    assert b"scratch" in pdm.load_library().polydet_last_error()
