"""ctypes binding of libpolydet.so (include/polydet.h), argument marshalling only.

Every stage of the determinant runs in the library's HIP kernels; this module allocates
device buffers with PyTorch, passes raw pointers and the current HIP stream, and decodes
the two's-complement limbs into Python integers. There is no fallback: if the library is
missing, loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolydet.so")
MAX_VARS = 8

OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, ECANCELLED = range(6)


def FORCE_PN(x: int) -> int:
    return (x & 0xFFF) << 8


def DET_LANES_LOG2(x: int) -> int:
    return ((x + 1) & 0xF) << 4


def PRIME_OFFSET(x: int) -> int:
    return (x & 0x3FF) << 20


UNFUSED_EVAL = 1
BATCH_PLAIN = 2
DET_LEFT_LOOKING = 4
DET_EXCHANGE = 8
HOST_ONLY = 1 << 31
STAGE_TIMING = 1 << 30
STAGES = ("reduce", "evaluate", "determinants", "finalize", "interpolate", "reconstruct")


class PolydetError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"polydet status {status}: {message}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nvars", ctypes.c_int32),
                ("deg", ctypes.c_int32 * MAX_VARS), ("coeff_bits", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nvars", ctypes.c_int32),
                ("deg", ctypes.c_int32 * MAX_VARS), ("D", ctypes.c_int32 * MAX_VARS),
                ("N", ctypes.c_int32 * MAX_VARS), ("G", ctypes.c_int64),
                ("ncoeff", ctypes.c_int64), ("nterms", ctypes.c_int64),
                ("pn", ctypes.c_int32), ("limbs", ctypes.c_int32),
                ("det_lanes", ctypes.c_int32), ("det_sign", ctypes.c_int32),
                ("in_bytes", ctypes.c_size_t), ("out_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("off_eval", ctypes.c_size_t),
                ("off_detv", ctypes.c_size_t), ("off_coef", ctypes.c_size_t),
                ("row_order", ctypes.c_uint8 * 32), ("det_left_looking", ctypes.c_int32),
                ("prime_group", ctypes.c_int32), ("coef_bytes", ctypes.c_size_t),
                ("off_den", ctypes.c_size_t), ("nslots", ctypes.c_int64),
                ("predicted_ms", ctypes.c_double), ("grid_slabs", ctypes.c_int32)]


TUNE_ORDERS = 33


class Rates(ctypes.Structure):
    """polydet_rates: the running-time prediction's rates, 0 = built-in."""
    _fields_ = [("det_updates_per_s", (ctypes.c_double * 33) * 2),
                ("reduce_bytes_per_s", ctypes.c_double), ("eval_bytes_per_s", ctypes.c_double),
                ("intt_bytes_per_s", ctypes.c_double), ("garner_ops_per_s", ctypes.c_double),
                ("launch_us", ctypes.c_double)]


RATE_SCALARS = ("reduce_bytes_per_s", "eval_bytes_per_s", "intt_bytes_per_s",
                "garner_ops_per_s", "launch_us")


class Tuning(ctypes.Structure):
    """polydet_tuning: [class][n] launch-mapping entries, 0 = built-in choice."""
    _fields_ = [("lanes", (ctypes.c_int32 * TUNE_ORDERS) * 2),
                ("left_looking", (ctypes.c_int32 * TUNE_ORDERS) * 2),
                ("tile_points", (ctypes.c_int32 * TUNE_ORDERS) * 2)]


EXPORTS = ["polydet_plan", "polydet_plan_batch", "polydet_plan_query", "polydet_plan_primes",
           "polydet_solve", "polydet_solve_batch", "polydet_plan_destroy",
           "polydet_status_string", "polydet_last_error", "polydet_limits",
           "polydet_stage_times", "polydet_set_tuning", "polydet_get_tuning",
           "polydet_plan_capped", "polydet_solve_primes", "polydet_reconstruct",
           "polydet_solve_stages", "polydet_set_rates", "polydet_get_rates",
           "polydet_solve_noalloc"]

# polydet_solve_noalloc's own workspace per device (POLYDET_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 128 << 20

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpolydet.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2010_12117_amd.build`"
                          " (the determinant path has no fallback)")
    # PyTorch, which owns device memory and streams here, ships its own HIP runtime under the
    # same soname as the system's. Whichever loads first serves the whole process, so torch
    # goes first: loaded the other way round, torch finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, u32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_size_t
    P64 = ctypes.POINTER(ctypes.c_int64)
    lib.polydet_plan.argtypes = [ctypes.POINTER(Shape), vp, u32, ctypes.POINTER(vp)]
    lib.polydet_plan_batch.argtypes = [ctypes.POINTER(Shape), i32, ctypes.POINTER(vp), u32,
                                       ctypes.POINTER(vp)]
    lib.polydet_plan_query.argtypes = [vp, i32, ctypes.POINTER(PlanInfo)]
    lib.polydet_plan_primes.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint32), i32]
    lib.polydet_solve.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.polydet_solve_batch.argtypes = [vp, vp, P64, vp, P64, vp, sz, vp]
    lib.polydet_plan_destroy.argtypes = [vp]
    lib.polydet_plan_destroy.restype = None
    lib.polydet_status_string.argtypes = [ctypes.c_int]
    lib.polydet_status_string.restype = ctypes.c_char_p
    lib.polydet_last_error.argtypes = []
    lib.polydet_last_error.restype = ctypes.c_char_p
    lib.polydet_limits.argtypes = [ctypes.POINTER(i32)] * 4
    lib.polydet_limits.restype = None
    lib.polydet_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), P64]
    lib.polydet_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.polydet_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.polydet_plan_capped.argtypes = [ctypes.POINTER(Shape), vp, u32, sz, ctypes.POINTER(vp)]
    lib.polydet_solve_primes.argtypes = [vp, vp, i32, i32, vp, sz, vp]
    lib.polydet_reconstruct.argtypes = [vp, vp, sz, vp, vp]
    lib.polydet_solve_stages.argtypes = [vp, i32, i32, vp, vp, vp, sz, vp]
    lib.polydet_set_rates.argtypes = [ctypes.POINTER(Rates)]
    lib.polydet_get_rates.argtypes = [ctypes.POINTER(Rates)]
    lib.polydet_solve_noalloc.argtypes = [vp, vp, vp, vp]
    for name in ["polydet_plan", "polydet_plan_batch", "polydet_plan_query",
                 "polydet_plan_primes", "polydet_solve", "polydet_solve_batch",
                 "polydet_stage_times", "polydet_set_tuning", "polydet_get_tuning",
                 "polydet_plan_capped", "polydet_solve_primes", "polydet_reconstruct",
                 "polydet_solve_stages", "polydet_set_rates", "polydet_get_rates",
                 "polydet_solve_noalloc"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    _install_default_tuning()
    _install_default_rates()
    return lib


# The launch-mapping table measured on the MI355X by autotune.py, shipped with the package.
# POLYDET_TUNING names another table file, or "builtin" for the library's own choices.
DEFAULT_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def _install_default_tuning():
    path = os.environ.get("POLYDET_TUNING", DEFAULT_TUNING)
    if path == "builtin" or not os.path.exists(path):
        return
    with open(path) as f:
        set_tuning(json.load(f))


# The prediction rates measured on the MI355X by calibrate.py, shipped with the package.
# POLYDET_RATES names another file, or "builtin" for the library's own values.
DEFAULT_RATES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rates_gfx950.json")


def _install_default_rates():
    path = os.environ.get("POLYDET_RATES", DEFAULT_RATES)
    if path == "builtin" or not os.path.exists(path):
        return
    with open(path) as f:
        set_rates(json.load(f))


def set_rates(table: Optional[dict]):
    """Install the running-time prediction's rates: {"det_updates_per_s": {"paired"|"other":
    {n: rate}}, "<scalar>": value, ...}; None restores the built-in rates."""
    lib = load_library()
    if table is None:
        _check(lib.polydet_set_rates(None))
        return
    r = Rates()
    for c, cls in enumerate(("paired", "other")):
        for n, v in table.get("det_updates_per_s", {}).get(cls, {}).items():
            r.det_updates_per_s[c][int(n)] = float(v)
    for f in RATE_SCALARS:
        setattr(r, f, float(table.get(f, 0.0)))
    _check(lib.polydet_set_rates(ctypes.byref(r)))


def get_rates() -> dict:
    lib = load_library()
    r = Rates()
    _check(lib.polydet_get_rates(ctypes.byref(r)))
    out = {"det_updates_per_s": {cls: {n: float(r.det_updates_per_s[c][n]) for n in range(1, 33)}
                                 for c, cls in enumerate(("paired", "other"))}}
    for f in RATE_SCALARS:
        out[f] = float(getattr(r, f))
    return out


def set_tuning(table: Optional[dict]):
    """Install a launch-mapping table: {"lanes"|"left_looking"|"tile_points": {"paired"|
    "other": {n: value}}}; None restores the library's built-in choices."""
    lib = load_library()
    if table is None:
        _check(lib.polydet_set_tuning(None))
        return
    t = Tuning()
    for field in ("lanes", "left_looking", "tile_points"):
        for c, cls in enumerate(("paired", "other")):
            for n, v in table.get(field, {}).get(cls, {}).items():
                getattr(t, field)[c][int(n)] = int(v)
    _check(lib.polydet_set_tuning(ctypes.byref(t)))


def get_tuning() -> dict:
    """The table in use, in set_tuning's form (zero entries left out)."""
    lib = load_library()
    t = Tuning()
    _check(lib.polydet_get_tuning(ctypes.byref(t)))
    out = {}
    for field in ("lanes", "left_looking", "tile_points"):
        out[field] = {cls: {n: int(getattr(t, field)[c][n]) for n in range(TUNE_ORDERS)
                            if getattr(t, field)[c][n]}
                      for c, cls in enumerate(("paired", "other"))}
    return out


def _check(status: int):
    if status != OK:
        lib = load_library()
        raise PolydetError(status, lib.polydet_last_error().decode() or
                           lib.polydet_status_string(status).decode())


def limits():
    lib = load_library()
    vals = [ctypes.c_int32() for _ in range(4)]
    lib.polydet_limits(*[ctypes.byref(v) for v in vals])
    return dict(max_n=vals[0].value, max_vars=vals[1].value, max_grid_per_var=vals[2].value,
                max_primes=vals[3].value)


def make_shape(n: int, deg: Sequence[int], coeff_bits: int = 63) -> Shape:
    s = Shape()
    s.n = int(n)
    s.nvars = len(deg)
    for v, d in enumerate(deg):
        s.deg[v] = int(d)
    s.coeff_bits = int(coeff_bits)
    return s


def shape_of(arr) -> tuple:
    """(n, deg tuple) of a coefficient array of shape (n, n, d1+1, ..., dk+1)."""
    shp = tuple(arr.shape)
    if len(shp) < 2 or shp[0] != shp[1]:
        raise ValueError("coefficients must have shape (n, n, d1+1, ..., dk+1)")
    return shp[0], tuple(x - 1 for x in shp[2:])


def coeff_bits_of(arr: np.ndarray) -> int:
    m = int(np.max(np.abs(arr.astype(object)))) if arr.size else 0
    return max(0, (m - 1).bit_length()) if m > 1 else 0


class Plan:
    """A plan (polydet_plan / polydet_plan_batch) and its queried information."""

    def __init__(self, handle, count: int):
        self._h = handle
        self.count = count
        self.infos = [self._query(i) for i in range(count)]

    def _query(self, i: int) -> dict:
        lib = load_library()
        info = PlanInfo()
        _check(lib.polydet_plan_query(self._h, i, ctypes.byref(info)))
        k = info.nvars
        d = {f: getattr(info, f) for f, _ in PlanInfo._fields_}
        for f in ("deg", "D", "N"):
            d[f] = tuple(getattr(info, f)[v] for v in range(k))
        d["row_order"] = tuple(int(info.row_order[i]) for i in range(info.n))
        arr = (ctypes.c_uint32 * max(1, info.pn))()
        _check(lib.polydet_plan_primes(self._h, i, arr, info.pn))
        d["primes"] = [int(arr[j]) for j in range(info.pn)]
        return d

    @property
    def info(self) -> dict:
        return self.infos[0]

    @property
    def handle(self):
        return self._h

    def stage_times(self) -> tuple:
        """(dict stage -> summed ms, number of solves) since the last call; the plan must
        have been made with STAGE_TIMING."""
        lib = load_library()
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int64()
        _check(lib.polydet_stage_times(self._h, ms, ctypes.byref(n)))
        return {s: float(ms[i]) for i, s in enumerate(STAGES)}, int(n.value)

    def close(self):
        if self._h:
            load_library().polydet_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan(n: int, deg: Sequence[int], host_coeffs: Optional[np.ndarray] = None,
         coeff_bits: Optional[int] = None, flags: int = 0,
         max_workspace: Optional[int] = None) -> Plan:
    """polydet_plan, or polydet_plan_capped when max_workspace (bytes) is given."""
    lib = load_library()
    if coeff_bits is None:
        coeff_bits = coeff_bits_of(host_coeffs) if host_coeffs is not None else 63
    s = make_shape(n, deg, coeff_bits)
    h = ctypes.c_void_p()
    ptr = None
    if host_coeffs is not None:
        host_coeffs = np.ascontiguousarray(host_coeffs, dtype=np.int64)
        ptr = host_coeffs.ctypes.data_as(ctypes.c_void_p)
    if max_workspace is None:
        _check(lib.polydet_plan(ctypes.byref(s), ptr, flags, ctypes.byref(h)))
    else:
        _check(lib.polydet_plan_capped(ctypes.byref(s), ptr, flags, int(max_workspace),
                                       ctypes.byref(h)))
    return Plan(h, 1)


def plan_batch(mats: Sequence[np.ndarray], use_coeffs: bool = True, flags: int = 0) -> Plan:
    lib = load_library()
    count = len(mats)
    shapes = (Shape * count)()
    ptrs = (ctypes.c_void_p * count)()
    keep = []
    for i, a in enumerate(mats):
        n, deg = shape_of(a)
        shapes[i] = make_shape(n, deg, coeff_bits_of(a))
        if use_coeffs:
            c = np.ascontiguousarray(a, dtype=np.int64)
            keep.append(c)
            ptrs[i] = c.ctypes.data
    h = ctypes.c_void_p()
    _check(lib.polydet_plan_batch(shapes, count, ptrs if use_coeffs else None, flags,
                                  ctypes.byref(h)))
    return Plan(h, count)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the determinant path runs only on the device")
    return torch


def _stream_ptr(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def solve_device(pl: Plan, d_coeffs, d_out=None, workspace=None, stream=None):
    """Enqueue polydet_solve on torch device tensors (int64 coefficients). Returns
    (out limbs as an int32 tensor of shape (ncoeff, limbs), workspace tensor)."""
    torch = _torch()
    info = pl.info
    if d_coeffs.dtype != torch.int64 or not d_coeffs.is_cuda or not d_coeffs.is_contiguous():
        raise ValueError("coefficients must be a contiguous int64 device tensor")
    if d_coeffs.numel() * 8 != info["in_bytes"]:
        raise ValueError("coefficient tensor size does not match the plan")
    if d_out is None:
        d_out = torch.empty((info["ncoeff"], info["limbs"]), dtype=torch.int32, device=d_coeffs.device)
    if workspace is None:
        workspace = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=d_coeffs.device)
    lib = load_library()
    _check(lib.polydet_solve(pl.handle, ctypes.c_void_p(d_coeffs.data_ptr()),
                             ctypes.c_void_p(d_out.data_ptr()),
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                             _stream_ptr(torch, stream)))
    return d_out, workspace


def solve_noalloc_device(pl: Plan, d_coeffs, d_out, stream=None):
    """Enqueue polydet_solve_noalloc: a solve whose workspace is the library's own device array
    (no allocation by the library; the caller passes the coefficients and the output)."""
    torch = _torch()
    info = pl.info
    if d_coeffs.dtype != torch.int64 or not d_coeffs.is_cuda or not d_coeffs.is_contiguous():
        raise ValueError("coefficients must be a contiguous int64 device tensor")
    if d_coeffs.numel() * 8 != info["in_bytes"]:
        raise ValueError("coefficient tensor size does not match the plan")
    if d_out.numel() * 4 < info["out_bytes"]:
        raise ValueError("output tensor smaller than the plan's output")
    lib = load_library()
    _check(lib.polydet_solve_noalloc(pl.handle, ctypes.c_void_p(d_coeffs.data_ptr()),
                                     ctypes.c_void_p(d_out.data_ptr()),
                                     _stream_ptr(torch, stream)))
    return d_out


def solve_stages_device(pl: Plan, stage_begin: int, stage_end: int, d_coeffs, d_out, workspace,
                        stream=None):
    """Enqueue polydet_solve_stages: stages [stage_begin, stage_end) of a solve (STAGES order)
    on a workspace that holds the earlier stages' outputs."""
    torch = _torch()
    lib = load_library()
    ptr = (lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None)
    _check(lib.polydet_solve_stages(pl.handle, int(stage_begin), int(stage_end), ptr(d_coeffs),
                                    ptr(d_out), ctypes.c_void_p(workspace.data_ptr()),
                                    workspace.numel(), _stream_ptr(torch, stream)))


def solve_primes_device(pl: Plan, d_coeffs, prime_begin: int, prime_end: int, workspace,
                        stream=None):
    """Enqueue polydet_solve_primes: S1-S4 for primes [prime_begin, prime_end), leaving their
    coefficient residues in the workspace's coefficient region."""
    torch = _torch()
    info = pl.info
    if d_coeffs.dtype != torch.int64 or not d_coeffs.is_cuda or not d_coeffs.is_contiguous():
        raise ValueError("coefficients must be a contiguous int64 device tensor")
    if d_coeffs.numel() * 8 != info["in_bytes"]:
        raise ValueError("coefficient tensor size does not match the plan")
    lib = load_library()
    _check(lib.polydet_solve_primes(pl.handle, ctypes.c_void_p(d_coeffs.data_ptr()),
                                    int(prime_begin), int(prime_end),
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    _stream_ptr(torch, stream)))


def reconstruct_device(pl: Plan, workspace, d_out=None, stream=None):
    """Enqueue polydet_reconstruct (S5) from the coefficient residues of all primes."""
    torch = _torch()
    info = pl.info
    if d_out is None:
        d_out = torch.empty((info["ncoeff"], info["limbs"]), dtype=torch.int32,
                            device=workspace.device)
    lib = load_library()
    _check(lib.polydet_reconstruct(pl.handle, ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel(), ctypes.c_void_p(d_out.data_ptr()),
                                   _stream_ptr(torch, stream)))
    return d_out


def coefficient_region(pl: Plan, workspace):
    """The workspace bytes that hold the coefficient residues (the state between calls of
    solve_primes_device), as a view."""
    info = pl.info
    return workspace[info["off_coef"]:info["off_coef"] + info["coef_bytes"]]


def solve_batch_device(pl: Plan, d_coeffs, coeff_offsets: Sequence[int], d_out,
                       out_offsets: Sequence[int], workspace=None, stream=None):
    torch = _torch()
    lib = load_library()
    if workspace is None:
        workspace = torch.empty(pl.infos[0]["workspace_bytes"], dtype=torch.uint8,
                                device=d_coeffs.device)
    if d_coeffs.dtype != torch.int64 or not d_coeffs.is_cuda or d_out.dtype != torch.int32:
        raise ValueError("coefficients must be int64 and outputs int32 device tensors")
    co = np.ascontiguousarray(coeff_offsets, dtype=np.int64)
    oo = np.ascontiguousarray(out_offsets, dtype=np.int64)
    P64 = ctypes.POINTER(ctypes.c_int64)
    _check(lib.polydet_solve_batch(pl.handle, ctypes.c_void_p(d_coeffs.data_ptr()),
                                   co.ctypes.data_as(P64), ctypes.c_void_p(d_out.data_ptr()),
                                   oo.ctypes.data_as(P64), ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel(), _stream_ptr(torch, stream)))
    return workspace


def limbs_to_ints(limbs: np.ndarray) -> List[int]:
    """Rows of little-endian two's-complement uint32 limbs -> Python ints."""
    limbs = np.asarray(limbs).view(np.uint32).astype(object)
    L = limbs.shape[-1]
    out = []
    for row in limbs.reshape(-1, L):
        x = 0
        for l in range(L - 1, -1, -1):
            x = (x << 32) | int(row[l])
        if x >> (32 * L - 1):
            x -= 1 << (32 * L)
        out.append(x)
    return out


def det(coeffs: np.ndarray, device: str = "cuda", flags: int = 0) -> np.ndarray:
    """Exact determinant of one polynomial matrix. `coeffs` is int64 of shape
    (n, n, d1+1, ..., dk+1); returns an object array of shape (D1+1, ..., Dk+1)."""
    torch = _torch()
    coeffs = np.ascontiguousarray(coeffs, dtype=np.int64)
    n, deg = shape_of(coeffs)
    pl = plan(n, deg, host_coeffs=coeffs, flags=flags)
    d_coeffs = torch.from_numpy(coeffs).to(device)
    out, _ = solve_device(pl, d_coeffs)
    torch.cuda.synchronize()
    vals = limbs_to_ints(out.cpu().numpy())
    box = tuple(d + 1 for d in pl.info["D"])
    res = np.empty(len(vals), dtype=object)
    for i, v in enumerate(vals):
        res[i] = v
    return res.reshape(box) if box else res.reshape(())
