"""Python binding of libletkf.so (include/letkf.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Tensors are
torch tensors on the plan's device (float64 / int32, contiguous); with
LETKF_FLAG_OBS_ON_HOST the observation arrays are host tensors instead.
Streams default to torch's current stream.  All arithmetic runs in the
library's gfx950 kernels: if the library is missing, loading raises instead
of falling back to anything else.

Before a call reaches the library, each letkf_io is checked against the
plan's problem descriptors: a tensor of the wrong size, dtype or device would
otherwise make the kernels read or write outside it.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Iterable, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libletkf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "letkf.h")

LETKF_OK, LETKF_EINVAL, LETKF_ENOMEM, LETKF_EDEVICE = 0, 1, 2, 3
LETKF_EBUSY, LETKF_ENONFINITE, LETKF_ENOTCONV, LETKF_EIO = 4, 5, 6, 7
LETKF_LOC_GAUSS, LETKF_LOC_GC, LETKF_LOC_NONE = 0, 1, 2
LETKF_PREC_FP64, LETKF_PREC_FP32, LETKF_PREC_BF16 = 0, 1, 2
LETKF_OBS_RHO, LETKF_OBS_U, LETKF_OBS_V = 0, 1, 2
LETKF_MAX_K = 64
LETKF_FLAG_PHASE_TIMING = 1
LETKF_FLAG_CYCLE = 2
LETKF_FLAG_OBS_ON_HOST = 4
LETKF_FLAG_DETERMINISTIC = 8
LETKF_FLAG_GRAPH_CAPTURE = 16
LETKF_FLAG_NSQRT = 32
LETKF_FORM_GRID, LETKF_FORM_PERSISTENT, LETKF_FORM_FUSED, LETKF_FORM_AUTO = 0, 1, 2, 3
PHASES = ("bin", "transpose", "obs_operator", "gram", "evd_update", "untranspose", "fused")


class letkf_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("k", ctypes.c_int32),
                ("n_obs_max", ctypes.c_int32), ("loc_len", ctypes.c_double),
                ("infl", ctypes.c_double), ("loc", ctypes.c_int32), ("precision", ctypes.c_int32)]


class letkf_options(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tune_cache_path", ctypes.c_char_p)]


class letkf_io(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int32), ("n_obs", ctypes.c_int32),
                ("xb", ctypes.c_void_p), ("xa", ctypes.c_void_p),
                ("obs_ix", ctypes.c_void_p), ("obs_iy", ctypes.c_void_p),
                ("obs_kind", ctypes.c_void_p), ("obs_val", ctypes.c_void_p),
                ("obs_var", ctypes.c_void_p)]


class letkf_tuning(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("form", ctypes.c_int32),
                ("ms_per_call", ctypes.c_double)]


class letkf_cycle_io(ctypes.Structure):
    _fields_ = [("io", letkf_io), ("n_steps", ctypes.c_int32), ("force_kx", ctypes.c_int32),
                ("tau", ctypes.c_double), ("force_amp", ctypes.c_double)]


_lib = None
# plan handle -> (problem descriptors, flags), for the argument checks
_plans: dict = {}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libletkf.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with paper_2308_03310_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, u64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p
    lib.letkf_plan.argtypes = [ctypes.POINTER(letkf_problem), i32, ctypes.POINTER(letkf_options),
                               ctypes.POINTER(vp)]
    lib.letkf_plan.restype = ctypes.c_int
    lib.letkf_analyze.argtypes = [vp, ctypes.POINTER(letkf_io), i32, vp]
    lib.letkf_analyze.restype = ctypes.c_int
    lib.letkf_cycle.argtypes = [vp, ctypes.POINTER(letkf_cycle_io), i32, vp]
    lib.letkf_cycle.restype = ctypes.c_int
    lib.letkf_advance.argtypes = [vp, ctypes.POINTER(letkf_cycle_io), i32, vp]
    lib.letkf_advance.restype = ctypes.c_int
    lib.letkf_status.argtypes = [vp, i32]
    lib.letkf_status.restype = ctypes.c_int
    lib.letkf_plan_destroy.argtypes = [vp]
    lib.letkf_plan_destroy.restype = ctypes.c_int
    lib.letkf_strerror.argtypes = [ctypes.c_int]
    lib.letkf_strerror.restype = ctypes.c_char_p
    lib.letkf_plan_workspace_bytes.argtypes = [vp]
    lib.letkf_plan_workspace_bytes.restype = u64
    lib.letkf_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int32), i32]
    lib.letkf_phase_times.restype = ctypes.c_int
    lib.letkf_eigh_batched.argtypes = [dp, i32, i32, dp, dp, dp, vp]
    lib.letkf_eigh_batched.restype = ctypes.c_int
    lib.letkf_invsqrt_batched.argtypes = [dp, i32, i32, dp, vp, vp, vp]
    lib.letkf_invsqrt_batched.restype = ctypes.c_int
    lib.letkf_analyze_noalloc.argtypes = [ctypes.POINTER(letkf_problem), ctypes.POINTER(letkf_io),
                                          dp, vp]
    lib.letkf_analyze_noalloc.restype = ctypes.c_int
    lib.letkf_tune.argtypes = [vp, ctypes.POINTER(letkf_io), i32, vp, ctypes.POINTER(letkf_tuning)]
    lib.letkf_tune.restype = ctypes.c_int
    lib.letkf_set_tuning.argtypes = [vp, ctypes.POINTER(letkf_tuning)]
    lib.letkf_set_tuning.restype = ctypes.c_int
    _lib = lib
    return lib


def header_functions(path: str = HEADER) -> list:
    """Names of the functions include/letkf.h declares."""
    txt = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|uint64_t)\s+(letkf_\w+)\s*\(", txt, re.M)))


class LetkfError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {letkf_strerror(code)} ({code})")


def _check(code: int, where: str) -> int:
    if code != LETKF_OK:
        raise LetkfError(code, where)
    return code


def _ptr(t, dtype=None, host: bool = False) -> int:
    if t is None:
        return 0
    import torch
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if host and t.is_cuda:
        raise TypeError("expected a host tensor (LETKF_FLAG_OBS_ON_HOST)")
    if not host and not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def letkf_strerror(code: int) -> str:
    return load_library().letkf_strerror(int(code)).decode()


def make_problem(nx, ny, k, n_obs_max, loc_len, infl, loc=LETKF_LOC_GAUSS,
                 precision=LETKF_PREC_FP64) -> letkf_problem:
    return letkf_problem(int(nx), int(ny), int(k), int(n_obs_max), float(loc_len), float(infl),
                         int(loc), int(precision))


def letkf_plan(problems: Sequence[letkf_problem], hbm_budget_bytes: int = 0, flags: int = 0,
               raise_on_error: bool = True, tune_cache_path: Optional[str] = None):
    """Returns the plan handle (int), or (code, None) when raise_on_error is False."""
    lib = load_library()
    arr = (letkf_problem * len(problems))(*problems) if len(problems) else None
    path = tune_cache_path.encode() if tune_cache_path else None
    opt = letkf_options(int(hbm_budget_bytes), int(flags), 0, path)
    h = ctypes.c_void_p()
    rc = lib.letkf_plan(arr, len(problems), ctypes.byref(opt), ctypes.byref(h))
    if rc == LETKF_OK and h.value:
        _plans[h.value] = ([letkf_problem(p.nx, p.ny, p.k, p.n_obs_max, p.loc_len, p.infl, p.loc,
                                          p.precision) for p in problems], int(flags))
    if not raise_on_error:
        return rc, h.value
    _check(rc, "letkf_plan")
    return h.value


def make_io(problem: int, xb, xa, obs=None, obs_on_host: bool = False) -> letkf_io:
    """obs: dict or tuple of tensors (ix, iy, kind int32; val, var float64) on
    the device, or on the host for a plan made with LETKF_FLAG_OBS_ON_HOST
    (obs_on_host=True).  The element counts are kept with the descriptor and
    checked against the plan's problem when the call is made, and so are
    references to the tensors: they live at least as long as the descriptor
    (the calls are asynchronous, so keep it, or the tensors, until the
    stream has run them)."""
    import torch
    if obs is None:
        n, p, counts = 0, (0, 0, 0, 0, 0), ()
    else:
        if isinstance(obs, dict):
            obs = (obs["ix"], obs["iy"], obs["kind"], obs["val"], obs["var"])
        ix, iy, kd, val, var = obs
        n = int(ix.numel())
        h = bool(obs_on_host)
        p = (_ptr(ix, torch.int32, h), _ptr(iy, torch.int32, h), _ptr(kd, torch.int32, h),
             _ptr(val, torch.float64, h), _ptr(var, torch.float64, h))
        counts = tuple(int(t.numel()) for t in (ix, iy, kd, val, var))
    io = letkf_io(int(problem), n, _ptr(xb, torch.float64), _ptr(xa, torch.float64), *p)
    io._numel = (int(xb.numel()), int(xa.numel())) + counts
    io._obs_on_host = bool(obs_on_host) and obs is not None
    io._keep = (xb, xa, obs)
    return io


def _validate(plan: int, io: letkf_io) -> None:
    """Sizes of io's arrays against the plan's problem (raises ValueError)."""
    entry = _plans.get(plan)
    if entry is None:
        return
    probs, flags = entry
    if not 0 <= io.problem < len(probs):
        raise ValueError(f"problem index {io.problem} out of range ({len(probs)} problems)")
    _validate_sizes(probs[io.problem], io, flags)


def _validate_sizes(p: letkf_problem, io: letkf_io, flags: int) -> None:
    counts = getattr(io, "_numel", None)
    if counts is None:
        raise ValueError("letkf_io must be made with make_io (its array sizes are checked)")
    state = p.nx * p.ny * 9 * p.k
    if counts[0] != state or counts[1] != state:
        raise ValueError(f"xb / xa hold {counts[0]} / {counts[1]} values, the problem "
                         f"needs {state} ([{p.k}][9][{p.ny}][{p.nx}])")
    if any(c != io.n_obs for c in counts[2:]):
        raise ValueError(f"observation arrays differ in length: {counts[2:]}")
    if io.n_obs > p.n_obs_max:
        raise ValueError(f"{io.n_obs} observations, the plan allows {p.n_obs_max}")
    host = bool(flags & LETKF_FLAG_OBS_ON_HOST)
    if io.n_obs > 0 and io._obs_on_host != host:
        raise ValueError("observation arrays must be " + ("host" if host else "device") +
                         " tensors for this plan")


def letkf_analyze(plan: int, ios: Iterable[letkf_io], stream=None) -> int:
    ios = list(ios)
    for io in ios:
        _validate(plan, io)
    arr = (letkf_io * len(ios))(*ios)
    return _check(load_library().letkf_analyze(plan, arr, len(ios), _stream(stream)),
                  "letkf_analyze")


def make_cycle_io(problem: int, x, obs=None, n_steps: int = 50, tau: float = 0.52,
                  force_amp: float = 1e-5, force_kx: int = 4,
                  obs_on_host: bool = False) -> letkf_cycle_io:
    """In-place cycle descriptor for ensemble x (advanced, then analysed)."""
    io = make_io(problem, x, x, obs, obs_on_host)
    c = letkf_cycle_io(io, int(n_steps), int(force_kx), float(tau), float(force_amp))
    c._io = io
    return c


def letkf_cycle(plan: int, ios: Iterable[letkf_cycle_io], stream=None) -> int:
    ios = list(ios)
    for c in ios:
        _validate(plan, getattr(c, "_io", c.io))
    arr = (letkf_cycle_io * len(ios))(*ios)
    return _check(load_library().letkf_cycle(plan, arr, len(ios), _stream(stream)), "letkf_cycle")


def letkf_advance(plan: int, ios: Iterable[letkf_cycle_io], stream=None) -> int:
    """The forecast step alone: each ensemble advanced n_steps BGK steps in place."""
    ios = list(ios)
    for c in ios:
        io = getattr(c, "_io", c.io)
        entry = _plans.get(plan)
        if entry is not None:
            probs, _ = entry
            if not 0 <= io.problem < len(probs):
                raise ValueError(f"problem index {io.problem} out of range")
            p = probs[io.problem]
            counts = getattr(io, "_numel", None)
            if counts is None or counts[0] != p.nx * p.ny * 9 * p.k:
                raise ValueError("advance: the ensemble does not fit the problem")
    arr = (letkf_cycle_io * len(ios))(*ios)
    return _check(load_library().letkf_advance(plan, arr, len(ios), _stream(stream)),
                  "letkf_advance")


def letkf_status(plan: int, sync: bool = True) -> int:
    return load_library().letkf_status(plan, 1 if sync else 0)


def letkf_plan_destroy(plan: Optional[int]) -> int:
    _plans.pop(plan, None)
    return load_library().letkf_plan_destroy(plan)


def letkf_plan_workspace_bytes(plan: int) -> int:
    return int(load_library().letkf_plan_workspace_bytes(plan))


def letkf_phase_times(plan: int):
    """(calls, {phase: summed ms}, {phase: launches per call}) since the last read."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    la = (ctypes.c_int32 * n)()
    calls = load_library().letkf_phase_times(plan, ms, la, n)
    if calls < 0:
        raise LetkfError(-calls, "letkf_phase_times")
    return calls, dict(zip(PHASES, list(ms))), dict(zip(PHASES, list(la)))


def letkf_eigh_batched(a, lam, vec, status=None, stream=None) -> int:
    """a [batch, k, k] float64 -> lam [batch, k], vec [batch, k, k] (columns)."""
    import torch
    batch, k = int(a.shape[0]), int(a.shape[-1])
    if a.numel() != batch * k * k or lam.numel() != batch * k or vec.numel() != batch * k * k:
        raise ValueError(f"eigh_batched: a {tuple(a.shape)}, lam {tuple(lam.shape)}, "
                         f"vec {tuple(vec.shape)} do not fit batch {batch}, k {k}")
    if status is not None and status.numel() < 1:
        raise ValueError("eigh_batched: status needs one int32")
    return _check(load_library().letkf_eigh_batched(
        _ptr(a, torch.float64), batch, k, _ptr(lam, torch.float64), _ptr(vec, torch.float64),
        _ptr(status, torch.int32) if status is not None else None, _stream(stream)),
        "letkf_eigh_batched")


def letkf_invsqrt_batched(a, x, status=None, steps=None, stream=None) -> int:
    """a [batch, k, k] float64 SPD -> x = a^-1/2 [batch, k, k] (coupled
    Newton-Schulz on MFMA); steps, if given, an int32 [batch] tensor that
    receives each matrix's step count."""
    import torch
    batch, k = int(a.shape[0]), int(a.shape[-1])
    if a.numel() != batch * k * k or x.numel() != batch * k * k:
        raise ValueError(f"invsqrt_batched: a {tuple(a.shape)}, x {tuple(x.shape)} do not fit "
                         f"batch {batch}, k {k}")
    if status is not None and status.numel() < 1:
        raise ValueError("invsqrt_batched: status needs one int32")
    if steps is not None and steps.numel() < batch:
        raise ValueError(f"invsqrt_batched: steps needs {batch} int32")
    return _check(load_library().letkf_invsqrt_batched(
        _ptr(a, torch.float64), batch, k, _ptr(x, torch.float64),
        _ptr(status, torch.int32) if status is not None else None,
        _ptr(steps, torch.int32) if steps is not None else None, _stream(stream)),
        "letkf_invsqrt_batched")


def letkf_analyze_noalloc(problem: letkf_problem, io: letkf_io, status, stream=None) -> int:
    """One analysis of one problem without a plan (the library's static
    workspace; nothing is allocated).  status: a device int32 tensor that
    receives the analysis' device status bits."""
    import torch
    _validate_sizes(problem, io, 0)
    if status is None or status.numel() < 1:
        raise ValueError("analyze_noalloc: status needs one int32")
    return _check(load_library().letkf_analyze_noalloc(
        ctypes.byref(problem), ctypes.byref(io), _ptr(status, torch.int32), _stream(stream)),
        "letkf_analyze_noalloc")


def letkf_tune(plan: int, ios: Iterable[letkf_io], stream=None) -> dict:
    """Autotune the plan's launch settings on these analyses; returns the setting kept."""
    ios = list(ios)
    for io in ios:
        _validate(plan, io)
    arr = (letkf_io * len(ios))(*ios)
    t = letkf_tuning()
    _check(load_library().letkf_tune(plan, arr, len(ios), _stream(stream), ctypes.byref(t)),
           "letkf_tune")
    return {"cell": t.cell, "form": t.form, "ms_per_call": t.ms_per_call}


def letkf_set_tuning(plan: int, cell: int, form: int) -> int:
    """Apply a setting: observation-cell edge and kernel form (LETKF_FORM_*)."""
    t = letkf_tuning(int(cell), int(form), 0.0)
    return _check(load_library().letkf_set_tuning(plan, ctypes.byref(t)), "letkf_set_tuning")
