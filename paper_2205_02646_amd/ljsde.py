"""Python binding of the RL-JSDE C ABI (``include/ljsde.h``).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``libljsde.so``. PyTorch provides device memory and streams.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libljsde.so")

OK = 0
EINVAL = -1
EUNSUPPORTED = -2
ENOMEM = -3
EHIP = -4
EBADID = -5

FP64 = 1
FP32 = 2
DFT_SPLITBF16 = 4
Q_ONES = 8
# pixel shapes: quadrant masks in flag bits 8..11 (0 = three-quarter sampling)
SHAPE_THREE_QUARTER = 0xE
SHAPE_QUARTER = 0x1


def SHAPE(mask: int) -> int:
    return (mask & 15) << 8
STATE_FP32 = 16
DENSE_C = 32
WEIGHTS = 64  # reported by plan_info for plans of plan_weights
INPUT_F64 = 128  # FP32 plans: double measurements (float output)
PLAIN_L = 4096  # plain L-JSDE (residual in the measurement domain, eq. (10) every iteration; FP64 arithmetic)

_NAMES = {EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", ENOMEM: "ENOMEM", EHIP: "EHIP", EBADID: "EBADID"}


class LjsdeError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_NAMES.get(code, code)}: {message}")
        self.code = code


class Job(ctypes.Structure):
    _fields_ = [
        ("measurements", ctypes.c_void_p),
        ("sensor_rows", ctypes.c_int),
        ("sensor_cols", ctypes.c_int),
        ("pattern_id", ctypes.c_int),
        ("out", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2205_02646_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i, d, u, vp = ctypes.c_int, ctypes.c_double, ctypes.c_uint, ctypes.c_void_p
    L.ljsde_plan.argtypes = [ctypes.POINTER(ctypes.c_uint8), i, i, i, i, i, d, d, u]
    L.ljsde_plan_weights.argtypes = [ctypes.POINTER(ctypes.c_double), i, i, i, i, i, d, d, u]
    L.ljsde_set_energy_floor.argtypes = [i, d]
    L.ljsde_reconstruct.argtypes = [vp, i, i, i, vp, vp]
    L.ljsde_reconstruct_diag.argtypes = [vp, i, i, i, vp, vp, vp]
    L.ljsde_reconstruct_batch.argtypes = [ctypes.POINTER(Job), i, vp]
    L.ljsde_reconstruct_noalloc.argtypes = [vp, i, i, i, vp, vp]
    L.ljsde_autotune.argtypes = [ctypes.POINTER(Job), i, vp]
    L.ljsde_synchronize.argtypes = [vp]
    L.ljsde_release.argtypes = [i]
    L.ljsde_last_error.restype = ctypes.c_char_p
    L.ljsde_class_count.argtypes = [i, i, i, vp]
    L.ljsde_class_tables.argtypes = [i, i, i, i, vp, vp, vp]
    L.ljsde_plan_info.argtypes = [i, vp, vp, vp, vp]
    for name in ("ljsde_plan", "ljsde_plan_weights", "ljsde_set_energy_floor", "ljsde_reconstruct", "ljsde_reconstruct_diag",
                 "ljsde_reconstruct_batch", "ljsde_reconstruct_noalloc", "ljsde_autotune", "ljsde_synchronize", "ljsde_release",
                 "ljsde_class_count", "ljsde_class_tables", "ljsde_plan_info", "ljsde_version"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int) -> int:
    if status < 0:
        raise LjsdeError(status, lib().ljsde_last_error().decode())
    return status


def last_error() -> str:
    return lib().ljsde_last_error().decode()


def version() -> int:
    return lib().ljsde_version()


def plan(pattern, window: int = 32, block: int = 4, iters: int = 100, rho: float = 0.7,
         gamma: float = 0.5, fp64: bool = False, splitbf16: bool = False, q_ones: bool = False,
         state_fp32: bool = False, shape: int = 0, dense_c: bool = False, input_f64: bool = False,
         plain_l: bool = False) -> int:
    """Register a plan for a pattern tile of quadrant codes; returns its id.
    ``shape`` is the pixel-shape mask (0 or SHAPE_THREE_QUARTER: L-shaped
    pixels; SHAPE_QUARTER: one transparent quadrant per pixel). ``dense_c``
    selects the dense form (FP64 arithmetic; float32 I/O for FP32 plans): per
    class the full C of eq. (14) in device memory, R as the loop state.
    ``input_f64``: an FP32 plan that takes float64 measurements (the output
    stays float32). ``plain_l``: plain L-JSDE, the residual kept in the
    measurement domain and eq. (10) evaluated densely (FP64 arithmetic; FP32
    plans take float32 I/O)."""
    pat = np.ascontiguousarray(np.asarray(pattern, dtype=np.uint8))
    if pat.ndim != 2:
        raise ValueError("pattern must be 2-D")
    flags = ((FP64 if fp64 else FP32) | (DFT_SPLITBF16 if splitbf16 else 0) | (Q_ONES if q_ones else 0)
             | (STATE_FP32 if state_fp32 else 0) | (DENSE_C if dense_c else 0) | SHAPE(shape)
             | (INPUT_F64 if input_f64 else 0) | (PLAIN_L if plain_l else 0))
    return _check(lib().ljsde_plan(pat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), pat.shape[0],
                                   pat.shape[1], window, block, iters, rho, gamma, flags))


def plan_weights(weights, window: int = 32, block: int = 4, iters: int = 100, rho: float = 0.7,
                 gamma: float = 0.5, q_ones: bool = False, fp64: bool = True, input_f64: bool = False,
                 plain_l: bool = False) -> int:
    """Register a plan for a general layout: ``weights`` is a [rows, cols, 4]
    tile of per-pixel quadrant weights (quadrant 2a + b of the footprint).
    Runs on the dense form in FP64; ``fp64=False`` takes float32
    measurements and returns float32 images (float64 measurements with
    ``input_f64``). ``plain_l``: plain L-JSDE instead of the dense form."""
    wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    if wt.ndim != 3 or wt.shape[2] != 4:
        raise ValueError("weights must be a [rows, cols, 4] tile")
    flags = ((FP64 if fp64 else FP32) | (PLAIN_L if plain_l else DENSE_C) | (Q_ONES if q_ones else 0)
             | (INPUT_F64 if input_f64 else 0))
    return _check(lib().ljsde_plan_weights(wt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), wt.shape[0],
                                           wt.shape[1], window, block, iters, rho, gamma, flags))


def set_energy_floor(pid: int, tau: float) -> None:
    _check(lib().ljsde_set_energy_floor(pid, tau))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_input(y, dtype):
    import torch
    if not (isinstance(y, torch.Tensor) and y.is_cuda):
        raise TypeError("measurements must be a CUDA (HIP) tensor")
    if y.dtype != dtype or y.dim() != 2 or not y.is_contiguous():
        raise TypeError(f"measurements must be a contiguous 2-D {dtype} tensor")
    return y


def _check_out(y, out, dtype):
    import torch
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.device == y.device):
        raise TypeError("out must be a CUDA (HIP) tensor on the device of the measurements")
    if out.shape != (2 * y.shape[0], 2 * y.shape[1]) or out.dtype != dtype or not out.is_contiguous():
        raise TypeError("out has the wrong shape, dtype or layout")


def _dtypes(pid: int):
    """(measurement dtype, output dtype) of a plan: the element types follow
    the plan, which the C ABI cannot check; a mismatch would make the kernels
    read or write twice (or half) the bytes."""
    import torch
    flags = plan_info(pid)["flags"]
    out = torch.float64 if flags & FP64 else torch.float32
    return (torch.float64 if flags & (FP64 | INPUT_F64) else torch.float32), out


def reconstruct(y, pid: int, out=None, fp64: Optional[bool] = None, stream=None, selections=None):
    """Reconstruct one image. ``y`` is a contiguous 2-D device tensor (float64
    for FP64 plans and FP32 plans with ``input_f64``, else float32); returns
    ``out`` (2R x 2C; float64 for FP64 plans, else float32)."""
    import torch
    ydt, odt = _dtypes(pid)
    plan_fp64 = odt == torch.float64
    if fp64 is not None and bool(fp64) != plan_fp64:
        raise TypeError(f"plan {pid} is an {'FP64' if plan_fp64 else 'FP32'} plan")
    _as_input(y, ydt)
    R, C = y.shape
    if out is None:
        out = torch.empty((2 * R, 2 * C), dtype=odt, device=y.device)
    else:
        _check_out(y, out, odt)
    if selections is None:
        _check(lib().ljsde_reconstruct(y.data_ptr(), R, C, pid, out.data_ptr(), _stream(stream)))
    else:
        _check(lib().ljsde_reconstruct_diag(y.data_ptr(), R, C, pid, out.data_ptr(), selections.data_ptr(),
                                            _stream(stream)))
    return out


def reconstruct_diag(y, pid: int, out=None, stream=None):
    """As ``reconstruct``; also returns the int16 selection sequences
    [n_windows, iters] (sigma * W + rho per iteration, -1 after a stop)."""
    import torch
    info = plan_info(pid)
    R, C = y.shape
    n_win = (2 * R // info["block"]) * (2 * C // info["block"])
    sel = torch.empty((n_win, info["iters"]), dtype=torch.int16, device=y.device)
    out = reconstruct(y, pid, out=out, stream=stream, selections=sel)
    return out, sel


def reconstruct_noalloc(y, pid: int, out, stream=None):
    """As ``reconstruct`` for an FP32 plan of the factorised form, through the
    entry point that allocates no device memory: ``out`` must be given, and
    the plan must already have reconstructed an image of this size (which
    built its tables)."""
    ydt, odt = _dtypes(pid)
    _as_input(y, ydt)
    _check_out(y, out, odt)
    R, C = y.shape
    _check(lib().ljsde_reconstruct_noalloc(y.data_ptr(), R, C, pid, out.data_ptr(), _stream(stream)))
    return out


def plan_info(pid: int) -> dict:
    w, b, it, fl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_uint()
    _check(lib().ljsde_plan_info(pid, ctypes.byref(w), ctypes.byref(b), ctypes.byref(it), ctypes.byref(fl)))
    return dict(window=w.value, block=b.value, iters=it.value, flags=fl.value)


def _jobs(items: Sequence) -> ctypes.Array:
    arr = (Job * len(items))()
    for k, (y, pid, out) in enumerate(items):
        arr[k] = Job(y.data_ptr(), y.shape[0], y.shape[1], pid, out.data_ptr())
    return arr


def reconstruct_batch(items: Iterable, stream=None) -> None:
    """``items``: sequence of (y, plan_id, out) device tensors of FP32 plans
    (y float32, or float64 for plans with ``input_f64``; out float32), or of
    plans of the dense form (one launch of the dense form over all images)."""
    import torch
    items = list(items)
    _check_items(items)
    arr = _jobs(items)
    _check(lib().ljsde_reconstruct_batch(arr, len(items), _stream(stream)))


def _check_items(items):
    import torch
    for y, pid, out in items:
        flags = plan_info(pid)["flags"]
        if flags & FP64 and not flags & DENSE_C:
            raise TypeError(f"plan {pid} is an FP64 plan of the factorised form: batches take FP32 plans "
                            "or plans of the dense form")
        ydt, odt = _dtypes(pid)
        _as_input(y, ydt)
        _check_out(y, out, odt)


def autotune(items: Iterable, stream=None) -> None:
    """Time the launch variants of the batched path on ``items`` (as for
    ``reconstruct_batch``) and keep the fastest for batches of that shape."""
    items = list(items)
    _check_items(items)
    arr = _jobs(items)
    _check(lib().ljsde_autotune(arr, len(items), _stream(stream)))


def synchronize(stream=None) -> None:
    _check(lib().ljsde_synchronize(_stream(stream)))


def release(pid: int) -> None:
    _check(lib().ljsde_release(pid))


def class_map(pid: int, sensor_rows: int, sensor_cols: int):
    """(class count, int32 class index per window in row-major block order)."""
    B = plan_info(pid)["block"]
    n_win = (2 * sensor_rows // B) * (2 * sensor_cols // B) if sensor_rows > 0 and sensor_cols > 0 else 0
    buf = np.empty(max(n_win, 1), dtype=np.int32)
    n = _check(lib().ljsde_class_count(pid, sensor_rows, sensor_cols, buf.ctypes.data))
    return n, buf[:n_win]


def class_tables(pid: int, sensor_rows: int, sensor_cols: int, cls: int, window: int):
    """FP64 tables of one class: (S [Ws*Ws, 4] complex, D [W*W], codes [Ws, Ws]);
    S is [Ws*Ws, 10] (pairs q <= q') for plans of ``plan_weights``."""
    ws = window // 2
    nspec = 10 if plan_info(pid)["flags"] & WEIGHTS else 4
    S = np.empty((ws * ws, nspec, 2), dtype=np.float64)
    D = np.empty(window * window, dtype=np.float64)
    codes = np.empty(ws * ws, dtype=np.int8)
    _check(lib().ljsde_class_tables(pid, sensor_rows, sensor_cols, cls, S.ctypes.data, D.ctypes.data,
                                    codes.ctypes.data))
    return S[..., 0] + 1j * S[..., 1], D, codes.reshape(ws, ws)
