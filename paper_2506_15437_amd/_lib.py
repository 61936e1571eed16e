"""ctypes binding of ``libfft2d.so``: the C ABI under the same names.

Only argument marshalling lives here; every step of the transform runs in the
library's HIP kernels. Pointers are passed as Python ints (device addresses),
streams as ints (hipStream_t values, 0 = default stream). Every function
raises ``Fft2dError`` when the library returns a non-zero status.

The library is built in-tree by ``paper_2506_15437_amd.build``; if it is
missing this module raises at import time instead of falling back to
anything else.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfft2d.so")

FORWARD = -1
INVERSE = +1
MAX_LEN = 16384

STATUS_NAMES = {
    0: "FFT2D_OK",
    1: "FFT2D_ERR_NULL_POINTER",
    2: "FFT2D_ERR_INVALID_SIZE",
    3: "FFT2D_ERR_INVALID_DIRECTION",
    4: "FFT2D_ERR_MISALIGNED",
    5: "FFT2D_ERR_WRONG_PLAN_KIND",
    6: "FFT2D_ERR_OUT_OF_MEMORY",
    7: "FFT2D_ERR_HIP",
    8: "FFT2D_ERR_INVALID_PLAN",
    9: "FFT2D_ERR_OVERLAP",
    10: "FFT2D_ERR_INCOMPLETE",
    11: "FFT2D_ERR_WRONG_DEVICE",
}

# Every symbol the public header declares.
EXPORTS = ("fft2d_plan", "fft2d_plan_batched", "fft2d_exec", "fft2d_exec_pass", "fft2d_exec_pass_timed",
           "fft2d_exec_pass_ablated",
           "fft2d_exec_batched",
           "fft2d_backward", "fft2d_destroy", "fft2d_status_string", "fft2d_last_error", "fft2d_plan_describe",
           "fft2d_plan_twiddles", "fft2d_exec_noalloc", "fft2d_probe_dft16", "fft2d_probe_tile_copy", "fft2d_probe_lds",
           "fft2d_version")


class Fft2dError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        self.name = STATUS_NAMES.get(status, "status %d" % status)
        super().__init__("%s: %s (%s)%s" % (where, self.name, status_string(status), (": " + detail) if detail else ""))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfft2d.so is not built (expected at %s); run `python -m paper_2506_15437_amd.build`"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    pp = ctypes.POINTER(vp)
    lib.fft2d_plan.argtypes = [pp, i64, i64, i64]
    lib.fft2d_plan_batched.argtypes = [pp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.fft2d_exec.argtypes = [vp, vp, vp, ci, vp]
    lib.fft2d_exec_pass.argtypes = [vp, vp, vp, ci, ci, vp]
    lib.fft2d_exec_pass_timed.argtypes = [vp, vp, vp, ci, ci, vp, vp, vp]
    lib.fft2d_exec_pass_ablated.argtypes = [vp, vp, vp, ci, ci, vp, vp, vp]
    lib.fft2d_exec_batched.argtypes = [vp, vp, vp, ci, vp]
    lib.fft2d_backward.argtypes = [vp, vp, vp, ci, vp]
    lib.fft2d_destroy.argtypes = [vp]
    lib.fft2d_status_string.argtypes = [ci]
    lib.fft2d_status_string.restype = ctypes.c_char_p
    lib.fft2d_last_error.argtypes = []
    lib.fft2d_last_error.restype = ctypes.c_char_p
    lib.fft2d_plan_describe.argtypes = [vp, ctypes.c_char_p, i64]
    lib.fft2d_plan_twiddles.argtypes = [vp, ci, vp, i64, ctypes.POINTER(i64)]
    lib.fft2d_exec_noalloc.argtypes = [i64, i64, i64, vp, vp, ci, vp]
    lib.fft2d_probe_dft16.argtypes = [ci, vp, vp, i64, ci, vp, vp, vp]
    lib.fft2d_probe_tile_copy.argtypes = [vp, vp, i64, i64, ci, ci, ci, vp, vp, vp]
    lib.fft2d_probe_lds.argtypes = [ci, ci, vp, i64, ctypes.POINTER(i64), vp, vp, vp]
    lib.fft2d_version.argtypes = []
    lib.fft2d_version.restype = ci
    for f in ("fft2d_plan", "fft2d_plan_batched", "fft2d_exec", "fft2d_exec_pass", "fft2d_exec_pass_timed",
              "fft2d_exec_pass_ablated",
              "fft2d_exec_batched", "fft2d_backward",
              "fft2d_destroy", "fft2d_plan_describe", "fft2d_plan_twiddles", "fft2d_exec_noalloc",
              "fft2d_probe_dft16", "fft2d_probe_tile_copy", "fft2d_probe_lds"):
        getattr(lib, f).restype = ci
    return lib


lib = _load()


def status_string(status: int) -> str:
    return lib.fft2d_status_string(int(status)).decode()


def last_error() -> str:
    return lib.fft2d_last_error().decode()


def _check(status, where):
    if status != 0:
        raise Fft2dError(status, where, last_error())


def version() -> int:
    return int(lib.fft2d_version())


def fft2d_plan(batch: int, rows: int, cols: int) -> int:
    """Create a uniform plan; returns the opaque handle as an int."""
    h = ctypes.c_void_p()
    _check(lib.fft2d_plan(ctypes.byref(h), int(batch), int(rows), int(cols)), "fft2d_plan")
    return int(h.value)


def fft2d_plan_batched(rows, cols) -> int:
    """Create a batched plan for shapes rows[i] x cols[i]; returns the handle."""
    n = len(rows)
    if len(cols) != n:
        raise ValueError("rows and cols must have the same length")
    ra = (ctypes.c_int64 * max(n, 1))(*[int(r) for r in rows])
    ca = (ctypes.c_int64 * max(n, 1))(*[int(c) for c in cols])
    h = ctypes.c_void_p()
    _check(lib.fft2d_plan_batched(ctypes.byref(h), n, ra, ca), "fft2d_plan_batched")
    return int(h.value)


def fft2d_exec(plan: int, in_ptr: int, out_ptr: int, direction: int, stream: int = 0) -> None:
    _check(lib.fft2d_exec(plan, in_ptr, out_ptr, int(direction), stream), "fft2d_exec")


def fft2d_exec_pass(plan: int, in_ptr: int, out_ptr: int, direction: int, pass_index: int, stream: int = 0) -> None:
    _check(lib.fft2d_exec_pass(plan, in_ptr, out_ptr, int(direction), int(pass_index), stream), "fft2d_exec_pass")


def fft2d_exec_pass_timed(plan: int, in_ptr: int, out_ptr: int, direction: int, pass_index: int,
                          start_event: int, stop_event: int, stream: int = 0) -> None:
    """start_event, stop_event: hipEvent_t handles (e.g. torch.cuda.Event(enable_timing=True).cuda_event
    once the event has been recorded); they take the pass kernel's own start and end times."""
    _check(lib.fft2d_exec_pass_timed(plan, in_ptr, out_ptr, int(direction), int(pass_index), start_event,
                                     stop_event, stream), "fft2d_exec_pass_timed")


ABLATE_ARITHMETIC = 1
ABLATE_EXCHANGE = 2


def fft2d_exec_pass_ablated(plan: int, in_ptr: int, out_ptr: int, pass_index: int, ablation: int,
                            start_event: int = 0, stop_event: int = 0, stream: int = 0) -> None:
    """One pass with its arithmetic (ABLATE_ARITHMETIC) or its arithmetic and LDS exchanges
    (ABLATE_EXCHANGE) switched off: the pass's data-movement floor. Events as for
    fft2d_exec_pass_timed, or both 0."""
    _check(lib.fft2d_exec_pass_ablated(plan, in_ptr, out_ptr, int(pass_index), int(ablation),
                                       start_event or None, stop_event or None, stream), "fft2d_exec_pass_ablated")


def pointer_array(ptrs):
    """Device pointers as a contiguous uint64 array (returned as is if it already is one),
    the layout of the ``const void* const*`` arrays of fft2d_exec_batched."""
    return np.ascontiguousarray(ptrs, dtype=np.uint64)


def fft2d_exec_batched(plan: int, in_ptrs, out_ptrs, direction: int, stream: int = 0) -> None:
    """in_ptrs, out_ptrs: sequences of device pointers, or uint64 arrays from pointer_array()
    (no per-call conversion: what a caller that replays one pointer set should pass)."""
    ia = pointer_array(in_ptrs)
    oa = pointer_array(out_ptrs)
    if ia.size != oa.size:
        raise ValueError("in_ptrs and out_ptrs differ in length")
    _check(lib.fft2d_exec_batched(plan, ia.ctypes.data, oa.ctypes.data, int(direction), stream),
           "fft2d_exec_batched")


def fft2d_backward(plan: int, grad_out_ptr: int, grad_in_ptr: int, forward_direction: int, stream: int = 0) -> None:
    _check(lib.fft2d_backward(plan, grad_out_ptr, grad_in_ptr, int(forward_direction), stream), "fft2d_backward")


def fft2d_exec_noalloc(batch: int, rows: int, cols: int, in_ptr: int, out_ptr: int, direction: int,
                       stream: int = 0) -> None:
    """fft2d_exec without a plan or any allocation (library-owned device array)."""
    _check(lib.fft2d_exec_noalloc(int(batch), int(rows), int(cols), in_ptr, out_ptr, int(direction), stream),
           "fft2d_exec_noalloc")


NOALLOC_WORK_BYTES = 64 * 1024 * 1024

DFT16_BUTTERFLY = 0
DFT16_MFMA = 1


def fft2d_probe_dft16(method: int, in_ptr: int, out_ptr: int, count: int, reps: int, start_event: int = 0,
                      stop_event: int = 0, stream: int = 0) -> None:
    """count 16-point vectors, (Pi F / 4)^reps applied in registers by butterflies or MFMA (rate probe)."""
    _check(lib.fft2d_probe_dft16(int(method), in_ptr, out_ptr, int(count), int(reps), start_event or None,
                                 stop_event or None, stream), "fft2d_probe_dft16")


def fft2d_probe_tile_copy(in_ptr: int, out_ptr: int, rows: int, cols: int, tile_cols: int, residues: int,
                          nontemporal: bool, start_event: int = 0, stop_event: int = 0, stream: int = 0) -> None:
    """Copy of a rows x cols grid in column tiles of tile_cols columns (access-pattern probe)."""
    _check(lib.fft2d_probe_tile_copy(in_ptr, out_ptr, int(rows), int(cols), int(tile_cols), int(residues),
                                     1 if nontemporal else 0, start_event or None, stop_event or None, stream),
           "fft2d_probe_tile_copy")


def fft2d_probe_lds(width_bytes: int, write: bool, sink_ptr: int, sink_floats: int, start_event: int = 0,
                    stop_event: int = 0, stream: int = 0) -> int:
    """LDS read or write bandwidth probe; returns the bytes the launch moves."""
    b = ctypes.c_int64(0)
    _check(lib.fft2d_probe_lds(int(width_bytes), 1 if write else 0, sink_ptr, int(sink_floats), ctypes.byref(b),
                               start_event or None, stop_event or None, stream), "fft2d_probe_lds")
    return int(b.value)


def fft2d_destroy(plan: int) -> None:
    _check(lib.fft2d_destroy(plan), "fft2d_destroy")


def fft2d_plan_twiddles(plan: int, which: int) -> np.ndarray:
    """One of a uniform plan's FP32 twiddle tables as complex64 (0 row pass, 1 column pass, 2 combine)."""
    n = ctypes.c_int64(0)
    _check(lib.fft2d_plan_twiddles(plan, int(which), None, 0, ctypes.byref(n)), "fft2d_plan_twiddles")
    out = np.zeros(max(n.value, 0), dtype=np.complex64)
    if n.value > 0:
        _check(lib.fft2d_plan_twiddles(plan, int(which), out.ctypes.data, n.value, ctypes.byref(n)),
               "fft2d_plan_twiddles")
    return out


def fft2d_plan_describe(plan: int) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib.fft2d_plan_describe(plan, buf, len(buf)), "fft2d_plan_describe")
    return buf.value.decode()
