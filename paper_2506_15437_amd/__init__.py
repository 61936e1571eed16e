"""MI355X (gfx950) complex 2D FFT: hand-written HIP kernels behind a C ABI.

The transform is the paper's radix-2 Cooley-Tukey 2D FFT (Brown, Davies,
Le Clair, arXiv 2506.15437: Section 2.2 / Listing 1 for the butterflies,
Section 5 / Fig. 6 for the row-then-column scheme), FP32 complex64 data:

    forward  X[k,l] = sum_{m,n} x[m,n] exp(-2 pi i (k m/M + l n/N))
    inverse  x[m,n] = (1/(M N)) sum_{k,l} X[k,l] exp(+2 pi i (k m/M + l n/N))

PyTorch supplies device memory and streams only; the transform runs in
``libfft2d.so``. The library is loaded on first use of any name below, and
that raises ImportError if it is not built (``python -m
paper_2506_15437_amd.build``): there is no other implementation to fall back to.

Torch-level API:
    fft2(x), ifft2(x)                  complex64 GPU tensors (..., M, N)
    fft2_batched(xs, direction)        list of 2D tensors of different shapes
    FFT2Function.apply(x, direction)   differentiable (adjoint kernel backward)
C-ABI-level API (same names as the C functions, pointers as ints):
    fft2d_plan, fft2d_plan_batched, fft2d_exec, fft2d_exec_pass, fft2d_exec_pass_timed,
    fft2d_exec_batched, fft2d_backward, fft2d_destroy, fft2d_plan_describe,
    fft2d_exec_noalloc (no plan, no allocation), fft2d_exec_pass_ablated,
    fft2d_probe_dft16, fft2d_probe_tile_copy and fft2d_probe_lds (measurement aids)
"""

from __future__ import annotations

_LIB_NAMES = ("EXPORTS", "FORWARD", "INVERSE", "LIB_PATH", "MAX_LEN", "Fft2dError", "fft2d_plan",
              "fft2d_plan_batched", "fft2d_exec", "fft2d_exec_pass", "fft2d_exec_pass_timed", "fft2d_exec_batched",
              "fft2d_backward", "fft2d_destroy", "fft2d_plan_describe", "fft2d_plan_twiddles", "fft2d_exec_noalloc", "NOALLOC_WORK_BYTES", "fft2d_exec_pass_ablated",
              "ABLATE_ARITHMETIC", "ABLATE_EXCHANGE", "fft2d_probe_dft16", "DFT16_BUTTERFLY", "DFT16_MFMA",
              "fft2d_probe_tile_copy", "fft2d_probe_lds",
              "status_string",
              "last_error", "version", "pointer_array")
_API_NAMES = ("Plan", "BatchedPlan", "get_plan", "fft2", "ifft2", "fft2_batched", "FFT2Function", "fft2_diff")

__all__ = list(_LIB_NAMES + _API_NAMES)


def __getattr__(name):
    if name in _LIB_NAMES:
        from . import _lib
        return getattr(_lib, name)
    if name in _API_NAMES:
        from . import api
        return getattr(api, name)
    raise AttributeError("module %r has no attribute %r" % (__name__, name))
