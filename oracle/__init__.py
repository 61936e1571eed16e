"""FP64 CPU oracle for the complex 2D FFT (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the package's smoke check and the
benchmark's CPU-baseline leg use this module; the product library never
imports it, and it imports nothing from the product library. It wraps the plain
C file ``fft_oracle.c`` (built with gcc into ``_oracle.so`` next to it).

Definition followed (the paper computes the discrete Fourier transform without writing it out; the sign
and normalisation below are this project's reading, pinned by tests against
closed forms, invariants and a brute-force evaluation):

    forward  X[k,l] = sum_{m,n} x[m,n] exp(-2 pi i (k m/M + l n/N))
    inverse  x[m,n] = (1/(M N)) sum_{k,l} X[k,l] exp(+2 pi i (k m/M + l n/N))

Arrays are numpy complex arrays of shape (..., M, N); results are complex128.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None

FORWARD = -1
INVERSE = +1


def build(force: bool = False) -> str:
    """Compile ``fft_oracle.c`` with gcc (-O3, OpenMP) if missing or stale."""
    stale = (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(lib):
    """Declare the C signatures on a loaded copy of the oracle library."""
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.oracle_fft1d_recursive.argtypes = [dp, i64, ci]
    lib.oracle_fft1d_listing.argtypes = [dp, dp, i64, ci]
    lib.oracle_fft1d_listing_steps.argtypes = [dp, dp, i64, ci, ci, ci, ci]
    lib.oracle_dft1d_direct.argtypes = [dp, dp, i64, ci]
    lib.oracle_dft2d_direct.argtypes = [dp, dp, i64, i64, ci]
    lib.oracle_fft2d.argtypes = [fp, dp, dp, i64, i64, i64, ci, ctypes.c_double, ci]
    lib.oracle_max_threads.argtypes = []
    for f in ("oracle_fft1d_recursive", "oracle_fft1d_listing", "oracle_fft1d_listing_steps",
              "oracle_dft1d_direct", "oracle_dft2d_direct", "oracle_fft2d", "oracle_max_threads"):
        getattr(lib, f).restype = ci
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed (code %d)" % (what, rc))


def _is_pow2(n):
    return n >= 1 and (n & (n - 1)) == 0


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def fft1d(x, sign=FORWARD) -> np.ndarray:
    """Length-n transform by the recursive radix-2 form (n a power of two)."""
    y = np.array(x, dtype=np.complex128, copy=True).ravel()
    _check(_load().oracle_fft1d_recursive(_dptr(y), y.size, int(sign)), "fft1d")
    return y


def fft1d_listing(x, sign=FORWARD) -> np.ndarray:
    """Length-n transform by the iterative bit-reversal + butterfly form."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    _check(_load().oracle_fft1d_listing(_dptr(re), _dptr(im), x.size, int(sign)), "fft1d_listing")
    return re + 1j * im


def fft1d_listing_steps(x, sign=FORWARD, permute=False, step_lo=0, step_hi=0) -> np.ndarray:
    """Only the butterfly steps step_lo..step_hi of the iterative form (optional permutation first)."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    rc = _load().oracle_fft1d_listing_steps(_dptr(re), _dptr(im), x.size, int(sign), int(bool(permute)),
                                            int(step_lo), int(step_hi))
    _check(rc, "fft1d_listing_steps")
    return re + 1j * im


def dft1d_direct(x, sign=FORWARD) -> np.ndarray:
    """The 1D definition evaluated term by term (any n >= 1)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).ravel())
    y = np.empty_like(x)
    _check(_load().oracle_dft1d_direct(_dptr(x), _dptr(y), x.size, int(sign)), "dft1d_direct")
    return y


def dft2d_direct(x, sign=FORWARD) -> np.ndarray:
    """The 2D definition evaluated term by term, one (M, N) grid (any M, N >= 1)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    if x.ndim != 2:
        raise ValueError("dft2d_direct takes one 2D grid")
    y = np.empty_like(x)
    _check(_load().oracle_dft2d_direct(_dptr(x), _dptr(y), x.shape[0], x.shape[1], int(sign)), "dft2d_direct")
    return y


def fft2(x, sign=FORWARD, scale=1.0, threads=0) -> np.ndarray:
    """2D transform over the last two axes: rows, then columns, then ``scale``.

    complex64 input is promoted exactly; complex128 input is used as is.
    """
    x = np.asarray(x)
    if x.ndim < 2:
        raise ValueError("fft2 needs at least 2 dimensions")
    M, N = x.shape[-2], x.shape[-1]
    if not (_is_pow2(M) and _is_pow2(N)):
        raise ValueError("oracle fft2 needs power-of-two sizes, got %dx%d" % (M, N))
    batch = int(np.prod(x.shape[:-2], dtype=np.int64)) if x.ndim > 2 else 1
    out = np.empty(x.shape, dtype=np.complex128)
    lib = _load()
    if x.dtype == np.complex64:
        xc = np.ascontiguousarray(x)
        fp = xc.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        rc = lib.oracle_fft2d(fp, None, _dptr(out), batch, M, N, int(sign), float(scale), int(threads))
    else:
        xc = np.ascontiguousarray(x, dtype=np.complex128)
        rc = lib.oracle_fft2d(None, _dptr(xc), _dptr(out), batch, M, N, int(sign), float(scale), int(threads))
    _check(rc, "fft2")
    return out


def fft2_forward(x, threads=0) -> np.ndarray:
    """Unscaled forward transform (exponent sign -1)."""
    return fft2(x, FORWARD, 1.0, threads)


def ifft2(x, threads=0) -> np.ndarray:
    """Inverse transform: exponent sign +1, scaled by 1/(M N)."""
    x = np.asarray(x)
    M, N = x.shape[-2], x.shape[-1]
    return fft2(x, INVERSE, 1.0 / (M * N), threads)


def adjoint(g, direction=FORWARD, threads=0) -> np.ndarray:
    """Adjoint (conjugate transpose) of the transform in ``direction``, applied to g.

    The forward transform F (sign -1, unscaled) has adjoint F^H = the unscaled
    sign +1 transform. The inverse transform (1/(MN)) F^H has adjoint
    (1/(MN)) F. This is the vector-Jacobian product of a complex-linear map
    under the convention grad = dL/dRe + i dL/dIm.
    """
    g = np.asarray(g)
    M, N = g.shape[-2], g.shape[-1]
    if direction == FORWARD:
        return fft2(g, INVERSE, 1.0, threads)
    return fft2(g, FORWARD, 1.0 / (M * N), threads)


def weighted_power_loss(x, w) -> float:
    """L(x) = sum |w * F x|^2 over every batch entry and frequency."""
    y = fft2_forward(x)
    return float(np.sum((np.asarray(w, dtype=np.float64) * np.abs(y)) ** 2))


def weighted_power_grad(x, w) -> np.ndarray:
    """Gradient of ``weighted_power_loss``: 2 F^H (w^2 * F x).

    With y = F x and L = sum w^2 |y|^2, dL/dy (as dL/dRe + i dL/dIm) is
    2 w^2 y, and the chain rule through the complex-linear F applies F^H.
    """
    w64 = np.asarray(w, dtype=np.float64)
    y = fft2_forward(x)
    return adjoint(2.0 * w64 * w64 * y, FORWARD)


def rel_l2(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2 computed in FP64."""
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((a - ref).ravel())
    return float(num / den) if den > 0 else float(num)
