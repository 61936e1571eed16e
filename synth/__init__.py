"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no Fourier arithmetic at all: it only draws numbers. Both
the FP64 oracle and the GPU path receive the very same float32 values from
here, so a parity comparison never depends on two generators agreeing.

Recipes (all from ``numpy.random.default_rng``, PCG64):

* complex grids: real and imaginary parts are ``2*u - 1`` with ``u`` drawn as
  float32 uniform on [0, 1). numpy's float32 uniforms are multiples of 2**-24,
  so ``2*u - 1`` is exact in float32 and lies in [-1, 1). The draw is one array
  of shape ``shape + (2,)`` read as interleaved (re, im) pairs.
* real weights: float32 uniform on [0, 1).
* batched shape lists: ``rows = 2**a``, ``cols = 2**b`` with ``a`` and ``b``
  integers drawn uniformly from [lo, hi] inclusive.
* per-item data of a batched list: item ``i`` uses ``default_rng([seed, i])``.
"""

from __future__ import annotations

import numpy as np

__all__ = ["complex_grid", "real_weights", "pow2_shapes", "batched_grids"]


def complex_grid(seed, shape) -> np.ndarray:
    """complex64 array of ``shape`` with re, im i.i.d. uniform on [-1, 1)."""
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    u = rng.random(shape + (2,), dtype=np.float32)
    v = (np.float32(2.0) * u - np.float32(1.0)).astype(np.float32)
    return np.ascontiguousarray(v).view(np.complex64).reshape(shape)


def real_weights(seed, shape) -> np.ndarray:
    """float32 array of ``shape`` with entries i.i.d. uniform on [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random(tuple(int(s) for s in shape), dtype=np.float32)


def pow2_shapes(seed, count, lo=6, hi=11):
    """``count`` shapes (2**a, 2**b) with a, b uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    a = rng.integers(lo, hi + 1, size=count)
    b = rng.integers(lo, hi + 1, size=count)
    return [(1 << int(x), 1 << int(y)) for x, y in zip(a, b)]


def batched_grids(seed, shapes):
    """One complex grid per shape; item ``i`` is drawn from seed ``[seed, i]``."""
    return [complex_grid([seed, i], s) for i, s in enumerate(shapes)]
