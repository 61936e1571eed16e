"""The FP64 oracle against its pins (CPU only), and the pins against planted mistakes."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    assert pin(oracle) == []


def test_gradient_finite_differences():
    """Gradient of sum |W * F x|^2 (batch 8 of 32x32, W real in [0,1)) against
    central differences in FP64. The loss is quadratic, so central differences
    are exact up to rounding for any step."""
    x = synth.complex_grid(6, (8, 32, 32)).astype(np.complex128)
    w = synth.real_weights(106, (32, 32))
    g = oracle.weighted_power_grad(x, w)
    rng = np.random.default_rng(7)
    h = 1e-3
    idx = [tuple(int(rng.integers(0, s)) for s in x.shape) for _ in range(24)]
    for i in idx:
        for unit in (1.0, 1j):
            xp = x.copy()
            xm = x.copy()
            xp[i] += h * unit
            xm[i] -= h * unit
            fd = (oracle.weighted_power_loss(xp, w) - oracle.weighted_power_loss(xm, w)) / (2 * h)
            an = g[i].real if unit == 1.0 else g[i].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (i, unit, fd, an)
    for _ in range(4):
        d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        fd = (oracle.weighted_power_loss(x + h * d, w) - oracle.weighted_power_loss(x - h * d, w)) / (2 * h)
        an = np.vdot(g, d).real
        assert abs(fd - an) <= 1e-9 * abs(an)


def test_complex64_promotion_is_exact():
    x = synth.complex_grid(3, (16, 32))
    a = oracle.fft2(x)
    b = oracle.fft2(x.astype(np.complex128))
    assert np.array_equal(a, b)


def test_batched_equals_loop():
    x = synth.complex_grid(4, (3, 8, 16))
    y = oracle.fft2(x)
    for i in range(3):
        assert np.array_equal(y[i], oracle.fft2(x[i]))


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft2(np.zeros((6, 8), np.complex64))


# ---------------------------------------------------------------- mutations
# Each entry plants one plausible mistake in a private copy of the oracle's C
# source; the pins must reject every mutant.
MUTATIONS = {
    "combine_sign": ("out[k + h] = e - t;", "out[k + h] = e + t;"),
    "twiddle_sign": ("w[j] = cos(a) + I * ((double)sign * sin(a));", "w[j] = cos(a) + I * (-(double)sign * sin(a));"),
    "twiddle_angle": ("double a = TWO_PI * (double)j / (double)n;", "double a = TWO_PI * (double)j / (double)(2 * n);"),
    "odd_half_dropped": ("rec(x + s, 2 * s, out + h, h, w_top, top_n);", "rec(x, 2 * s, out + h, h, w_top, top_n);"),
    "twiddle_stride": ("cplx t = w_top[k * step] * out[k + h];", "cplx t = w_top[k] * out[k + h];"),
    "listing_no_permute": ("  if (permute) {", "  if (0) {"),
    "listing_twiddle_index": ("int64_t q = spec << (last - s);", "int64_t q = spec;"),
    "listing_butterfly": ("re[b] = re[a] - fr;", "re[b] = re[a] + fr;"),
    "listing_cross_term": ("double fi = re[b] * ti + im[b] * tr;", "double fi = re[b] * ti - im[b] * tr;"),
    "no_scale": ("if (scale != 1.0)", "if (0)"),
    "direct_phase_transposed": ("int64_t p = (((k * m) % M) * N + ((l * n) % N) * M) % MN;",
                                "int64_t p = (((k * m) % M) * M + ((l * n) % N) * N) % MN;"),
    "column_pass_skipped": ("rec(col, 1, tmp, M, wM, M);", "memcpy(tmp, col, sizeof(cplx) * (size_t)M);"),
}


class _Mutant:
    """The oracle's Python surface bound to a mutated build of its C file."""

    def __init__(self, lib):
        self._lib = lib

    def __getattr__(self, name):
        fn = getattr(oracle, name)
        lib = self._lib

        def call(*a, **k):
            saved = oracle._lib
            oracle._lib = lib
            try:
                return fn(*a, **k)
            finally:
                oracle._lib = saved
        return call


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = open(oracle._SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, "mutation anchor not found once: %r" % old
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / ("mut_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(path), "-lm"],
                   check=True)
    mutant = _Mutant(oracle._bind(ctypes.CDLL(str(so))))
    fails = P.run_all(mutant, quick=True)
    assert fails, "planted mistake %s passed every pin" % name


# ------------------------------------------------------------ seeded inputs
def test_synth_reproducible_and_in_range():
    a = synth.complex_grid(1, (64, 32))
    b = synth.complex_grid(1, (64, 32))
    assert a.dtype == np.complex64 and a.shape == (64, 32)
    assert a.tobytes() == b.tobytes()
    v = a.view(np.float32)
    assert v.min() >= -1.0 and v.max() < 1.0
    # 2u - 1 is exact: every value is a multiple of 2**-23
    assert np.all(np.mod(v.astype(np.float64) * 2 ** 23, 1.0) == 0)
    w = synth.real_weights(105, (4, 4))
    assert w.dtype == np.float32 and w.min() >= 0 and w.max() < 1


def test_synth_shapes():
    shapes = synth.pow2_shapes(4, 512)
    assert len(shapes) == 512
    logs = np.log2(np.array(shapes))
    assert logs.min() == 6 and logs.max() == 11
    assert shapes == synth.pow2_shapes(4, 512)
