"""The plan's FP32 twiddle tables against FP64 values of the documented layout:
every entry must be its exact angle's cos/sin rounded once to FP32 (no
recurrence, which would drift by several units in the last place)."""

from __future__ import annotations

import re

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


def _radices(desc, which):
    part = re.search(r"%s\[L=\d+ radix=([0-9x]+)" % which, desc).group(1)
    return [int(r) for r in part.split("x")]


def _expected(radices):
    vals, ns = [], 1
    for p, R in enumerate(radices):
        if p > 0:
            for r in range(1, R):
                k = np.arange(ns, dtype=np.float64)
                vals.append(np.exp(-2j * np.pi * (k * r) / (ns * R)))
        ns *= R
    return np.concatenate(vals) if vals else np.zeros(0, np.complex128)


def _check_rounded_once(got, exact, what):
    ref32 = exact.astype(np.complex64)
    ulp = np.spacing(np.float32(1.0)) / 2  # half a unit in the last place at 1, an upper bound below 1
    err = np.maximum(np.abs(got.real.astype(np.float64) - exact.real), np.abs(got.imag.astype(np.float64) - exact.imag))
    same = np.mean((got == ref32))
    say("%s: %d entries, %.4f%% identical to FP64 rounded once, max error %.3g" % (what, got.size, 100 * same,
                                                                                  float(err.max(initial=0))))
    assert float(err.max(initial=0)) <= ulp * 1.0001
    assert same >= 0.999


@pytest.mark.parametrize("shape", [(4096, 4096), (1024, 16384), (64, 2048)], ids=lambda s: "%dx%d" % s)
def test_plan_twiddle_tables(F, shape):
    plan = F.Plan(1, *shape)
    try:
        desc = plan.describe()
        for which, name in ((0, "row"), (1, "col")):
            got = F.fft2d_plan_twiddles(plan.handle, which)
            exact = _expected(_radices(desc, name))
            assert got.size == exact.size, (name, got.size, exact.size)
            _check_rounded_once(got, exact, "%s %s table" % (shape, name))
        comb = F.fft2d_plan_twiddles(plan.handle, 2)
        if "split=1 " in desc:
            assert comb.size == 0
        else:
            M = shape[0]
            _check_rounded_once(comb, np.exp(-2j * np.pi * np.arange(M) / M), "%s combine table" % (shape,))
    finally:
        plan.close()
