"""GPU checks of the adjoint kernels behind torch.autograd (loss = sum |W * FFT2(x)|^2)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check, dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


def _loss(F, xd, wd, direction):
    y = F.fft2_diff(xd, direction)
    return (wd * wd * (y.real * y.real + y.imag * y.imag)).sum()


def test_gradient_8x2048x2048_vs_oracle(F):
    """Batch 8 of 2048 x 2048, W real uniform [0, 1) from seed 105, x from seed 5."""
    import torch
    say("case autograd 8x2048x2048")
    x = synth.complex_grid(5, (8, 2048, 2048))
    w = synth.real_weights(105, (2048, 2048))
    xd = dev(x).requires_grad_(True)
    wd = dev(w)
    loss = _loss(F, xd, wd, F.FORWARD)
    loss.backward()
    g = host(xd.grad)
    ref = oracle.weighted_power_grad(x, w)
    check(g, ref, "autograd 8x2048^2 gradient")
    del xd, loss
    torch.cuda.empty_cache()


@pytest.mark.parametrize("direction", [-1, 1])
def test_gradient_32x32_finite_differences(F, direction):
    """Batch 8 of 32 x 32 (x seed 6, W seed 106): the GPU gradient against FP64
    central differences of the oracle loss (exact for a quadratic loss), and
    against FP32 directional differences of the GPU loss itself."""
    import torch
    say("case autograd 8x32x32 direction %d" % direction)
    x = synth.complex_grid(6, (8, 32, 32))
    w = synth.real_weights(106, (32, 32))
    xd = dev(x).requires_grad_(True)
    wd = dev(w)
    _loss(F, xd, wd, direction).backward()
    g = host(xd.grad).astype(np.complex128)

    def oracle_loss(v):
        y = oracle.fft2(v, direction, 1.0 if direction == -1 else 1.0 / (32 * 32))
        return float(np.sum((w.astype(np.float64) * np.abs(y)) ** 2))

    x64 = x.astype(np.complex128)
    rng = np.random.default_rng(3)
    h = 0.25
    for _ in range(16):
        i = tuple(int(rng.integers(0, s)) for s in x.shape)
        for unit in (1.0, 1j):
            xp, xm = x64.copy(), x64.copy()
            xp[i] += h * unit
            xm[i] -= h * unit
            fd = (oracle_loss(xp) - oracle_loss(xm)) / (2 * h)
            an = g[i].real if unit == 1.0 else g[i].imag
            assert abs(fd - an) <= 1e-5 * max(1.0, float(np.max(np.abs(g)))), (i, unit, fd, an)
    # FP32 directional difference of the GPU loss
    d = synth.complex_grid(7, x.shape)
    dd = dev(d)
    with torch.no_grad():
        hh = 0.5
        lp = float(_loss(F, xd + hh * dd, wd, direction))
        lm = float(_loss(F, xd - hh * dd, wd, direction))
    fd = (lp - lm) / (2 * hh)
    an = float(np.vdot(g, d.astype(np.complex128)).real)
    say("directional fd=%.6e analytic=%.6e" % (fd, an))
    assert abs(fd - an) <= 1e-3 * abs(an)


def test_adjoint_identity_and_inverse_adjoint(F):
    """Re<F a, b> = Re<a, F^H b> through the C ABI, both directions, on a split plan size."""
    say("case adjoint identity")
    for shape, direction in (((256, 512), -1), ((256, 512), 1), ((4096, 1024), -1)):
        a = synth.complex_grid(21, shape)
        b = synth.complex_grid(22, shape)
        plan = F.get_plan(1, shape[0], shape[1], "cuda")
        fa = host(plan(dev(a), direction)).astype(np.complex128)
        fhb = host(plan.backward(dev(b), direction)).astype(np.complex128)
        lhs = np.vdot(b.astype(np.complex128), fa).real
        rhs = np.vdot(fhb, a.astype(np.complex128)).real
        say("adjoint %s dir %d: %.6e vs %.6e" % (shape, direction, lhs, rhs))
        assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1.0)
        check(fhb, oracle.adjoint(b, direction), "adjoint %s dir %d vs oracle" % (shape, direction))
