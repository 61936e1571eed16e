"""GPU parity of the whole-grid kernel (a small grid's 2D transform in one
launch) and of batches large enough to run as several launches, through the C
ABI, against the FP64 oracle (relative L2 and element-wise bounds of
tests/gpu_util.py per case)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check, dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

GRID_SHAPES = [(64, 64), (64, 128), (128, 64), (128, 128), (64, 256), (256, 64), (32, 32), (32, 64), (64, 32),
               (32, 128), (128, 32), (32, 256), (256, 32)]


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


def _two_pass(F, plan, xd, direction):
    """The same plan's row pass then column pass (two launches)."""
    import torch
    z = torch.empty_like(xd)
    s = int(torch.cuda.current_stream().cuda_stream)
    F.fft2d_exec_pass(plan.handle, xd.data_ptr(), z.data_ptr(), direction, 0, s)
    F.fft2d_exec_pass(plan.handle, z.data_ptr(), z.data_ptr(), direction, 1, s)
    return z


@pytest.mark.parametrize("batch", [1, 37])
@pytest.mark.parametrize("shape", GRID_SHAPES, ids=lambda s: "%dx%d" % s)
def test_whole_grid_kernel(F, shape, batch, monkeypatch):
    """Forward, inverse, in place and adjoint of grids on the one-launch path
    (forced, whatever the batch); the two-pass kernels of the same plan give
    the same result."""
    say("case whole-grid batch %d shape %dx%d" % ((batch,) + shape))
    monkeypatch.setenv("FFT2D_GRID", "on")
    x = synth.complex_grid(500 + batch + shape[0] + 3 * shape[1], (batch,) + shape)
    xd = dev(x)
    plan = F.Plan(batch, *shape)
    try:
        assert " grid[" in plan.describe(), plan.describe()
        for direction, ref in ((F.FORWARD, oracle.fft2_forward(x)), (F.INVERSE, oracle.ifft2(x))):
            y = host(plan(xd, direction))
            check(y, ref, "whole-grid b%d %dx%d dir %+d" % ((batch,) + shape + (direction,)))
            z = host(_two_pass(F, plan, xd, direction))
            diff = rel_l2(y, z)
            say("whole-grid b%d %dx%d dir %+d vs two-pass %.3e (bitwise equal: %s)" %
                ((batch,) + shape + (direction, diff, bool(np.array_equal(y, z)))))
            assert diff <= 1e-6, diff
            w = xd.clone()
            plan(w, direction, out=w)  # in place
            assert np.array_equal(host(w), y)
        g = plan.backward(xd, F.FORWARD)
        check(host(g), oracle.adjoint(x, oracle.FORWARD), "whole-grid b%d %dx%d adjoint" % ((batch,) + shape))
    finally:
        plan.close()


@pytest.mark.parametrize("shape,batch,expected", [((64, 64), 1, True), ((64, 128), 31, False),
                                                  ((64, 128), 32, True), ((128, 128), 127, False),
                                                  ((256, 64), 128, True), ((256, 256), 1000, False),
                                                  ((32, 32), 1, True), ((32, 256), 31, False), ((256, 32), 32, True),
                                                  ((16, 16), 1000, False), ((32, 512), 1000, False)])
def test_whole_grid_choice(F, shape, batch, expected, monkeypatch):
    """By default small batches of the larger grids keep the two passes."""
    say("case whole-grid choice b%d %dx%d" % ((batch,) + shape))
    monkeypatch.delenv("FFT2D_GRID", raising=False)
    plan = F.Plan(batch, *shape)
    try:
        assert (" grid[" in plan.describe()) == expected, plan.describe()
    finally:
        plan.close()


def test_whole_grid_switch_off(F, monkeypatch):
    """FFT2D_GRID=off keeps small grids on the two-pass path."""
    say("case whole-grid switched off")
    monkeypatch.setenv("FFT2D_GRID", "off")
    plan = F.Plan(2, 64, 64)
    try:
        assert " grid[" not in plan.describe(), plan.describe()
        x = synth.complex_grid(77, (2, 64, 64))
        check(host(plan(dev(x), F.FORWARD)), oracle.fft2_forward(x), "64x64 two-pass")
    finally:
        plan.close()


def _chunked_case(F, batch, rows, cols, seed, picks):
    """In-place forward transform of `batch` grids generated on the device;
    the grids at `picks` are checked against the oracle."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    x = torch.empty((batch, rows, cols), dtype=torch.complex64, device="cuda")
    x.view(torch.float32).uniform_(-1.0, 1.0, generator=gen)
    idx = torch.tensor(picks, dtype=torch.int64, device="cuda")
    before = host(x.index_select(0, idx))
    plan = F.Plan(batch, rows, cols)
    try:
        say("plan %s" % plan.describe())
        plan(x, F.FORWARD, out=x)
        after = host(x.index_select(0, idx))
    finally:
        plan.close()
        del x
        torch.cuda.empty_cache()
    check(after, oracle.fft2_forward(before), "chunked b%d %dx%d picks %s" % (batch, rows, cols, picks))


def test_chunked_whole_grid_batch(F):
    """2^19 + 3 grids of 64 x 64 (4 GiB): two launches of the whole-grid kernel."""
    say("case chunked 64x64 batch 2^19+3")
    b = (1 << 19) + 3
    _chunked_case(F, b, 64, 64, 11, [0, 1, (1 << 19) - 1, 1 << 19, b - 1])


def test_chunked_split_batch(F):
    """513 grids of 2048 x 2048 (16 GiB, split transform with its work buffer):
    two launches of each pass, the second at an offset into the work buffer."""
    say("case chunked 2048x2048 batch 513")
    _chunked_case(F, 513, 2048, 2048, 12, [0, 511, 512])


def test_batch_beyond_2_pow_32_work_items(F):
    """2^32 grids of 1 x 2 (2^33 points, 64 GiB in place): one launch would need
    2^32 work-items; the plan runs it as four."""
    say("case 2^32 grids of 1x2")
    b = 1 << 32
    _chunked_case(F, b, 1, 2, 13, [0, (1 << 30) - 1, 1 << 30, (3 << 30) + 5, b - 1])
