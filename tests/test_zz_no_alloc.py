"""fft2d_exec_noalloc (the allocation-free entry point, no plan) through the C
ABI, against fft2d_exec on a plan of the same shape: both bounds of
tests/gpu_util.py, on calls in a row with a smaller input second, out of
place and in place (the in-place split shapes use the library's device array
as work buffer), and its size limit."""

from __future__ import annotations

import pytest

import oracle
import synth
from tests.gpu_util import check, check_dev, dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


def _pair(F, batch, rows, cols, seed, direction, in_place):
    """(no-alloc result, fft2d_exec result, input) for one shape."""
    import torch
    shape = (batch, rows, cols) if batch > 1 else (rows, cols)
    x = dev(synth.complex_grid(seed, shape))
    s = int(torch.cuda.current_stream().cuda_stream)
    plan = F.Plan(batch, rows, cols)
    try:
        ref = torch.empty_like(x) if not in_place else x.clone()
        F.fft2d_exec(plan.handle, (ref if in_place else x).data_ptr(), ref.data_ptr(), direction, s)
        y = x.clone() if in_place else torch.empty_like(x)
        F.fft2d_exec_noalloc(batch, rows, cols, (y if in_place else x).data_ptr(), y.data_ptr(), direction, s)
        torch.cuda.synchronize()
        say("no-alloc %dx%dx%d dir %+d %s, plan %s" % (batch, rows, cols, direction,
                                                       "in place" if in_place else "out of place", plan.describe()))
    finally:
        plan.close()
    return y, ref, x


# (batch, rows, cols, seed, direction, in place), each followed by a smaller call
SEQUENCES = [
    [(1, 4096, 4096, 1, -1, False), (2, 256, 512, 2, +1, True)],      # split out of place, then plain in place
    [(2, 2048, 2048, 3, -1, True), (1, 2048, 2048, 4, +1, True)],     # split in place: the whole work buffer, then half
    [(37, 64, 64, 5, -1, False), (3, 32, 32, 6, +1, False)],          # whole-grid kernel
    [(1, 8192, 8192, 7, -1, False), (4096, 1, 1024, 8, -1, True)],    # 512 MiB split, then a batch of 1D rows
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "%dx%dx%d-then-%dx%dx%d" % (s[0][:3] + s[1][:3]))
def test_noalloc_matches_fft2d_exec(F, seq):
    for batch, rows, cols, seed, direction, in_place in seq:
        say("case no-alloc %dx%dx%d seed %d" % (batch, rows, cols, seed))
        y, ref, x = _pair(F, batch, rows, cols, seed, direction, in_place)
        check_dev(y, ref, "no-alloc vs fft2d_exec %dx%dx%d dir %+d" % (batch, rows, cols, direction))
        if batch * rows * cols <= (1 << 22):
            xh = host(x)
            want = oracle.fft2_forward(xh) if direction == -1 else oracle.ifft2(xh)
            check(host(y), want, "no-alloc vs oracle %dx%dx%d dir %+d" % (batch, rows, cols, direction))
        del y, ref, x


def test_noalloc_limits(F):
    """An in-place split call needing more than the 64 MiB work buffer is
    rejected before anything is enqueued (the output is untouched); the same
    shape out of place needs no work buffer and runs; bad arguments are
    rejected like fft2d_exec's."""
    import torch
    say("case no-alloc limits")
    s = int(torch.cuda.current_stream().cuda_stream)
    x = torch.zeros((3, 2048, 2048), dtype=torch.complex64, device="cuda")
    x[0, 0, 0] = 1.0
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec_noalloc(3, 2048, 2048, x.data_ptr(), x.data_ptr(), F.FORWARD, s)
    assert e.value.status == 2 and "work buffer" in str(e.value), str(e.value)
    torch.cuda.synchronize()
    assert float(x[0, 0, 0].real) == 1.0 and float(torch.abs(x).sum()) == 1.0
    y = torch.empty_like(x)
    F.fft2d_exec_noalloc(3, 2048, 2048, x.data_ptr(), y.data_ptr(), F.FORWARD, s)
    torch.cuda.synchronize()
    want = torch.zeros_like(y)
    want[0] = 1.0  # the delta's transform is all ones; the two zero grids stay zero
    check_dev(y, want, "no-alloc delta of 3x2048^2 out of place")
    for args, status in (((1, 3, 8), 2), ((0, 8, 8), 2), ((1, 8, 32768), 2)):
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_exec_noalloc(*args, x.data_ptr(), y.data_ptr(), F.FORWARD, s)
        assert e.value.status == status
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec_noalloc(1, 8, 8, x.data_ptr(), y.data_ptr(), 2, s)
    assert e.value.status == 3
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec_noalloc(1, 8, 8, x.data_ptr() + 4, y.data_ptr(), F.FORWARD, s)
    assert e.value.status == 4
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec_noalloc(1, 64, 64, x.data_ptr(), x.data_ptr() + 8, F.FORWARD, s)
    assert e.value.status == 9
