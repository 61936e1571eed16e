"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every comparison against the oracle applies two bounds (tests/gpu_util.py):
relative L2 over the whole output <= 1e-5 (FP32 against FP64), and every
element within 1e-5 of the reference's RMS magnitude; both measured errors are
printed for every case.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, check, check_dev, dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


def _check(F, x, direction, tag):
    y = host(F.fft2(dev(x)) if direction == -1 else F.ifft2(dev(x)))
    ref = oracle.fft2_forward(x) if direction == -1 else oracle.ifft2(x)
    err, _ = check(y, ref, tag)
    return y, err


def test_64x64_forward_vs_oracle_and_direct(F):
    say("case 64x64 forward seed 0")
    x = synth.complex_grid(0, (64, 64))
    y, _ = _check(F, x, -1, "64x64 fwd")
    direct = oracle.dft2d_direct(x.astype(np.complex128))
    check(y, direct, "64x64 vs direct DFT")


SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (4, 8), (8, 4), (16, 16), (32, 64), (64, 32), (128, 128), (256, 512),
          (512, 256), (1024, 64), (64, 1024), (2048, 32), (32, 2048), (4096, 8), (8, 4096), (8192, 4), (4, 8192),
          (16384, 2), (2, 16384), (1, 16384), (16384, 1), (1, 64), (64, 1), (1024, 1024)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_shapes_forward_inverse(F, shape):
    say("case shape %dx%d" % shape)
    x = synth.complex_grid(hash(shape) % 1000, shape)
    _check(F, x, -1, "%dx%d fwd" % shape)
    _check(F, x, +1, "%dx%d inv" % shape)


@pytest.mark.parametrize("batch,shape", [(3, (16, 64)), (5, (8, 256)), (7, (64, 16)), (3, (2, 2048)), (2, (128, 4096)),
                                         (3, (4096, 2)), (5, (1, 512)), (9, (32, 1))])
def test_ragged_batches(F, batch, shape):
    """Batches whose vector count leaves the last workgroup partly empty."""
    say("case batch %d shape %dx%d" % ((batch,) + shape))
    x = synth.complex_grid(batch, (batch,) + shape)
    _check(F, x, -1, "b%d %dx%d fwd" % ((batch,) + shape))
    _check(F, x, +1, "b%d %dx%d inv" % ((batch,) + shape))


def test_4096_round_trip(F):
    """4096 x 4096 forward + inverse (128 MiB), the plain path."""
    say("case 4096x4096 round trip seed 1")
    x = synth.complex_grid(1, (4096, 4096))
    xd = dev(x)
    yd = F.fft2(xd)
    y = host(yd)
    check(y, oracle.fft2_forward(x), "4096^2 fwd")
    zd = F.ifft2(yd)
    z = host(zd)
    check(z, x, "4096^2 round trip")
    check(z, oracle.ifft2(y), "4096^2 inv (of GPU fwd)")


@pytest.mark.parametrize("shape,seed", [((8192, 8192), 2), ((16384, 2048), 3)], ids=["8192x8192", "16384x2048"])
def test_large_forward(F, shape, seed):
    say("case %dx%d forward seed %d" % (shape + (seed,)))
    x = synth.complex_grid(seed, shape)
    _check(F, x, -1, "%dx%d fwd" % shape)


def test_maximum_grid_16384x16384(F):
    """The largest supported grid (2^14 per dimension, 2 GiB of complex64):
    forward against the full FP64 oracle, and the inverse round trip."""
    import torch
    say("case 16384x16384 forward + inverse")
    x = synth.complex_grid(9, (16384, 16384))
    xd = dev(x)
    plan = F.get_plan(1, 16384, 16384, "cuda")
    y = plan(xd, F.FORWARD)
    check(host(y), oracle.fft2_forward(x), "16384x16384 fwd")
    z = plan(y, F.INVERSE)
    check_dev(z, xd, "16384x16384 round trip")
    del xd, y, z
    torch.cuda.empty_cache()


def test_1d_batch_4096_rows_of_16384(F):
    """rows = 1: a batch of 4096 one-dimensional length-16384 transforms (the
    paper's single-core FFT length, Section 4), forward and inverse; every row
    against the FP64 oracle (whole output and row by row), all rows against
    Parseval."""
    import torch
    say("case 1D batch 4096 x 16384")
    x = synth.complex_grid(0, (4096, 1, 16384))
    plan = F.get_plan(4096, 1, 16384, "cuda")
    xd = dev(x)
    y = plan(xd, F.FORWARD)
    z = plan(y, F.INVERSE)
    torch.cuda.synchronize()
    yh = host(y)
    ref = oracle.fft2_forward(x)
    check(yh, ref, "1D batch 4096x16384 fwd, all rows")
    # row by row: the worst row's relative L2 and element error against its own RMS
    d = np.abs(yh.astype(np.complex128) - ref)[:, 0, :]
    rms = np.sqrt(np.mean(np.abs(ref[:, 0, :]) ** 2, axis=1))
    row_rel = np.sqrt(np.mean(d ** 2, axis=1)) / rms
    row_max = d.max(axis=1) / rms
    say("1D rows: worst row rel_l2=%.3e worst row max_elem=%.3e" % (row_rel.max(), row_max.max()))
    assert row_rel.max() <= TOL and row_max.max() <= TOL
    del ref, d
    lhs = torch.sum(torch.abs(y.to(torch.complex128)) ** 2, dim=(1, 2))
    rhs = 16384 * torch.sum(torch.abs(xd.to(torch.complex128)) ** 2, dim=(1, 2))
    parseval = float(torch.max(torch.abs(lhs - rhs) / rhs))
    say("1D batch 4096x16384 parseval=%.2e" % parseval)
    assert parseval <= 1e-5
    check_dev(z, xd, "1D batch 4096x16384 round trip")


@pytest.mark.parametrize("shape", [(64, 64), (256, 512), (4096, 1024)], ids=["64x64-whole-grid", "256x512",
                                                                          "4096x1024-split"])
def test_exec_captured_in_hip_graph(F, shape):
    """fft2d_exec enqueues kernels only, so it can be captured in a HIP graph
    (torch.cuda.CUDAGraph); every replay, with eager work between replays,
    equals the eager result bit for bit."""
    import torch
    say("case HIP graph capture %dx%d" % shape)
    x = dev(synth.complex_grid(31, shape))
    y = torch.empty_like(x)
    plan = F.get_plan(1, shape[0], shape[1], "cuda")
    eager = plan(x, F.FORWARD)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.exec_ptr(x.data_ptr(), y.data_ptr(), F.FORWARD, torch.cuda.current_stream().cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), rep
        other = plan(x, F.INVERSE)  # eager work between replays
        torch.cuda.synchronize()
        del other
    check(host(y), oracle.fft2_forward(host(x)), "graph replay %dx%d" % shape)
    del g


def test_in_place_matches_out_of_place_and_is_deterministic(F):
    import torch
    say("case in-place 512x1024")
    x = synth.complex_grid(8, (512, 1024))
    a = F.fft2(dev(x))
    b = F.fft2(dev(x))
    c = dev(x)
    F.fft2(c, out=c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, c)


def test_rejects_bad_tensors(F):
    import torch
    with pytest.raises(TypeError):
        F.fft2(torch.zeros(8, 8, dtype=torch.complex128, device="cuda"))
    with pytest.raises(TypeError):
        F.fft2(torch.zeros(8, 8, dtype=torch.complex64))
    with pytest.raises(ValueError):
        F.fft2(torch.zeros(6, 8, dtype=torch.complex64, device="cuda"))


def test_abi_errors_on_device_pointers(F):
    import torch
    say("case ABI errors")
    x = torch.zeros(4, 64, 64, dtype=torch.complex64, device="cuda")
    p = F.get_plan(4, 64, 64, x.device)
    base = x.data_ptr()
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec(p.handle, base + 4, base + 4, -1, 0)
    assert e.value.status == 4
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec(p.handle, base, base + 8 * 64, -1, 0)
    assert e.value.status == 9
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec(p.handle, base, base, 2, 0)
    assert e.value.status == 3
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec_batched(p.handle, [base], [base], -1, 0)
    assert e.value.status == 5
    q = F.fft2d_plan(1, 8, 8)
    F.fft2d_destroy(q)
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_exec(q, base, base, -1, 0)
    assert e.value.status == 8
    assert "C=" in p.describe()


# Split column transforms (row pass with an M1-point combine + column pass of
# length rows/M1), forced at sizes the oracle handles in well under a second.
SPLIT_CASES = [(1, (32, 1024), 16), (2, (64, 1024), 16), (1, (256, 2048), 8), (3, (64, 2048), 8),
               (1, (512, 4096), 4), (2, (128, 4096), 4), (1, (64, 8192), 2), (1, (64, 8192), 4),
               (2, (32, 8192), 4), (1, (2048, 1024), 16),
               (1, (8192, 2048), 8), (1, (64, 16384), 2), (2, (32, 16384), 2)]


@pytest.mark.parametrize("combine", ["xrow", "xrow-narrow", "classic"])
@pytest.mark.parametrize("batch,shape,m1", SPLIT_CASES, ids=lambda v: str(v))
def test_split_transform(F, batch, shape, m1, combine, monkeypatch):
    """Forward, inverse, adjoint and in-place split transforms against the
    oracle, with every row pass with combine: the last FFT stage across the
    workgroup's rows (xrow, the default where it exists; with few tiles and
    4096-point rows its 64-points-per-thread form, xrow-narrow forcing the
    32-point one) and the separate combine exchange (classic)."""
    say("case split batch %d shape %dx%d m1 %d %s" % ((batch,) + shape + (m1, combine)))
    monkeypatch.setenv("FFT2D_SPLIT", str(m1))
    monkeypatch.setenv("FFT2D_COMBINE", combine.split("-")[0])
    monkeypatch.setenv("FFT2D_COMBINE_WIDE", "off" if combine == "xrow-narrow" else "auto")
    plan = F.Plan(batch, *shape)
    try:
        desc = plan.describe()
        assert ("split=%d " % m1) in desc, desc
        if combine == "classic":
            assert " combine]" in desc, desc
        if combine == "xrow-narrow":
            assert " E=64 " not in desc.split("col[")[0], desc
        x = synth.complex_grid(m1 + batch, (batch,) + shape)
        xd = dev(x)
        y = host(plan(xd, F.FORWARD))
        check(y, oracle.fft2_forward(x), "split fwd")
        z = host(plan(xd, F.INVERSE))
        check(z, oracle.ifft2(x), "split inv")
        g = host(plan.backward(xd, F.FORWARD))
        check(g, oracle.adjoint(x, -1), "split adjoint")
        # in place through the work buffer: the same kernels, so the same result
        w = dev(x)
        plan(w, F.FORWARD, out=w)
        assert np.array_equal(host(w), y)
    finally:
        plan.close()


def test_auto_split_choice(F):
    say("case auto split choice")
    import os
    assert os.environ.get("FFT2D_SPLIT") is None
    p = F.Plan(1, 4096, 4096)
    q = F.Plan(1, 64, 64)
    r = F.Plan(1, 8192, 8192)
    u = F.Plan(1, 4096, 16384)
    v = F.Plan(1, 2048, 16384)  # split from 2048 rows
    w = F.Plan(1, 1024, 16384)
    try:
        assert "split=1 " in w.describe(), w.describe()
        assert "split=2 " in u.describe(), u.describe()
        assert "split=2 " in v.describe(), v.describe()
        assert "split=4 " in p.describe(), p.describe()
        assert "split=1 " in q.describe(), q.describe()
        assert "split=4 " in r.describe(), r.describe()
        assert " E=64 " in r.describe().split("col[")[1], r.describe()  # 8192 columns: wide column pass
    finally:
        p.close()
        q.close()
        r.close()
        u.close()
        v.close()
        w.close()


@pytest.mark.parametrize("shape,mode,col_e", [((8192, 4096), "auto", 64), ((8192, 4096), "narrow", 32),
                                              ((16384, 4096), "auto", 64), ((16384, 4096), "narrow", 32),
                                              ((16384, 2048), "auto", 64), ((4096, 16384), "auto", 64)],
                         ids=lambda v: str(v))
def test_split_column_kernel_width(F, shape, mode, col_e, monkeypatch):
    """Split plans' column passes of length 2048 and 4096 with 64 points per
    thread (the default) and with 32, against the oracle (forward and
    inverse)."""
    say("case split column width %dx%d %s" % (shape + (mode,)))
    if mode == "auto":
        monkeypatch.delenv("FFT2D_SPLIT_COLUMN", raising=False)
    else:
        monkeypatch.setenv("FFT2D_SPLIT_COLUMN", mode)
    plan = F.Plan(1, *shape)
    try:
        desc = plan.describe()
        say(desc)
        col = desc[desc.index("col["):]
        assert ("E=%d " % col_e) in col, desc
        x = synth.complex_grid(40 + shape[1] // 1024, shape)
        xd = dev(x)
        check(host(plan(xd, F.FORWARD)), oracle.fft2_forward(x), "split column E=%d %dx%d fwd" % ((col_e,) + shape))
        check(host(plan(xd, F.INVERSE)), oracle.ifft2(x), "split column E=%d %dx%d inv" % ((col_e,) + shape))
    finally:
        plan.close()


@pytest.mark.parametrize("shape,stages", [((4096, 4096), "two"), ((2, 4096, 4096), "two"), ((8192, 2048), "two"),
                                          ((8192, 8192), "two"), ((16384, 2048), "two"),
                                          ((16384, 2048), "classic"), ((8192, 8192), "classic"),
                                          ((4096, 4096), "two-nt"), ((8192, 8192), "two-plain")],
                         ids=lambda v: str(v))
def test_split_column_stages(F, shape, stages, monkeypatch):
    """Split plans whose column pass runs a two-stage radix schedule (32 x 32
    for 1024-point columns, 64 x 32 for 2048-point columns: one LDS exchange;
    the default; with nontemporal loads forced on or off) and three stages
    (classic), forward and inverse, against the oracle."""
    say("case split column stages %s %s" % (shape, stages))
    monkeypatch.setenv("FFT2D_COLUMN_STAGES", stages.split("-")[0])
    if "-" in stages:  # nontemporal column loads forced on (two-nt) or off (two-plain)
        monkeypatch.setenv("FFT2D_COLUMN_NT", "on" if stages.endswith("nt") else "off")
    batch, rows, cols = (1,) + shape if len(shape) == 2 else shape
    plan = F.Plan(batch, rows, cols)
    try:
        desc = plan.describe()
        say(desc)
        col = desc[desc.index("col["):]
        assert ("radix=32x32 " in col or "radix=64x32 " in col) == stages.startswith("two"), desc
        if "-" in stages:
            assert (" nt" in col) == stages.endswith("nt"), desc
        x = synth.complex_grid(50 + cols // 1024, (batch, rows, cols) if batch > 1 else (rows, cols))
        xd = dev(x)
        check(host(plan(xd, F.FORWARD)), oracle.fft2_forward(x), "column stages %s %s fwd" % (stages, shape))
        check(host(plan(xd, F.INVERSE)), oracle.ifft2(x), "column stages %s %s inv" % (stages, shape))
    finally:
        plan.close()


@pytest.mark.parametrize("mode", ["on", "off"])
@pytest.mark.parametrize("shape", [(1024, 1024), (512, 1024), (3, 1, 1024), (4096, 1024)], ids=lambda v: str(v))
def test_row_wave_shuffle(F, shape, mode, monkeypatch):
    """The 1024-point row pass with one row per wave, its second exchange in
    registers across the wave's 16-lane rows (v_permlane32_swap and
    v_permlane16_swap; on, the default) or through the LDS (off), forward and
    inverse, against the oracle."""
    say("case row wave shuffle %s %s" % (shape, mode))
    monkeypatch.setenv("FFT2D_ROW_SHUFFLE", mode)
    monkeypatch.setenv("FFT2D_FEW_TILES", "on")
    monkeypatch.setenv("FFT2D_SPLIT", "off")
    batch, rows, cols = (1,) + shape if len(shape) == 2 else shape
    plan = F.Plan(batch, rows, cols)
    try:
        desc = plan.describe()
        say(desc)
        assert (" shuffle" in desc[desc.index("row["):desc.index("col[")]) == (mode == "on"), desc
        x = synth.complex_grid(60 + rows // 256, (batch, rows, cols) if batch > 1 else (rows, cols))
        xd = dev(x)
        check(host(plan(xd, F.FORWARD)), oracle.fft2_forward(x), "row shuffle %s fwd" % (shape,))
        check(host(plan(xd, F.INVERSE)), oracle.ifft2(x), "row shuffle %s inv" % (shape,))
    finally:
        plan.close()


@pytest.mark.parametrize("shape", [(1024, 1024), (512, 512), (2048, 1024)], ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("mode", ["auto", "off"])
def test_few_tiles_column_kernel(F, shape, mode, monkeypatch):
    """Passes with few tiles use narrower tiles by default (4-8 columns; one
    row of 1024); both kernels against the oracle."""
    say("case few-tiles column kernel %dx%d %s" % (shape + (mode,)))
    if mode == "auto":
        monkeypatch.delenv("FFT2D_FEW_TILES", raising=False)
    else:
        monkeypatch.setenv("FFT2D_FEW_TILES", mode)
    plan = F.Plan(1, *shape)
    try:
        desc = plan.describe()
        col = desc[desc.index("col["):]
        narrow = (" C=4 " in col) or (" C=8 " in col and shape[0] == 512)
        assert narrow == (mode == "auto"), desc
        if shape == (1024, 1024):  # 256 row tiles of 4 rows: one row per tile instead
            row = desc[desc.index("row["):desc.index("col[")]
            assert (" C=1 " in row) == (mode == "auto"), desc
        x = synth.complex_grid(60 + shape[0] // 512, shape)
        xd = dev(x)
        check(host(plan(xd, F.FORWARD)), oracle.fft2_forward(x), "few-tiles %s %dx%d fwd" % ((mode,) + shape))
        check(host(plan(xd, F.INVERSE)), oracle.ifft2(x), "few-tiles %s %dx%d inv" % ((mode,) + shape))
    finally:
        plan.close()


@pytest.mark.parametrize("shape", [(4096, 1024), (1024, 4096)], ids=lambda s: "%dx%d" % s)
def test_exec_pass_split_plan(F, shape):
    """fft2d_exec_pass 0 then 1 with the same arguments equals fft2d_exec, for a
    split plan called out of place (the intermediate lives in the output) and
    in place (it goes through the plan's work buffer)."""
    import torch
    say("case exec_pass split %dx%d" % shape)
    x = dev(synth.complex_grid(70, shape))
    plan = F.Plan(1, *shape)
    try:
        assert "split=1 " not in plan.describe(), plan.describe()
        s = int(torch.cuda.current_stream().cuda_stream)
        ref = plan(x, F.FORWARD)
        y = torch.empty_like(x)
        F.fft2d_exec_pass(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, 0, s)
        F.fft2d_exec_pass(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, 1, s)
        w = x.clone()
        F.fft2d_exec_pass(plan.handle, w.data_ptr(), w.data_ptr(), F.FORWARD, 0, s)
        F.fft2d_exec_pass(plan.handle, w.data_ptr(), w.data_ptr(), F.FORWARD, 1, s)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        assert torch.equal(w, ref)
        check(host(ref), oracle.fft2_forward(host(x)), "exec_pass split %dx%d" % shape)
    finally:
        plan.close()


@pytest.mark.parametrize("shape", [(4096, 4096), (64, 2048), (1024, 1024), (64, 64)], ids=lambda s: "%dx%d" % s)
def test_exec_pass_timed(F, shape):
    """fft2d_exec_pass_timed gives the same results as fft2d_exec_pass, bit for
    bit (a split plan, a plain one, one with narrow few-tile passes and a
    whole-grid plan, whose passes run as two launches here), within the FP32
    tolerance of the FP64 oracle, and its events, bound to the pass's kernel,
    span a positive time no longer than events recorded around the same
    launch."""
    import torch
    say("case exec_pass_timed %dx%d" % shape)
    x_h = synth.complex_grid(71, shape)
    x = dev(x_h)
    plan = F.Plan(1, *shape)
    try:
        stream = torch.cuda.current_stream()
        s = int(stream.cuda_stream)
        ref = torch.empty_like(x)
        F.fft2d_exec_pass(plan.handle, x.data_ptr(), ref.data_ptr(), F.FORWARD, 0, s)
        F.fft2d_exec_pass(plan.handle, x.data_ptr(), ref.data_ptr(), F.FORWARD, 1, s)
        y = torch.empty_like(x)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
        for e in ev:
            e.record(stream)
        torch.cuda.synchronize()
        kernel_ms, outer_ms = [], []
        for index in (0, 1):
            a, b, outer_a, outer_b = ev[4 * index:4 * index + 4]
            outer_a.record(stream)
            F.fft2d_exec_pass_timed(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, index,
                                    a.cuda_event, b.cuda_event, s)
            outer_b.record(stream)
            torch.cuda.synchronize()
            kernel_ms.append(a.elapsed_time(b))
            outer_ms.append(outer_a.elapsed_time(outer_b))
        assert torch.equal(y, ref)
        check(host(y), oracle.fft2_forward(x_h), "exec_pass_timed %dx%d" % shape)
        say("exec_pass_timed %dx%d kernel ms %s, between outer markers %s" % (shape + (kernel_ms, outer_ms)))
        for k, o in zip(kernel_ms, outer_ms):
            assert 0.0 < k <= o * 1.02 + 1e-3
        with pytest.raises(F.Fft2dError):
            F.fft2d_exec_pass_timed(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, 0, 0, ev[1].cuda_event, s)
    finally:
        plan.close()


@pytest.mark.parametrize("shape", [(4096, 4096), (256, 2048), (2, 8, 16384)], ids=lambda s: "x".join(map(str, s)))
def test_agrees_with_torch_fft2(F, shape):
    """Secondary FP32 sanity check: the library's forward and inverse agree with
    torch.fft.fft2 / ifft2 (the vendor FFT under torch, default norm: forward
    unscaled, inverse 1/(M N)) within the FP32 tolerance."""
    import torch
    say("case torch.fft %s" % (shape,))
    x = dev(synth.complex_grid(72, shape))
    for direction, ref in ((F.FORWARD, torch.fft.fft2(x)), (F.INVERSE, torch.fft.ifft2(x))):
        y = F.fft2(x) if direction == F.FORWARD else F.ifft2(x)
        check_dev(y, ref, "torch.fft %s dir %+d" % (shape, direction))
