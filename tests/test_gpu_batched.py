"""GPU parity of the batched path: many shapes, one persistent launch, HIP graph.

Every output is held to both bounds of tests/gpu_util.py (relative L2 and
element-wise against the FP64 oracle); the worst of each is printed."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, dev, errors, errors_dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


@pytest.fixture(autouse=True)
def _tune_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("FFT2D_TUNE_CACHE", str(tmp_path / "tune.txt"))
    # every transform in the persistent kernel unless a test says otherwise (large grids of a
    # plan would otherwise run as plain transforms and bypass the kernel paths under test)
    monkeypatch.setenv("FFT2D_BATCH_PLAIN", "off")


# every length 1 ... 2048 appears as rows and as cols, plus degenerate 1 x 1
MIXED = [(1, 1), (1, 2), (2, 1), (4, 8), (8, 4), (16, 32), (32, 16), (64, 64), (1, 512), (512, 1), (128, 256),
         (256, 128), (1024, 16), (16, 1024), (2048, 8), (8, 2048), (64, 2048), (2048, 64), (512, 512), (2, 4096),
         (4096, 2), (16384, 1), (1, 16384), (8192, 4), (4, 8192), (16384, 2)]


class Worst:
    """Largest relative L2 and element error over many outputs; asserts both bounds per output."""

    def __init__(self, tag):
        self.tag, self.rel, self.elem = tag, 0.0, 0.0

    def add(self, y, ref, what):
        rel, mx = errors(y, ref)
        self.rel, self.elem = max(self.rel, rel), max(self.elem, mx)
        assert rel <= TOL and mx <= TOL, (self.tag, what, rel, mx)

    def report(self):
        say("%s worst rel_l2=%.3e worst max_elem=%.3e" % (self.tag, self.rel, self.elem))


def _run(F, plan, xs, direction, outs=None):
    ins = [dev(x) for x in xs]
    res = plan(ins, direction, outs)
    return ins, res


@pytest.mark.parametrize("tune,sync,guided", [("off", "auto", "0"), ("full", "auto", "0"), ("off", "fenced", "0"),
                                               ("off", "auto", "1"), ("full", "auto", "1")])
def test_batched_mixed_shapes(F, tune, sync, guided, monkeypatch):
    """Forward and inverse of every length 1 .. 16384 as rows and as columns;
    sync "fenced" forces the single-queue path with agent-scope release / acquire;
    guided "1" groups the work in large units first (merged tile runs)."""
    monkeypatch.setenv("FFT2D_TUNE", tune)
    monkeypatch.setenv("FFT2D_BATCH_SYNC", sync)
    monkeypatch.setenv("FFT2D_BATCH_GUIDED", guided)
    say("case batched mixed shapes tune=%s sync=%s guided=%s" % (tune, sync, guided))
    xs = synth.batched_grids(11, MIXED)
    plan = F.BatchedPlan(MIXED)
    try:
        say(plan.describe())
        assert ("fenced" in plan.describe()) == (sync == "fenced")
        assert (" guided " in plan.describe()) == (guided == "1")
        _, ys = _run(F, plan, xs, F.FORWARD)
        _, zs = _run(F, plan, xs, F.INVERSE)
        wf, wi = Worst("batched mixed fwd"), Worst("batched mixed inv")
        for x, y, z, s in zip(xs, ys, zs, MIXED):
            wf.add(host(y), oracle.fft2_forward(x), s)
            wi.add(host(z), oracle.ifft2(x), s)
        wf.report()
        wi.report()
    finally:
        plan.close()


# tall transforms: split (row pass with combine + short columns) where a
# combine configuration exists for the row length, plain otherwise
SPLIT_SHAPES = [(2048, 512), (2048, 1024), (2048, 2048), (2048, 4096), (2048, 8192), (4096, 1024), (8192, 2048),
                (16384, 512), (4096, 8192), (2048, 256), (32, 32)]
SPLIT_EXPECTED = 8  # the first eight are split


@pytest.mark.parametrize("split,guided", [("auto", "0"), ("off", "0"), ("auto", "1")])
def test_batched_split_transforms(F, split, guided, monkeypatch):
    """Forward, inverse, in place and half in place for tall grids in one plan,
    split (row pass with an M1-point combine, columns of M / M1) or not, with
    fixed or guided work groups."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.setenv("FFT2D_BATCH_SPLIT", split)
    monkeypatch.setenv("FFT2D_BATCH_GUIDED", guided)
    say("case batched split=%s guided=%s" % (split, guided))
    xs = synth.batched_grids(14, SPLIT_SHAPES)
    plan = F.BatchedPlan(SPLIT_SHAPES)
    try:
        desc = plan.describe()
        say(desc)
        assert (" split=%d " % (SPLIT_EXPECTED if split == "auto" else 0)) in desc, desc
        ins, ys = _run(F, plan, xs, F.FORWARD)
        _, zs = _run(F, plan, xs, F.INVERSE)
        wf, wi = Worst("batched split=%s fwd" % split), Worst("batched split=%s inv" % split)
        for x, y, z, s in zip(xs, ys, zs, SPLIT_SHAPES):
            wf.add(host(y), oracle.fft2_forward(x), s)
            wi.add(host(z), oracle.ifft2(x), s)
        wf.report()
        wi.report()
        inplace = [t.clone() for t in ins]
        plan(inplace, F.FORWARD, inplace)
        torch.cuda.synchronize()
        for u, v in zip(ys, inplace):
            assert torch.equal(u, v)
        # every other transform in place (per-transform pointers)
        mixed_in = [t.clone() for t in ins]
        mixed_out = [t if k % 2 == 0 else torch.empty_like(t) for k, t in enumerate(mixed_in)]
        plan(mixed_in, F.FORWARD, mixed_out)
        torch.cuda.synchronize()
        for u, v in zip(ys, mixed_out):
            assert torch.equal(u, v)
    finally:
        plan.close()


@pytest.mark.parametrize("whole", ["auto", "off"])
def test_batched_whole_grid_items(F, whole, monkeypatch):
    """Grids of 64 x 64 ... 128 x 128, 64 x 256 and 256 x 64 run as one item each
    (one pass through HBM) unless FFT2D_BATCH_GRID=off; forward, inverse and in
    place match the oracle."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.setenv("FFT2D_BATCH_GRID", whole)
    shapes = [(64, 64), (64, 128), (128, 64), (64, 64), (128, 128), (32, 64), (64, 256), (256, 64), (256, 128)] * 2
    say("case batched whole-grid items %s" % whole)
    xs = synth.batched_grids(15, shapes)
    plan = F.BatchedPlan(shapes)
    try:
        desc = plan.describe()
        say(desc)
        assert (" whole=%d " % (14 if whole == "auto" else 0)) in desc, desc
        ins, ys = _run(F, plan, xs, F.FORWARD)
        _, zs = _run(F, plan, xs, F.INVERSE)
        wf, wi = Worst("batched whole=%s fwd" % whole), Worst("batched whole=%s inv" % whole)
        for x, y, z, s in zip(xs, ys, zs, shapes):
            wf.add(host(y), oracle.fft2_forward(x), s)
            wi.add(host(z), oracle.ifft2(x), s)
        wf.report()
        wi.report()
        inplace = [t.clone() for t in ins]
        plan(inplace, F.FORWARD, inplace)
        torch.cuda.synchronize()
        for u, v in zip(ys, inplace):
            assert torch.equal(u, v)
    finally:
        plan.close()


def test_batched_replay_pointer_change_and_in_place(F, monkeypatch):
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    shapes = [(64, 128), (256, 64), (32, 32), (1024, 256)]
    say("case batched replay / pointer change")
    xs = synth.batched_grids(12, shapes)
    plan = F.BatchedPlan(shapes)
    try:
        ins = [dev(x) for x in xs]
        a = plan(ins, F.FORWARD)
        b = plan(ins, F.FORWARD)  # graph replay, same pointers
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert torch.equal(u, v)
        outs = [torch.empty_like(t) for t in ins]  # new output pointers
        c = plan(ins, F.FORWARD, outs)
        torch.cuda.synchronize()
        for u, v in zip(a, c):
            assert torch.equal(u, v)
        inplace = [t.clone() for t in ins]
        plan(inplace, F.FORWARD, inplace)
        for u, v in zip(a, inplace):
            assert torch.equal(u, v)
        w = Worst("batched replay")
        for x, u, s in zip(xs, a, shapes):
            w.add(host(u), oracle.fft2_forward(x), s)
        w.report()
    finally:
        plan.close()


def test_batched_rejects_bad_input(F, monkeypatch):
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    plan = F.BatchedPlan([(8, 8), (16, 16)])
    try:
        a = torch.zeros(8, 8, dtype=torch.complex64, device="cuda")
        b = torch.zeros(16, 16, dtype=torch.complex64, device="cuda")
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_exec_batched(plan.handle, [a.data_ptr(), b.data_ptr() + 4], [a.data_ptr(), b.data_ptr()], -1, 0)
        assert e.value.status == 4
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_exec_batched(plan.handle, [a.data_ptr(), b.data_ptr()], [a.data_ptr(), b.data_ptr() + 8], -1, 0)
        assert e.value.status == 9
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_exec(plan.handle, a.data_ptr(), a.data_ptr(), -1, 0)
        assert e.value.status == 5
        with pytest.raises(ValueError):
            plan([a], F.FORWARD)
        with pytest.raises(ValueError):
            plan([a, b], F.FORWARD, [a])  # too few outputs
        with pytest.raises(ValueError):
            plan([a, b], F.FORWARD, [a, a])  # an output of the wrong shape
    finally:
        plan.close()


def test_batched_512_uneven_shapes(F):
    """512 transforms of 2^a x 2^b, a, b in [6, 11] drawn from seed 4, one persistent launch.

    Every output is checked against the FP64 oracle, against the plain path
    (fft2d_exec of the same shape) on the GPU, and against Parseval."""
    import torch
    shapes = synth.pow2_shapes(4, 512)
    say("case batched 512 shapes, %d points" % sum(r * c for r, c in shapes))
    xs = synth.batched_grids(4, shapes)
    plan = F.BatchedPlan(shapes)
    try:
        say(plan.describe())
        ins = [dev(x) for x in xs]
        ys = plan(ins, F.FORWARD)
        torch.cuda.synchronize()
        worst_plain = [0.0, 0.0]
        for x_d, y in zip(ins, ys):
            ref = F.fft2(x_d)
            rel, mx = errors_dev(y, ref)
            worst_plain = [max(worst_plain[0], rel), max(worst_plain[1], mx)]
            # Parseval: sum |Y|^2 = M N sum |x|^2
            m, n = x_d.shape
            lhs = float(torch.sum(torch.abs(y.to(torch.complex128)) ** 2))
            rhs = m * n * float(torch.sum(torch.abs(x_d.to(torch.complex128)) ** 2))
            assert abs(lhs - rhs) <= 1e-5 * rhs
        say("batched 512 vs plain path worst rel_l2=%.3e worst max_elem=%.3e" % tuple(worst_plain))
        assert worst_plain[0] <= 2 * TOL and worst_plain[1] <= 2 * TOL
        w = Worst("batched 512 all vs oracle")
        for i in range(len(shapes)):
            w.add(host(ys[i]), oracle.fft2_forward(xs[i]), (i, shapes[i]))
        w.report()
    finally:
        plan.close()


def test_batched_gave_up_wait_is_reported(F, monkeypatch):
    """Every column wait is told by the host to give up at once (spin limit -1):
    the launch still drains, and the next call reports FFT2D_ERR_INCOMPLETE once."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.setenv("FFT2D_BATCH_SPIN_LIMIT", "-1")
    shapes = [(64, 64), (256, 128)]
    say("case batched forced give-up")
    xs = [dev(x) for x in synth.batched_grids(13, shapes)]
    plan = F.BatchedPlan(shapes)
    try:
        plan(xs, F.FORWARD)
        torch.cuda.synchronize()
        with pytest.raises(F.Fft2dError) as e:
            plan(xs, F.FORWARD)
        assert e.value.status == 10
        torch.cuda.synchronize()
    finally:
        plan.close()
    monkeypatch.setenv("FFT2D_BATCH_SPIN_LIMIT", str(1 << 24))
    plan = F.BatchedPlan(shapes)
    try:
        ys = plan(xs, F.FORWARD)
        ys = plan(xs, F.FORWARD)  # no error is left over from the other plan
        w = Worst("batched after give-up")
        for x, y, s in zip(xs, ys, shapes):
            w.add(host(y), oracle.fft2_forward(host(x)), s)
        w.report()
    finally:
        plan.close()


def test_batched_undrained_queue_is_reported(F, monkeypatch):
    """The end-of-launch drain check: told by the host to expect more pops per
    queue than any launch makes (FFT2D_BATCH_DRAIN_SLACK), it reports an
    undrained queue, and the next call returns FFT2D_ERR_INCOMPLETE once; with
    the default (0) a full launch reports nothing, over several calls."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    shapes = [(64, 64), (256, 128), (2048, 1024), (16, 4096)]
    say("case batched drain check")
    xs_h = synth.batched_grids(16, shapes)
    xs = [dev(x) for x in xs_h]
    monkeypatch.setenv("FFT2D_BATCH_DRAIN_SLACK", str(1 << 20))
    plan = F.BatchedPlan(shapes)
    try:
        plan(xs, F.FORWARD)
        torch.cuda.synchronize()
        with pytest.raises(F.Fft2dError) as e:
            plan(xs, F.FORWARD)
        assert e.value.status == 10 and "undrained" in str(e.value), str(e.value)
        torch.cuda.synchronize()
    finally:
        plan.close()
    monkeypatch.delenv("FFT2D_BATCH_DRAIN_SLACK")
    plan = F.BatchedPlan(shapes)
    try:
        for _ in range(4):
            ys = plan(xs, F.FORWARD)
            torch.cuda.synchronize()
        w = Worst("batched after drain checks")
        for x, y, s in zip(xs_h, ys, shapes):
            w.add(host(y), oracle.fft2_forward(x), s)
        w.report()
    finally:
        plan.close()


# every row and column length 32 ... 16384 that has two radix/tile variants, with partly filled tiles,
# plus split transforms (their column lengths take variants too)
VARIANT_SHAPES = [(4, 32), (32, 4), (8, 64), (64, 8), (16, 128), (128, 16), (8, 256), (256, 8), (4, 512),
                  (512, 4), (2, 1024), (1024, 2), (2, 2048), (2048, 2), (2, 4096), (4096, 2), (2, 8192),
                  (8192, 2), (1, 16384), (16384, 1), (2048, 1024), (1024, 512), (64, 64)]


@pytest.mark.parametrize("variant", ["0", "1"])
def test_batched_every_variant(F, variant, monkeypatch):
    """Each radix/tile variant of the batched kernel's configuration table,
    forced for every length (FFT2D_BATCH_VARIANT), forward and inverse against
    the oracle."""
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.setenv("FFT2D_BATCH_VARIANT", variant)
    say("case batched variant %s" % variant)
    xs = synth.batched_grids(17, VARIANT_SHAPES)
    plan = F.BatchedPlan(VARIANT_SHAPES)
    try:
        desc = plan.describe()
        say(desc)
        listed = desc.split(" variants=")[1].split()[0].split(",")
        assert len(listed) >= 20 and all(v.endswith(":" + variant) for v in listed), desc
        _, ys = _run(F, plan, xs, F.FORWARD)
        _, zs = _run(F, plan, xs, F.INVERSE)
        wf, wi = Worst("batched variant %s fwd" % variant), Worst("batched variant %s inv" % variant)
        for x, y, z, s in zip(xs, ys, zs, VARIANT_SHAPES):
            wf.add(host(y), oracle.fft2_forward(x), s)
            wi.add(host(z), oracle.ifft2(x), s)
        wf.report()
        wi.report()
    finally:
        plan.close()


def test_batched_tuner_choice_is_cached(F, monkeypatch, tmp_path):
    """FFT2D_TUNE=full tunes grid, order, group size and every length's
    variant, and appends the choice to the cache; a second plan of the same
    shapes takes it from the cache (same description) and computes the same
    result bit for bit; a cache file of junk makes the plan tune again."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FFT2D_TUNE_CACHE", str(cache))
    shapes = synth.pow2_shapes(18, 48)
    say("case batched tuner cache, %d points" % sum(r * c for r, c in shapes))
    xs = [dev(x) for x in synth.batched_grids(18, shapes)]
    monkeypatch.setenv("FFT2D_TUNE", "full")
    a = F.BatchedPlan(shapes)
    try:
        da = a.describe()
        say(da)
        assert "tune=tuned" in da and " variants=" in da
        ya = a(xs, F.FORWARD)
        torch.cuda.synchronize()
    finally:
        a.close()
    assert len(cache.read_text().splitlines()) == 1
    monkeypatch.setenv("FFT2D_TUNE", "cached")
    b = F.BatchedPlan(shapes)
    try:
        db = b.describe()
        assert "tune=cache" in db and db.replace("tune=cache", "tune=tuned") == da, (da, db)
        yb = b(xs, F.FORWARD)
        torch.cuda.synchronize()
        for u, v in zip(ya, yb):
            assert torch.equal(u, v)
    finally:
        b.close()
    cache.write_bytes(bytes(range(256)) * 8)
    c = F.BatchedPlan(shapes)
    try:
        assert "tune=tuned" in c.describe()
    finally:
        c.close()
    w = Worst("batched tuned plan")
    for x, y, s in zip(xs, ya, shapes):
        w.add(host(y), oracle.fft2_forward(host(x)), s)
    w.report()


@pytest.mark.parametrize("shapes,expected", [
    ([(2048, 2048), (64, 64), (2048, 2048), (256, 128), (1024, 4096), (1024, 256), (2048, 2048)], 4),
    ([(2048, 2048), (2048, 2048)], 2),
], ids=["mixed", "all-plain"])
def test_batched_plain_transforms(F, shapes, expected, monkeypatch):
    """Grids that hold a large share of a plan's points run as plain transforms
    (a uniform plan's kernels over the whole GPU) beside the persistent kernel:
    forward, inverse, in place, half in place and a pointer change, against the
    oracle and against the same plan with FFT2D_BATCH_PLAIN=off."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.delenv("FFT2D_BATCH_PLAIN")
    say("case batched plain transforms %s" % (shapes,))
    xs = synth.batched_grids(21, shapes)
    plan = F.BatchedPlan(shapes)
    try:
        desc = plan.describe()
        say(desc)
        import re
        nq = int(re.search(r" queues=(\d+) ", desc).group(1))
        total = sum(r * c for r, c in shapes)
        rule = sum(1 for r, c in shapes if r * c >= (1 << 22) and r * c * 2 * nq >= total)
        assert (" plain=%d " % rule) in desc, desc
        if nq == 8:
            assert rule == expected, (rule, expected)
        if rule == len(shapes):
            assert " items=0 " in desc, desc
        ins, ys = _run(F, plan, xs, F.FORWARD)
        _, zs = _run(F, plan, xs, F.INVERSE)
        wf, wi = Worst("batched plain fwd"), Worst("batched plain inv")
        for x, y, z, s in zip(xs, ys, zs, shapes):
            wf.add(host(y), oracle.fft2_forward(x), s)
            wi.add(host(z), oracle.ifft2(x), s)
        wf.report()
        wi.report()
        inplace = [t.clone() for t in ins]
        plan(inplace, F.FORWARD, inplace)
        torch.cuda.synchronize()
        for u, v in zip(ys, inplace):
            assert torch.equal(u, v)
        mixed_in = [t.clone() for t in ins]
        mixed_out = [t if k % 2 == 0 else torch.empty_like(t) for k, t in enumerate(mixed_in)]
        plan(mixed_in, F.FORWARD, mixed_out)
        torch.cuda.synchronize()
        for u, v in zip(ys, mixed_out):
            assert torch.equal(u, v)
    finally:
        plan.close()
    monkeypatch.setenv("FFT2D_BATCH_PLAIN", "off")
    ref_plan = F.BatchedPlan(shapes)
    try:
        assert " plain=0 " in ref_plan.describe()
        _, rs = _run(F, ref_plan, xs, F.FORWARD)
        for y, r, s in zip(ys, rs, shapes):
            rel, mx = errors_dev(y, r)
            assert rel <= TOL and mx <= TOL, (s, rel, mx)
    finally:
        ref_plan.close()


def test_batched_plain_transforms_of_one_tensor(F, monkeypatch):
    """Plain transforms of one shape whose buffers follow each other (slices of
    one tensor) run as one uniform batch; out of place, in place, and with the
    slices given out of order (then grid by grid), all against the oracle."""
    import torch
    monkeypatch.setenv("FFT2D_TUNE", "off")
    monkeypatch.delenv("FFT2D_BATCH_PLAIN")
    shapes = [(2048, 2048)] * 4
    say("case batched plain transforms of one tensor")
    x = synth.complex_grid(22, (4, 2048, 2048))
    ref = oracle.fft2_forward(x)
    plan = F.BatchedPlan(shapes)
    try:
        assert " plain=4 " in plan.describe(), plan.describe()
        xd = dev(x)
        yd = torch.empty_like(xd)
        plan([xd[k] for k in range(4)], F.FORWARD, [yd[k] for k in range(4)])
        w = Worst("batched plain, one tensor")
        for k in range(4):
            w.add(host(yd[k]), ref[k], shapes[k])
        zd = xd.clone()
        plan([zd[k] for k in range(4)], F.FORWARD, [zd[k] for k in range(4)])
        for k in range(4):
            w.add(host(zd[k]), ref[k], shapes[k])
        order = [2, 0, 3, 1]
        od = torch.empty_like(xd)
        plan([xd[k] for k in order], F.FORWARD, [od[k] for k in order])
        for k in range(4):
            w.add(host(od[k]), ref[k], shapes[k])
        w.report()
    finally:
        plan.close()
