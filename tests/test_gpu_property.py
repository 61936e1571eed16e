"""Property test: random power-of-two shapes and seeds against the FP64 oracle.

Shapes are 2^a x 2^b with a, b in [0, 11] (product at most 2^20 points) and a
batch of 1 to 3; hypothesis runs derandomised, so every run draws the same
cases. Forward and inverse must match the oracle within both parity bounds
(relative L2 and element-wise) and the inverse must undo the forward."""

from __future__ import annotations

import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.gpu_util import check, dev, host  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


@settings(max_examples=40, deadline=None, derandomize=True)
@given(a=st.integers(0, 11), b=st.integers(0, 11), batch=st.integers(1, 3), seed=st.integers(0, 2**31 - 1))
def test_random_shapes_match_oracle(F, a, b, batch, seed):
    if a + b > 20:
        a = 20 - b
    shape = (batch, 1 << a, 1 << b)
    x = synth.complex_grid(seed, shape)
    xd = dev(x)
    plan = F.get_plan(batch, shape[1], shape[2], "cuda")
    y = plan(xd, F.FORWARD)
    z = plan(y, F.INVERSE)
    check(host(y), oracle.fft2_forward(x), "property %s seed %d fwd" % (shape, seed))
    check(host(z), x, "property %s seed %d round trip" % (shape, seed))


# Split column transforms on random shapes: N = 1024 ... 8192 columns, the
# row count a multiple of the split factor M1 the plan would choose for N,
# both row passes with combine (last stage across rows, separate combine
# exchange), forced through FFT2D_SPLIT / FFT2D_COMBINE at sizes the oracle
# handles quickly.
_M1 = {1024: 16, 2048: 8, 4096: 4, 8192: 4}


@settings(max_examples=20, deadline=None, derandomize=True)
@given(b=st.integers(10, 13), k=st.integers(1, 5), batch=st.integers(1, 2), cross_row=st.booleans(),
       seed=st.integers(0, 2**31 - 1))
def test_random_split_shapes_match_oracle(F, b, k, batch, cross_row, seed):
    import os
    cols = 1 << b
    m1 = _M1[cols]
    rows = m1 << k
    while rows * cols * batch > (1 << 21) and rows > 2 * m1:
        rows //= 2
    shape = (batch, rows, cols)
    saved = {v: os.environ.get(v) for v in ("FFT2D_SPLIT", "FFT2D_COMBINE")}
    os.environ["FFT2D_SPLIT"] = str(m1)
    os.environ["FFT2D_COMBINE"] = "xrow" if cross_row else "classic"
    try:
        plan = F.Plan(batch, rows, cols)
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    try:
        desc = plan.describe()
        assert ("split=%d " % m1) in desc, desc
        assert ("combine xrow" in desc) == cross_row, desc
        x = synth.complex_grid(seed, shape)
        xd = dev(x)
        y = plan(xd, F.FORWARD)
        z = plan(y, F.INVERSE)
        check(host(y), oracle.fft2_forward(x), "split property %s seed %d fwd" % (shape, seed))
        check(host(z), x, "split property %s seed %d round trip" % (shape, seed))
    finally:
        plan.close()


# Batched plans of random shape sets (2^a x 2^b, a, b in [0, 11], at most 2^21
# points per set), with fixed or guided work groups and the untuned schedule:
# every transform forward and inverse against the oracle.
@settings(max_examples=12, deadline=None, derandomize=True)
@given(dims=st.lists(st.tuples(st.integers(0, 11), st.integers(0, 11)), min_size=1, max_size=12),
       guided=st.booleans(), seed=st.integers(0, 2**31 - 1))
def test_random_batched_sets_match_oracle(F, dims, guided, seed):
    import os
    shapes = []
    total = 0
    for a, b in dims:
        if total + (1 << (a + b)) > (1 << 21):
            continue
        shapes.append((1 << a, 1 << b))
        total += 1 << (a + b)
    if not shapes:
        shapes = [(1, 1)]
    saved = {v: os.environ.get(v) for v in ("FFT2D_TUNE", "FFT2D_BATCH_GUIDED")}
    os.environ["FFT2D_TUNE"] = "off"
    os.environ["FFT2D_BATCH_GUIDED"] = "1" if guided else "0"
    try:
        plan = F.BatchedPlan(shapes)
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    try:
        assert (" guided " in plan.describe()) == guided, plan.describe()
        xs = synth.batched_grids(seed % 1000, shapes)
        ys = plan([dev(x) for x in xs], F.FORWARD)
        zs = plan([dev(x) for x in xs], F.INVERSE)
        for x, y, z, s in zip(xs, ys, zs, shapes):
            check(host(y), oracle.fft2_forward(x), "batched property %s guided %d fwd" % (s, guided))
            check(host(z), oracle.ifft2(x), "batched property %s guided %d inv" % (s, guided))
    finally:
        plan.close()
