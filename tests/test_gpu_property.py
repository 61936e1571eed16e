"""Property test: random power-of-two shapes and seeds against the FP64 oracle.

Shapes are 2^a x 2^b with a, b in [0, 11] (product at most 2^20 points) and a
batch of 1 to 3; hypothesis runs derandomised, so every run draws the same
cases. Forward and inverse must match the oracle within the parity bound and
the inverse must undo the forward."""

from __future__ import annotations

import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.gpu_util import TOL, dev, host, rel_l2, say  # noqa: E402

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
    ef = rel_l2(host(y), oracle.fft2_forward(x))
    ei = rel_l2(host(z), x)
    say("property %s seed %d: fwd %.2e round trip %.2e" % (shape, seed, ef, ei))
    assert ef <= TOL and ei <= TOL
