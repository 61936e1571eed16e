"""The radix-16 stage on the vector ALU against the matrix cores
(fft2d_probe_dft16): both kernels must compute (Pi F / 4)^reps x, F the
16-point DFT and Pi the base-4 digit swap, checked against the FP64 oracle's
16-point transform with both bounds of tests/gpu_util.py; then both DFT16
rates are measured and printed (the numbers behind the choice of butterflies
over MFMA for the pass kernels)."""

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


def oracle_probe(x, reps):
    """(Pi F / 4)^reps x in FP64 with the oracle's 16-point transform; scaling
    by 2^-16 after every 8 applications as the kernels do."""
    y = x.astype(np.complex128)
    idx = np.arange(16)
    perm = (idx >> 2) + 4 * (idx & 3)  # point 4q + r -> q + 4r
    for it in range(reps):
        f = oracle.fft2(y.reshape(-1, 1, 16), oracle.FORWARD).reshape(-1, 16)
        y = np.empty_like(f)
        y[:, perm] = f
        if it % 8 == 7:
            y *= 2.0 ** -16
    return y


@pytest.mark.parametrize("reps", [8, 64])
def test_dft16_probe_matches_oracle(F, reps):
    import torch
    say("case dft16 probe reps %d" % reps)
    x = synth.complex_grid(23, (4096, 16))
    ref = oracle_probe(x, reps)
    s = int(torch.cuda.current_stream().cuda_stream)
    for method, name in ((F.DFT16_BUTTERFLY, "butterfly"), (F.DFT16_MFMA, "mfma")):
        xd = dev(x)
        y = torch.empty_like(xd)
        F.fft2d_probe_dft16(method, xd.data_ptr(), y.data_ptr(), 4096, reps, 0, 0, s)
        check(host(y), ref, "dft16 %s reps %d" % (name, reps))
        F.fft2d_probe_dft16(method, xd.data_ptr(), xd.data_ptr(), 4096, reps, 0, 0, s)  # in place
        assert torch.equal(xd, y)


def test_dft16_rates(F):
    """Both methods on 2^20 vectors, 512 applications each, timed with events
    bound to the kernel launch; prints G DFT16/s and the issued FLOP/s."""
    import torch
    say("case dft16 rates")
    count, reps = 1 << 20, 512
    s = torch.cuda.current_stream()
    x = torch.zeros((count, 16), dtype=torch.complex64, device="cuda")
    x.view(torch.float32).uniform_(-1, 1)
    y = torch.empty_like(x)
    rates = {}
    for method, name, flops in ((F.DFT16_BUTTERFLY, "butterfly", 5 * 16 * 4), (F.DFT16_MFMA, "mfma", 2 * 32 * 32)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        b.record(s)
        torch.cuda.synchronize()
        F.fft2d_probe_dft16(method, x.data_ptr(), y.data_ptr(), count, reps, 0, 0, int(s.cuda_stream))  # warm-up
        ms = []
        for _ in range(3):
            F.fft2d_probe_dft16(method, x.data_ptr(), y.data_ptr(), count, reps, a.cuda_event, b.cuda_event,
                                int(s.cuda_stream))
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        t = min(ms)
        rates[name] = count * reps / (t * 1e-3)
        say("dft16 %s: %.3f ms, %.1f G DFT16/s, %.1f TFLOP/s issued (%d flop per DFT16)"
            % (name, t, rates[name] / 1e9, rates[name] * flops / 1e12, flops))
        assert np.isfinite(host(y)).all()
    say("dft16 butterfly / mfma rate: %.2f" % (rates["butterfly"] / rates["mfma"]))
