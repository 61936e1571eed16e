"""The C ABI from a plain C program (tests/c/abi_roundtrip.c, built by
__graft_entry__.build()): no C++ and no Python on the call path. The program
transforms a grid read from a file, forward and back, and its outputs are
compared with the FP64 oracle here."""

from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check, say

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_roundtrip")


@pytest.mark.parametrize("shape", [(64, 64), (512, 256), (4096, 1024)], ids=lambda s: "%dx%d" % s)
def test_c_client_round_trip(shape, tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(BIN), "tests/c/abi_roundtrip is not built: run __graft_entry__.build()"
    say("case C client %dx%d" % shape)
    x = synth.complex_grid(41, shape)
    src, fwd, rt = (str(tmp_path / n) for n in ("in.bin", "fwd.bin", "rt.bin"))
    x.tofile(src)
    r = subprocess.run([BIN, str(shape[0]), str(shape[1]), src, fwd, rt], capture_output=True, text=True,
                       timeout=120)
    say(r.stdout.strip())
    assert r.returncode == 0, r.stderr
    y = np.fromfile(fwd, dtype=np.complex64).reshape(shape)
    z = np.fromfile(rt, dtype=np.complex64).reshape(shape)
    check(y, oracle.fft2_forward(x), "C client %dx%d fwd" % shape)
    check(z, x, "C client %dx%d round trip" % shape)
