"""The access-pattern and LDS probes behind the pass kernels' design
(fft2d_probe_tile_copy, fft2d_probe_lds): the tile copy must reproduce its
input bit for bit for every tile width and cache hint, both probes reject bad
arguments, and their rates are measured and printed."""

from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


@pytest.mark.parametrize("tile_cols,rows", [(16, 4096), (32, 2048), (64, 1024)])
@pytest.mark.parametrize("nt", [False, True])
def test_tile_copy_is_exact(F, tile_cols, rows, nt):
    say("case tile copy %d columns nt=%s" % (tile_cols, nt))
    x = synth.complex_grid(70 + tile_cols, (rows, 128))
    xd = dev(x)
    import torch
    yd = torch.zeros_like(xd)
    F.fft2d_probe_tile_copy(xd.data_ptr(), yd.data_ptr(), rows, 128, tile_cols, 2, nt)
    assert np.array_equal(host(yd), x)


def test_probe_arguments(F):
    say("case probe arguments")
    import torch
    xd = torch.zeros(2048 * 64, dtype=torch.complex64, device="cuda")
    yd = torch.zeros_like(xd)
    for bad in [dict(tile_cols=8), dict(rows=1000), dict(residues=0)]:
        args = dict(rows=2048, cols=64, tile_cols=16, residues=1)
        args.update(bad)
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_probe_tile_copy(xd.data_ptr(), yd.data_ptr(), args["rows"], args["cols"], args["tile_cols"],
                                    args["residues"], False)
        assert e.value.status == 2
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_probe_tile_copy(xd.data_ptr(), xd.data_ptr() + 8, 2048, 64, 16, 1, False)
    assert e.value.status == 9
    sink = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_probe_lds(8, False, sink.data_ptr(), sink.numel())
    assert e.value.status == 2
    with pytest.raises(F.Fft2dError) as e:
        F.fft2d_probe_lds(12, False, sink.data_ptr(), sink.numel())
    assert e.value.status == 2


def test_probe_rates(F):
    """8192 x 8192 column-tile copies (M1 = 4, the 8192^2 split column pass's
    rows) with 128-, 256- and 512-byte row segments, each after a 1 GiB read,
    and the LDS bandwidth per CU; printed, not asserted."""
    import bench
    import torch
    res = bench.probe_rates(F, torch, iters=5)
    for k, v in res.items():
        say("probe %s: %s" % (k, v))
    assert all(v["ms"] > 0 for v in res.values())
