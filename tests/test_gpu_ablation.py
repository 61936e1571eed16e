"""The measurement variants of the pass kernels (fft2d_exec_pass_ablated):
they must move every point exactly as the pass does, so that their duration
is the pass's data-movement floor. With the exchanges switched off the pass
is a copy with the pass's access pattern (identity, or for the row pass with
combine the row permutation M2*c + m2 -> M1*m2 + c); with only the
arithmetic switched off the output is a reordering of the input. Both are
checked bit for bit (as multisets, by sorting the 64-bit patterns on the
device, and position by position where the position is fixed)."""

from __future__ import annotations

import re

import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_15437_amd as F
    return F


SHAPES = [(1, 4096, 4096), (1, 8192, 8192), (1, 16384, 2048), (8, 2048, 2048), (1, 1024, 1024), (4096, 1, 16384)]


def _bits(t):
    import torch
    return t.view(torch.int64).reshape(-1)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_ablated_passes_move_every_point(F, shape):
    import torch
    batch, rows, cols = shape
    say("case ablated passes %dx%dx%d" % shape)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(rows + cols + batch)
    x = torch.empty(shape, dtype=torch.complex64, device="cuda")
    x.view(torch.float32).uniform_(-1.0, 1.0, generator=gen)
    plan = F.Plan(*shape)
    s = int(torch.cuda.current_stream().cuda_stream)
    try:
        desc = plan.describe()
        m1 = int(re.search(r"split=(\d+)", desc).group(1))
        say(desc)
        for p in ((0, 1) if rows > 1 else (0,)):
            for mode in (F.ABLATE_EXCHANGE, F.ABLATE_ARITHMETIC):
                # pass 0 reads x and writes out; pass 1 reads and writes the intermediate (out)
                out = torch.empty_like(x) if p == 0 else x.clone()
                before = x if p == 0 else out.clone()
                F.fft2d_exec_pass_ablated(plan.handle, x.data_ptr(), out.data_ptr(), p, mode, 0, 0, s)
                torch.cuda.synchronize()
                same_multiset = torch.equal(torch.sort(_bits(out))[0], torch.sort(_bits(before))[0])
                if mode == F.ABLATE_EXCHANGE:
                    if p == 0 and m1 > 1:
                        want = before.reshape(batch, m1, rows // m1, cols).transpose(1, 2).reshape(shape)
                    else:
                        want = before
                    exact = torch.equal(_bits(out), _bits(want.contiguous()))
                else:
                    exact = True
                say("ablated pass %d mode %d: permutation of the input %s, positions %s"
                    % (p, mode, same_multiset, exact))
                assert same_multiset and exact, (p, mode)
                del out, before
    finally:
        plan.close()


def test_ablation_needs_a_compiled_variant(F):
    import torch
    say("case ablation without variant")
    x = torch.zeros((512, 512), dtype=torch.complex64, device="cuda")
    plan = F.Plan(1, 512, 512)
    try:
        with pytest.raises(F.Fft2dError) as e:
            F.fft2d_exec_pass_ablated(plan.handle, x.data_ptr(), x.data_ptr(), 0, F.ABLATE_EXCHANGE)
        assert e.value.status == 2
    finally:
        plan.close()
