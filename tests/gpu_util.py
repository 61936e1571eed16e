"""Helpers for the GPU parity tests: host <-> device copies and error metrics.

Every comparison against the FP64 oracle applies two bounds:

* relative L2 over the whole output, ``||y - ref||_2 / ||ref||_2 <= TOL``;
* element by element, ``max_i |y_i - ref_i| <= ELEM_TOL * ||ref||_2 / sqrt(P)``,
  i.e. every point within ELEM_TOL of the reference's RMS magnitude.

The FP32 transforms measure 1e-7 ... 3e-7 relative L2, so their largest
element error sits near 1e-6 of the RMS magnitude: the element bound leaves
about ten times that, and a wrong tile, row or column (an error of 1e-4 in a
few percent of the points), which the global norm alone would let through,
fails it.
"""

from __future__ import annotations

import math
import sys

import numpy as np

# Relative L2 error bound of every FP32 result against the FP64 oracle.
TOL = 1e-5
# Element-wise bound, in units of the reference's RMS magnitude.
ELEM_TOL = 1e-5


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def errors(a, ref):
    """(relative L2, largest element error over the reference's RMS magnitude),
    both in FP64. An all-zero reference gives absolute errors instead."""
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    if ref.size == 0:
        return 0.0, 0.0
    d = np.abs(a - ref).ravel()
    den = float(np.linalg.norm(ref.ravel()))
    num = float(np.linalg.norm(d))
    mx = float(d.max())
    rms = den / math.sqrt(ref.size)
    return (num / den if den > 0 else num), (mx / rms if rms > 0 else mx)


def rel_l2(a, ref) -> float:
    return errors(a, ref)[0]


def errors_dev(y, ref):
    """errors() of two device tensors, computed on the device in complex128."""
    import torch
    y = y.detach().to(torch.complex128)
    ref = ref.detach().to(torch.complex128)
    if ref.numel() == 0:
        return 0.0, 0.0
    d = torch.abs(y - ref)
    den = float(torch.linalg.vector_norm(ref))
    num = float(torch.linalg.vector_norm(d))
    mx = float(d.max())
    rms = den / math.sqrt(ref.numel())
    return (num / den if den > 0 else num), (mx / rms if rms > 0 else mx)


def say(*args):
    """Print and flush at once, so a GPU run names its case before each step."""
    print(*args, flush=True)
    sys.stdout.flush()


def check(a, ref, tag, tol=TOL, elem_tol=ELEM_TOL):
    """Assert both bounds for host arrays; prints both metrics; returns them."""
    rel, mx = errors(a, ref)
    say("%s rel_l2=%.3e max_elem=%.3e" % (tag, rel, mx))
    assert rel <= tol and mx <= elem_tol, (tag, rel, mx)
    return rel, mx


def check_dev(y, ref, tag, tol=TOL, elem_tol=ELEM_TOL):
    """check() for two device tensors (no copy to the host)."""
    rel, mx = errors_dev(y, ref)
    say("%s rel_l2=%.3e max_elem=%.3e" % (tag, rel, mx))
    assert rel <= tol and mx <= elem_tol, (tag, rel, mx)
    return rel, mx
