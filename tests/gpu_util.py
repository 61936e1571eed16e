"""Helpers for the GPU parity tests: host <-> device copies and error metrics."""

from __future__ import annotations

import sys

import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, ref) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((a - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def say(*args):
    """Print and flush at once, so a GPU run names its case before each step."""
    print(*args, flush=True)
    sys.stdout.flush()


# Relative L2 error bound of every FP32 result against the FP64 oracle.
TOL = 1e-5
