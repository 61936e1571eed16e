"""Torch-facing wrappers: plans, fft2/ifft2, batched lists and autograd.

Tensors must be complex64, on a HIP ("cuda") device. Work is enqueued on the
tensor's current torch stream; nothing here synchronises.
"""

from __future__ import annotations

import collections
import threading

import torch

from . import _lib
from ._lib import FORWARD, INVERSE


def _is_pow2(n: int) -> bool:
    return n >= 1 and (n & (n - 1)) == 0


def _stream_handle(device) -> int:
    return int(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(x, name="x"):
    if not isinstance(x, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if x.dtype != torch.complex64:
        raise TypeError("%s must be complex64, got %s" % (name, x.dtype))
    if x.device.type != "cuda":
        raise TypeError("%s must be on a GPU device, got %s" % (name, x.device))
    if x.dim() < 2:
        raise ValueError("%s needs at least 2 dimensions (rows, cols)" % name)
    M, N = x.shape[-2], x.shape[-1]
    if not (_is_pow2(M) and _is_pow2(N)) or M > _lib.MAX_LEN or N > _lib.MAX_LEN:
        raise ValueError("%s: rows and cols must be powers of two in [1, %d], got %dx%d" % (name, _lib.MAX_LEN, M, N))


class Plan:
    """A uniform plan: ``batch`` grids of ``rows`` x ``cols`` on one device."""

    def __init__(self, batch: int, rows: int, cols: int, device=None):
        self.batch, self.rows, self.cols = int(batch), int(rows), int(cols)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.handle = _lib.fft2d_plan(self.batch, self.rows, self.cols)

    @property
    def numel(self) -> int:
        return self.batch * self.rows * self.cols

    def exec_ptr(self, in_ptr: int, out_ptr: int, direction: int, stream: int) -> None:
        _lib.fft2d_exec(self.handle, in_ptr, out_ptr, direction, stream)

    def backward_ptr(self, g_ptr: int, gx_ptr: int, forward_direction: int, stream: int) -> None:
        _lib.fft2d_backward(self.handle, g_ptr, gx_ptr, forward_direction, stream)

    def _check_io(self, x, out):
        _check_tensor(x)
        if x.device != self.device:
            raise ValueError("tensor on %s, plan on %s" % (x.device, self.device))
        if x.numel() != self.numel or x.shape[-2:] != (self.rows, self.cols):
            raise ValueError("tensor shape %s does not match plan %dx%dx%d" %
                             (tuple(x.shape), self.batch, self.rows, self.cols))
        if out is not None:
            _check_tensor(out, "out")
            if out.shape != x.shape or not out.is_contiguous():
                raise ValueError("out must be contiguous with the input's shape")

    def __call__(self, x, direction=FORWARD, out=None):
        self._check_io(x, out)
        x = x.contiguous()
        if out is None:
            out = torch.empty_like(x)
        with torch.cuda.device(self.device):
            self.exec_ptr(x.data_ptr(), out.data_ptr(), direction, _stream_handle(x.device))
        return out

    def backward(self, g, forward_direction=FORWARD, out=None):
        self._check_io(g, out)
        g = g.contiguous()
        if out is None:
            out = torch.empty_like(g)
        with torch.cuda.device(self.device):
            self.backward_ptr(g.data_ptr(), out.data_ptr(), forward_direction, _stream_handle(g.device))
        return out

    def describe(self) -> str:
        return _lib.fft2d_plan_describe(self.handle)

    def close(self):
        """Free the plan. The C call waits for nothing, so the plan's device is
        synchronised first: no queued work may still use the plan's memory."""
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.fft2d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass


class BatchedPlan:
    """Many 2D transforms of different shapes run by one persistent launch."""

    def __init__(self, shapes, device=None):
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.handle = _lib.fft2d_plan_batched([r for r, _ in self.shapes], [c for _, c in self.shapes])

    def exec_ptrs(self, in_ptrs, out_ptrs, direction: int, stream: int) -> None:
        """in_ptrs / out_ptrs: one device pointer per planned grid, as sequences or as
        uint64 arrays from ``pointer_array`` (no conversion per call)."""
        ia = _lib.pointer_array(in_ptrs)
        oa = _lib.pointer_array(out_ptrs)
        if ia.size != len(self.shapes) or oa.size != len(self.shapes):
            raise ValueError("expected %d input and output pointers, got %d and %d"
                             % (len(self.shapes), ia.size, oa.size))
        _lib.fft2d_exec_batched(self.handle, ia, oa, direction, stream)

    def __call__(self, xs, direction=FORWARD, outs=None):
        if len(xs) != len(self.shapes):
            raise ValueError("expected %d tensors, got %d" % (len(self.shapes), len(xs)))
        for i, (x, s) in enumerate(zip(xs, self.shapes)):
            _check_tensor(x, "xs[%d]" % i)
            if tuple(x.shape) != s or not x.is_contiguous() or x.device != self.device:
                raise ValueError("xs[%d] must be contiguous with shape %s on %s" % (i, s, self.device))
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        if len(outs) != len(self.shapes):
            raise ValueError("expected %d output tensors, got %d" % (len(self.shapes), len(outs)))
        for i, (o, s) in enumerate(zip(outs, self.shapes)):
            _check_tensor(o, "outs[%d]" % i)
            if tuple(o.shape) != s or not o.is_contiguous() or o.device != self.device:
                raise ValueError("outs[%d] must be contiguous with shape %s on %s" % (i, s, self.device))
        with torch.cuda.device(self.device):
            self.exec_ptrs([x.data_ptr() for x in xs], [o.data_ptr() for o in outs], direction,
                           _stream_handle(self.device))
        return outs

    def describe(self) -> str:
        return _lib.fft2d_plan_describe(self.handle)

    def close(self):
        """Free the plan. The C call waits for nothing, so the plan's device is
        synchronised first: no queued work may still use the plan's memory."""
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.fft2d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass


_plans = collections.OrderedDict()
_plans_lock = threading.Lock()


PLAN_CACHE_SIZE = 32  # plans kept by get_plan (least recently used evicted beyond this)


def get_plan(batch: int, rows: int, cols: int, device) -> Plan:
    """Cached uniform plan for (device, batch, rows, cols). At most PLAN_CACHE_SIZE
    plans are kept; an evicted plan is freed when its last reference goes."""
    dev = torch.device(device)
    key = (dev.index if dev.index is not None else torch.cuda.current_device(), int(batch), int(rows), int(cols))
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            p = Plan(batch, rows, cols, device=torch.device("cuda", key[0]))
            _plans[key] = p
            while len(_plans) > PLAN_CACHE_SIZE:
                _plans.popitem(last=False)
        else:
            _plans.move_to_end(key)
        return p


def clear_plan_cache() -> None:
    """Forget every plan cached by get_plan (each is freed with its last reference)."""
    with _plans_lock:
        _plans.clear()


def _plan_for(x) -> Plan:
    M, N = x.shape[-2], x.shape[-1]
    batch = x.numel() // (M * N) if x.numel() else 0
    if batch == 0:
        raise ValueError("empty tensor")
    return get_plan(batch, M, N, x.device)


def fft2(x, out=None):
    """Unscaled forward 2D FFT over the last two dimensions."""
    _check_tensor(x)
    return _plan_for(x)(x, FORWARD, out)


def ifft2(x, out=None):
    """Inverse 2D FFT over the last two dimensions (scaled by 1/(M N))."""
    _check_tensor(x)
    return _plan_for(x)(x, INVERSE, out)


def fft2_batched(xs, direction=FORWARD, plan=None):
    """Transform a list of 2D tensors of (possibly) different shapes in one launch."""
    if plan is None:
        plan = BatchedPlan([tuple(x.shape) for x in xs], device=xs[0].device)
    return plan(xs, direction)


class FFT2Function(torch.autograd.Function):
    """y = fft2(x) (direction FORWARD) or ifft2(x) (INVERSE), differentiable.

    The backward pass is the adjoint kernel (fft2d_backward): F^H g for the
    forward transform, (1/(M N)) F g for the inverse, which is the gradient
    under torch's convention grad = dL/dRe + i dL/dIm.
    """

    @staticmethod
    def forward(ctx, x, direction=FORWARD):
        _check_tensor(x)
        plan = _plan_for(x)
        ctx.plan = plan
        ctx.direction = int(direction)
        return plan(x, int(direction))

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        return ctx.plan.backward(g, ctx.direction), None


def fft2_diff(x, direction=FORWARD):
    return FFT2Function.apply(x, direction)
