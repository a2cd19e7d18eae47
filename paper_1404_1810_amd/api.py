"""PyTorch-facing binding of the AM-QFT library.

Torch supplies device memory and the current HIP stream; every transform step
runs in the HIP kernels of libamqft.so, reached through the C ABI.

Storage conventions (last dimension = the transform axis):
  complex128 / complex64 tensors       -> AMQFT_C128 / AMQFT_C64
  float16 / bfloat16 tensors (..., n, 2) -> AMQFT_C32H / AMQFT_C32B
                                           (interleaved re/im, FP32 math)
  int32 tensors (..., n, 2)              -> AMQFT_C32I (fixed point, variants
                                           1, 3, 5, 7, Q2.29 constants)
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

_DTYPES = {torch.complex128: _lib.C128, torch.complex64: _lib.C64,
           torch.float16: _lib.C32H, torch.bfloat16: _lib.C32B, torch.int32: _lib.C32I}
_PAIRS = (_lib.C32H, _lib.C32B, _lib.C32I)  # storage with a trailing (re, im) dimension


def _storage(x: torch.Tensor):
    """(amqft dtype, n, batch) of a tensor in one of the storage layouts."""
    if x.dtype not in _DTYPES:
        raise TypeError("unsupported dtype %s" % x.dtype)
    dt = _DTYPES[x.dtype]
    if dt in _PAIRS:
        if x.dim() < 2 or x.shape[-1] != 2:
            raise ValueError("half/bfloat16/int32 storage must have a trailing (re, im) dimension of size 2")
        n = x.shape[-2]
        batch = x.numel() // (2 * n) if n else 0
    else:
        if x.dim() < 1:
            raise ValueError("need at least one dimension")
        n = x.shape[-1]
        batch = x.numel() // n if n else 0
    return dt, n, batch


def _stream_handle(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


class Plan:
    """An amqft_plan (constants and workspace live on the device)."""

    def __init__(self, n: int, batch: int, variant: int = 4, dtype: int = _lib.C64, flags: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.amqft_plan_create(ctypes.byref(h), int(n), int(batch), int(variant), int(dtype),
                                         int(flags)), "amqft_plan_create")
        self._h = h
        self.n, self.batch, self.variant, self.dtype, self.flags = int(n), int(batch), int(variant), int(dtype), int(flags)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.load().amqft_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            if self._h is not None and self._h.value and torch.cuda.is_available():
                torch.cuda.synchronize()
            self.close()
        except Exception:
            pass

    def _check_tensor(self, t: torch.Tensor, name: str):
        if not t.is_cuda:
            raise ValueError("%s must be a GPU tensor (the AM-QFT path has no CPU fallback)" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        dt, n, batch = _storage(t)
        if dt != self.dtype or n != self.n or batch != self.batch:
            raise ValueError("%s does not match the plan (dtype %d n %d batch %d)" % (name, self.dtype, self.n,
                                                                                     self.batch))

    def exec(self, x: torch.Tensor, out: torch.Tensor | None = None, adjoint: bool = False) -> torch.Tensor:
        self._check_tensor(x, "input")
        y = torch.empty_like(x) if out is None else out
        self._check_tensor(y, "output")
        if y.device != x.device:
            raise ValueError("output is on %s, input on %s" % (y.device, x.device))
        fn = _lib.load().amqft_exec_adjoint if adjoint else _lib.load().amqft_exec
        _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                      _stream_handle(x.device)), "amqft_exec" + ("_adjoint" if adjoint else ""))
        return y

    def power_loss_grad(self, x: torch.Tensor, w: torch.Tensor):
        self._check_tensor(x, "x")
        self._check_tensor(w, "w")
        g = torch.empty_like(x)
        ldt = torch.float64 if self.dtype == _lib.C128 else torch.float32
        loss = torch.empty(self.batch, dtype=ldt, device=x.device)
        _lib.check(_lib.load().amqft_power_loss_grad(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(loss.data_ptr()), _stream_handle(x.device)), "amqft_power_loss_grad")
        return loss, g

    def describe(self) -> str:
        return _describe(self._h)

    def workspace_bytes(self) -> int:
        sz = ctypes.c_size_t()
        _lib.check(_lib.load().amqft_plan_workspace_size(self._h, ctypes.byref(sz)), "workspace_size")
        return int(sz.value)

    def constants(self, n: int | None = None):
        import numpy as np
        n = self.n if n is None else n
        out = np.zeros(max(n // 4, 1), dtype=np.float64)
        _lib.check(_lib.load().amqft_plan_constants(self._h, int(n), ctypes.c_void_p(out.ctypes.data), out.size),
                   "amqft_plan_constants")
        return out


def _describe(h) -> str:
    buf = ctypes.create_string_buffer(512)
    _lib.check(_lib.load().amqft_plan_describe(h, buf, 512), "amqft_plan_describe")
    return buf.value.decode()


_plan_cache: dict = {}


def get_plan(n: int, batch: int, variant: int, dtype: int, flags: int = 0, device=None) -> Plan:
    """Cached plan per shape and device.  A plan that owns a workspace may not
    run on two streams at once, so those are cached per stream as well."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    key = (n, batch, variant, dtype, flags, dev)
    p = _plan_cache.get(key)
    if p is not None:
        return p
    skey = key + (torch.cuda.current_stream(dev).cuda_stream,)
    p = _plan_cache.get(skey)
    if p is None:
        with torch.cuda.device(dev):
            p = Plan(n, batch, variant, dtype, flags)
        _plan_cache[skey if p.workspace_bytes() > 0 else key] = p
    return p


def fft(x: torch.Tensor, variant: int = 4, flags: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Unnormalised forward DFT (eq. qft_0A) along the last axis by AM-QFT."""
    x = x.contiguous()
    dt, n, batch = _storage(x)
    return get_plan(n, batch, variant, dt, flags, x.device).exec(x, out=out)


def adjoint(g: torch.Tensor, variant: int = 4, flags: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """F^H g (unnormalised inverse DFT) along the last axis."""
    g = g.contiguous()
    dt, n, batch = _storage(g)
    return get_plan(n, batch, variant, dt, flags, g.device).exec(g, out=out, adjoint=True)


def fft_(x: torch.Tensor, variant: int = 4, flags: int = 0) -> torch.Tensor:
    """The forward transform in place (AMQFT_FLAG_IN_PLACE: no workspace up to
    one workgroup's LDS, about a quarter of a signal above it where the
    in-place path exists; the plan refuses other sizes).  x must be
    contiguous; it is overwritten and returned."""
    if not x.is_contiguous():
        raise ValueError("an in-place transform needs a contiguous tensor")
    dt, n, batch = _storage(x)
    return get_plan(n, batch, variant, dt, flags | _lib.FLAG_IN_PLACE, x.device).exec(x, out=x)


def adjoint_(g: torch.Tensor, variant: int = 4, flags: int = 0) -> torch.Tensor:
    """F^H g in place (see fft_)."""
    if not g.is_contiguous():
        raise ValueError("an in-place transform needs a contiguous tensor")
    dt, n, batch = _storage(g)
    return get_plan(n, batch, variant, dt, flags | _lib.FLAG_IN_PLACE, g.device).exec(g, out=g, adjoint=True)


def ifft(X: torch.Tensor, variant: int = 4) -> torch.Tensor:
    """Normalised inverse DFT = F^H X / N (the scaling is the caller's step)."""
    return adjoint(X, variant) / X.shape[-1]


class AMQFTFunction(torch.autograd.Function):
    """y = F x with the hand-written adjoint kernel as its backward:
    for a real loss L, dL/dx* convention (PyTorch) gives grad_x = F^H grad_y."""

    @staticmethod
    def forward(ctx, x, variant: int = 4):
        ctx.variant = variant
        return fft(x, variant)

    @staticmethod
    def backward(ctx, grad_y):
        return adjoint(grad_y.contiguous(), ctx.variant), None


def amqft(x: torch.Tensor, variant: int = 4) -> torch.Tensor:
    """Differentiable AM-QFT forward transform (complex64/complex128)."""
    return AMQFTFunction.apply(x, variant)


def power_loss(x: torch.Tensor, w: torch.Tensor, variant: int = 4):
    """Fused per-signal loss sum_k |w * F x|^2 and its gradient 2 F^H(|w|^2 F x)
    in one kernel: returns (loss[batch], grad_x)."""
    x = x.contiguous()
    w = w.contiguous()
    dt, n, batch = _storage(x)
    return get_plan(n, batch, variant, dt, 0, x.device).power_loss_grad(x, w)


class ManyPlan:
    """amqft_plan_create_many: signals of different power-of-two lengths in one
    packed buffer (signal i: lengths[i] points at complex element offsets[i];
    offsets has count+1 entries).  Executed by one persistent launch for the
    short lengths plus one launch sequence per long length class; the first
    out-of-place execution autotunes the launch shapes."""

    def __init__(self, lengths, offsets, variant: int = 4, dtype: int = _lib.C64, flags: int = 0):
        import numpy as np
        lib = _lib.load()
        L = np.ascontiguousarray(lengths, dtype=np.int64)
        O = np.ascontiguousarray(offsets, dtype=np.int64)
        if O.shape[0] != L.shape[0] + 1:
            raise ValueError("offsets needs count+1 entries")
        h = ctypes.c_void_p()
        _lib.check(lib.amqft_plan_create_many(ctypes.byref(h), int(L.shape[0]), ctypes.c_void_p(L.ctypes.data),
                                              ctypes.c_void_p(O.ctypes.data), int(variant), int(dtype), int(flags)),
                   "amqft_plan_create_many")
        self._h = h
        self.count = int(L.shape[0])
        self.total = int(O[-1]) if O.shape[0] else 0
        self.variant, self.dtype = int(variant), int(dtype)

    def close(self):
        if self._h is not None and self._h.value:
            _lib.load().amqft_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            if self._h is not None and self._h.value and torch.cuda.is_available():
                torch.cuda.synchronize()
            self.close()
        except Exception:
            pass

    def describe(self) -> str:
        return _describe(self._h)

    def workspace_bytes(self) -> int:
        sz = ctypes.c_size_t()
        _lib.check(_lib.load().amqft_plan_workspace_size(self._h, ctypes.byref(sz)), "workspace_size")
        return int(sz.value)

    def _check_buffer(self, t: torch.Tensor, name: str):
        if not t.is_cuda:
            raise ValueError("%s must be a GPU tensor (the AM-QFT path has no CPU fallback)" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        dt = _DTYPES.get(t.dtype)
        if dt != self.dtype:
            raise ValueError("%s has dtype %s, the plan %d" % (name, t.dtype, self.dtype))
        npts = t.numel() // (2 if dt in _PAIRS else 1)
        if npts < self.total:
            raise ValueError("%s holds %d points, the plan's offsets reach %d" % (name, npts, self.total))

    def exec(self, x: torch.Tensor, out: torch.Tensor | None = None, adjoint: bool = False,
             graph: bool = False) -> torch.Tensor:
        self._check_buffer(x, "input")
        if out is not None:
            self._check_buffer(out, "output")
            if out.device != x.device:
                raise ValueError("output is on %s, input on %s" % (out.device, x.device))
        y = torch.empty_like(x) if out is None else out
        lib = _lib.load()
        st = _stream_handle(x.device)
        if graph:
            rc = lib.amqft_exec_graph(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      1 if adjoint else 0, st)
            _lib.check(rc, "amqft_exec_graph")
        else:
            fn = lib.amqft_exec_adjoint if adjoint else lib.amqft_exec
            _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), st), "amqft_exec")
        return y


def exec_graph(plan: Plan, x: torch.Tensor, out: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
    """Run a single-length plan through its captured HIP graph (captured on the
    first call for this (x, out) pair)."""
    plan._check_tensor(x, "input")
    plan._check_tensor(out, "output")
    _lib.check(_lib.load().amqft_exec_graph(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), 1 if adjoint else 0,
                                            _stream_handle(x.device)), "amqft_exec_graph")
    return out


def exec_noalloc(x: torch.Tensor, variant: int = 4, adjoint: bool = False,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """amqft_exec_noalloc: the transform along the last axis with no plan and no
    allocation inside the library (its workspace is a fixed device array per
    GPU; calls that overlap on one GPU race).  `out` may be given so that the
    call allocates nothing at all."""
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("input must be a contiguous GPU tensor (the AM-QFT path has no CPU fallback)")
    dt, n, batch = _storage(x)
    y = torch.empty_like(x) if out is None else out
    if y.device != x.device or y.dtype != x.dtype or y.shape != x.shape or not y.is_contiguous():
        raise ValueError("output must be a contiguous tensor of the input's shape, dtype and device")
    with torch.cuda.device(x.device):
        _lib.check(_lib.load().amqft_exec_noalloc(int(n), int(batch), int(variant), int(dt), 1 if adjoint else 0,
                                                  ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                                  _stream_handle(x.device)), "amqft_exec_noalloc")
    return y


_REAL_KINDS = {"rdft": _lib.RDFT, "dct0": _lib.DCT0, "dst0": _lib.DST0}
_REAL_DTYPES = {torch.float64: _lib.C128, torch.float32: _lib.C64}


class RealPlan:
    """amqft_plan_create_real: RDFT, DCT-0 or DST-0 of real signals of
    periodization n, batch signals back to back (see include/amqft.h for the
    strides).  Two real signals share one complex lane of the recursion."""

    def __init__(self, n: int, batch: int, kind: str = "rdft", variant: int = 4, dtype: int = _lib.C64,
                 flags: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.amqft_plan_create_real(ctypes.byref(h), int(n), int(batch), _REAL_KINDS[kind], int(variant),
                                              int(dtype), int(flags)), "amqft_plan_create_real")
        self._h = h
        self.n, self.batch, self.kind, self.variant, self.dtype = int(n), int(batch), kind, int(variant), int(dtype)

    def close(self):
        if self._h is not None and self._h.value:
            _lib.load().amqft_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            if self._h is not None and self._h.value and torch.cuda.is_available():
                torch.cuda.synchronize()
            self.close()
        except Exception:
            pass

    def describe(self) -> str:
        return _describe(self._h)

    @property
    def in_len(self) -> int:
        return {"rdft": self.n, "dct0": self.n // 2 + 1, "dst0": self.n // 2 - 1}[self.kind]

    def exec(self, x: torch.Tensor, out: torch.Tensor | None = None, adjoint: bool = False) -> torch.Tensor:
        rdt = torch.float64 if self.dtype == _lib.C128 else torch.float32
        if not x.is_cuda or not x.is_contiguous() or x.dtype != rdt:
            raise ValueError("input must be a contiguous GPU tensor of dtype %s" % rdt)
        if x.numel() != self.batch * self.in_len or (x.dim() and x.shape[-1] != self.in_len):
            raise ValueError("input does not match the plan (batch %d x %d)" % (self.batch, self.in_len))
        if self.kind == "rdft":
            shape = tuple(x.shape[:-1]) + (self.n // 2 + 1,)
            y = torch.empty(shape, dtype=torch.complex128 if rdt == torch.float64 else torch.complex64,
                            device=x.device) if out is None else out
            want = self.batch * (self.n // 2 + 1)
        else:
            y = torch.empty_like(x) if out is None else out
            want = self.batch * self.in_len
        if not y.is_cuda or not y.is_contiguous() or y.device != x.device or y.numel() != want:
            raise ValueError("output does not match the plan")
        fn = _lib.load().amqft_exec_adjoint if adjoint else _lib.load().amqft_exec
        _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                      _stream_handle(x.device)), "amqft_exec")
        return y


def _real(kind: str, x: torch.Tensor, n: int, variant: int) -> torch.Tensor:
    x = x.contiguous()
    if x.dtype not in _REAL_DTYPES:
        raise TypeError("real transforms take float32 or float64 tensors")
    batch = x.numel() // x.shape[-1] if x.shape[-1] else 0
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    key = ("real", kind, n, batch, variant, _REAL_DTYPES[x.dtype], dev)
    p = _plan_cache.get(key)
    if p is None:
        with torch.cuda.device(dev):
            p = RealPlan(n, batch, kind, variant, _REAL_DTYPES[x.dtype])
        _plan_cache[key] = p
    return p.exec(x)


def rdft(x: torch.Tensor, variant: int = 4) -> torch.Tensor:
    """R(k), k = 0..n/2, of real signals along the last axis (n = x.shape[-1])."""
    return _real("rdft", x, x.shape[-1], variant)


def dct0(s: torch.Tensor, variant: int = 4) -> torch.Tensor:
    """DCT-0 (eq. qft_0B) of s(0..n/2) along the last axis (n = 2 (len - 1))."""
    return _real("dct0", s, 2 * (s.shape[-1] - 1), variant)


def dst0(s: torch.Tensor, variant: int = 4) -> torch.Tensor:
    """DST-0 (eq. qft_0C) of s(1..n/2-1) along the last axis (n = 2 (len + 1))."""
    return _real("dst0", s, 2 * (s.shape[-1] + 1), variant)
