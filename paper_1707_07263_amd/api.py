"""torch-facing helpers over the C ABI: plan cache, fft / ifft / fft2 /
fft_many, and the differentiable transform.

torch supplies device memory and streams only; every transform runs in the
library's HIP kernels.  Complex64 data are ``torch.complex64`` tensors;
16-bit data are real ``torch.float16`` / ``torch.bfloat16`` tensors with a
trailing dimension of 2 (re, im), since torch has no complex bfloat16.
"""
from __future__ import annotations

import threading

import torch

from . import autotune, capi

_DT = {torch.complex64: capi.FFT_C64, torch.float16: capi.FFT_C16F, torch.bfloat16: capi.FFT_C16BF}


class Plan:
    """Owns one library plan handle."""

    def __init__(self, handle: int, kind: str):
        self.handle = handle
        self.kind = kind
        self.workspace = None  # torch tensor backing a caller-owned workspace
        # batched plans whose kernel waits on completion counters (the
        # two-launch kernel never waits)
        self.waits = kind == "many" and capi.fft_plan_info(handle)["pass_variant"][0] != "many_2launch"

    def __del__(self):
        try:
            capi.fft_destroy(self.handle)
        except Exception:
            pass

    def info(self) -> dict:
        return capi.fft_plan_info(self.handle)

    def exec(self, x: torch.Tensor, out: torch.Tensor, stream: int | None = None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        capi.fft_exec(self.handle, x.data_ptr(), out.data_ptr(), stream)

    def set_scale(self, s: float) -> None:
        capi.fft_set_scale(self.handle, s)

    def ensure_workspace(self, device) -> None:
        need = capi.fft_workspace_size(self.handle)
        if need and (self.workspace is None or self.workspace.numel() < need):
            self.workspace = torch.empty(need, dtype=torch.uint8, device=device)
            capi.fft_set_workspace(self.handle, self.workspace.data_ptr(), need)


_cache: dict = {}
_lock = threading.Lock()


def get_plan(shape, batch: int, dtype: int, direction: int, *, scale=None,
             schedule: str | None = None, device=None) -> Plan:
    """Cached plan for `batch` transforms of `shape` (1 or 2 dims)."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    if schedule is None:
        schedule = autotune.schedule_for(shape, batch, dtype)
    key = ("plan", tuple(int(s) for s in shape), int(batch), dtype, direction, scale, schedule, dev)
    with _lock:
        p = _cache.get(key)
        if p is None:
            with torch.cuda.device(dev):
                h = capi.fft_plan_ex(list(shape), batch, len(shape), dtype, direction, schedule)
                p = Plan(h, "strided")
                if scale is not None:
                    p.set_scale(scale)
            _cache[key] = p
    return p


def get_many_plan(sizes, dtype: int, direction: int, *, scale=None, schedule=None,
                  device=None) -> Plan:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    if schedule is None:
        schedule = autotune.many_schedule_for(sizes, dtype)
    key = ("many", tuple(int(s) for s in sizes), dtype, direction, scale, schedule, dev)
    with _lock:
        p = _cache.get(key)
        if p is None:
            with torch.cuda.device(dev):
                h = capi.fft_plan_many_ex([int(s) for s in sizes], dtype, direction, schedule)
                p = Plan(h, "many")
                if scale is not None:
                    p.set_scale(scale)
            _cache[key] = p
    return p


def clear_cache() -> None:
    with _lock:
        _cache.clear()


def _check_input(x: torch.Tensor, ndim_fft: int):
    if not x.is_cuda:
        raise ValueError("input must be a GPU tensor (the transforms run in HIP kernels only)")
    if x.dtype == torch.complex64:
        shape = x.shape[x.dim() - ndim_fft:]
        lead = x.shape[:x.dim() - ndim_fft]
    elif x.dtype in (torch.float16, torch.bfloat16):
        if x.shape[-1] != 2:
            raise ValueError("16-bit complex data need a trailing dimension of 2 (re, im)")
        shape = x.shape[x.dim() - 1 - ndim_fft:x.dim() - 1]
        lead = x.shape[:x.dim() - 1 - ndim_fft]
    else:
        raise ValueError(f"unsupported dtype {x.dtype}")
    if len(shape) != ndim_fft:
        raise ValueError("input has too few dimensions")
    batch = 1
    for s in lead:
        batch *= int(s)
    return list(shape), batch


def _run(x, ndim_fft, inverse, scale, out, schedule):
    shape, batch = _check_input(x, ndim_fft)
    x = x.contiguous()
    direction = capi.FFT_INVERSE if inverse else capi.FFT_FORWARD
    plan = get_plan(shape, batch, _DT[x.dtype], direction, scale=scale, schedule=schedule,
                    device=x.device)
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the input's shape and dtype")
    if out.data_ptr() == x.data_ptr():
        plan.ensure_workspace(x.device)
    plan.exec(x, out)
    return out


def fft(x: torch.Tensor, inverse: bool = False, *, scale: float | None = None,
        out: torch.Tensor | None = None, schedule: str | None = None) -> torch.Tensor:
    """1-D transform along the last axis (eq. 1; with inverse=True eq. 2)."""
    return _run(x, 1, inverse, scale, out, schedule)


def ifft(x: torch.Tensor, **kw) -> torch.Tensor:
    return fft(x, inverse=True, **kw)


def fft2(x: torch.Tensor, inverse: bool = False, *, scale: float | None = None,
         out: torch.Tensor | None = None, schedule: str | None = None) -> torch.Tensor:
    """2-D transform over the last two axes: rows, then columns."""
    return _run(x, 2, inverse, scale, out, schedule)


def ifft2(x: torch.Tensor, **kw) -> torch.Tensor:
    return fft2(x, inverse=True, **kw)


def fft_many(packed: torch.Tensor, sizes, inverse: bool = False, *, scale=None,
             out: torch.Tensor | None = None, schedule: str | None = None) -> torch.Tensor:
    """Independent 1-D transforms of lengths `sizes` packed back to back, in
    one persistent launch."""
    if not packed.is_cuda:
        raise ValueError("input must be a GPU tensor")
    if packed.dtype not in _DT:
        raise ValueError(f"unsupported dtype {packed.dtype}")
    packed = packed.contiguous()
    total = packed.numel() if packed.dtype == torch.complex64 else packed.numel() // 2
    if sum(int(s) for s in sizes) != total:
        raise ValueError("sizes do not add up to the packed length")
    direction = capi.FFT_INVERSE if inverse else capi.FFT_FORWARD
    plan = get_many_plan(sizes, _DT[packed.dtype], direction, scale=scale, schedule=schedule,
                         device=packed.device)
    if out is None:
        out = torch.empty_like(packed)
    elif out.shape != packed.shape or out.dtype != packed.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of the packed input's shape and dtype")
    plan.exec(packed, out)
    if plan.waits:
        # kernels whose second passes wait on completion counters: a wait that
        # ran out (e.g. workgroups that were not resident) leaves wrong
        # results, so read the flag (this synchronises)
        if capi.fft_many_watchdog(plan.handle, clear=True) == capi.FFT_ERR_WATCHDOG:
            raise RuntimeError("fft_many: a dependency wait expired; the results are invalid")
    return out


class FFTFunction(torch.autograd.Function):
    """y = F x along the last axis (eq. 1, unscaled), differentiable.

    For a real loss torch passes grad_y = dL/dRe(y) + i dL/dIm(y); since F is
    linear and holomorphic, grad_x = F^H grad_y, the inverse-direction
    transform with scale 1 (the adjoint), run by the same HIP kernels.
    """

    @staticmethod
    def forward(ctx, x):
        if x.dtype != torch.complex64:
            raise ValueError("FFTFunction takes complex64 input")
        return fft(x)

    @staticmethod
    def backward(ctx, g):
        return fft(g.contiguous(), inverse=True, scale=1.0)


def fft_autograd(x: torch.Tensor) -> torch.Tensor:
    return FFTFunction.apply(x)


def variants() -> list:
    out = []
    for i in range(capi.fft_variant_count()):
        d = capi.fft_variant_describe(i)
        d["name"] = capi.fft_variant_name(i)
        out.append(d)
    return out
