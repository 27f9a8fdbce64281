"""Shared helpers for the GPU tests (not collected by pytest)."""
import math

import numpy as np
import pytest

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


def require_gpu():
    if torch is None or not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU (select with -m 'not gpu' on CPU hosts)")
    from paper_1707_07263_amd import capi
    capi.load()  # fails loudly if the HIP library is missing
    return torch.device("cuda:0")


def rel_l2_rows(got, ref, n):
    """Per-transform relative L2 error (FP64 sums); rows of length n."""
    g = np.asarray(got, dtype=np.complex128).reshape(-1, n)
    r = np.asarray(ref, dtype=np.complex128).reshape(-1, n)
    num = np.sqrt(np.sum(np.abs(g - r) ** 2, axis=1))
    den = np.sqrt(np.sum(np.abs(r) ** 2, axis=1))
    out = np.where(den > 0, num / np.where(den > 0, den, 1), num)
    return out


def tol_fp32(n_total):
    """rel-L2 bound for the FP32 path: 1e-6 * log2(N) (at least 1e-6)."""
    return 1e-6 * max(1.0, math.log2(max(n_total, 1)))


def to_gpu_c64(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to(dev)


def to_gpu_16(x, dev, dt):
    """complex array -> [..., 2] 16-bit tensor (round to nearest even)."""
    a = np.ascontiguousarray(x, dtype=np.complex128)
    pair = np.stack([a.real, a.imag], axis=-1)
    t = torch.from_numpy(pair.astype(np.float32)).to(dt)
    return t.to(dev)


def from_gpu_16(t):
    a = t.float().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def quantised(x, dt):
    """The value a 16-bit tensor actually holds, as complex128 (oracle input)."""
    pair = np.stack([np.asarray(x).real, np.asarray(x).imag], axis=-1).astype(np.float32)
    t = torch.from_numpy(pair).to(dt).float().numpy().astype(np.float64)
    return t[..., 0] + 1j * t[..., 1]
