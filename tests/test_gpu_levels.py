"""The per-level global-memory method (one radix-2 kernel per butterfly
level, Sec. 2.2) kept as an ablation: parity with the FP64 oracle through
the C ABI, both directions, in place, caller scale and 16-bit storage."""
import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import capi, workloads
from gpu_helpers import from_gpu_16, quantised, rel_l2_rows, require_gpu, tol_fp32, to_gpu_16, to_gpu_c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LEVELS = "method=levels"


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def run(x, n, dev, inverse=False, inplace=False, scale=None):
    xt = to_gpu_c64(x, dev)
    batch = xt.numel() // n
    h = capi.fft_plan_ex([n], batch, 1, capi.FFT_C64,
                         capi.FFT_INVERSE if inverse else capi.FFT_FORWARD, LEVELS)
    try:
        if scale is not None:
            capi.fft_set_scale(h, scale)
        assert capi.fft_plan_info(h)["pass_variant"] == ["levels_radix2"]
        out = xt if inplace else torch.empty_like(xt)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("lg", list(range(1, 17)) + [20])
@pytest.mark.parametrize("inverse", [False, True])
def test_levels_parity(dev, lg, inverse):
    n = 1 << lg
    b = 3 if lg <= 16 else 2
    x = workloads.normal_batch(n, b, seed=300 + lg).astype(np.complex64)
    got = run(x, n, dev, inverse=inverse)
    ref = oracle.fft(x, inverse=inverse)
    assert rel_l2_rows(got, ref, n).max() <= tol_fp32(n)


@pytest.mark.parametrize("lg", [9, 10])  # odd and even level counts
def test_levels_in_place_and_scale(dev, lg):
    n = 1 << lg
    x = workloads.normal_batch(n, 4, seed=lg).astype(np.complex64)
    got = run(x, n, dev, inplace=True)
    assert rel_l2_rows(got, oracle.fft(x), n).max() <= tol_fp32(n)
    got = run(x, n, dev, inverse=True, scale=0.25)
    assert rel_l2_rows(got, oracle.fft(x, inverse=True, scale=0.25), n).max() <= tol_fp32(n)


@pytest.mark.parametrize("tname,tol", [("float16", 1e-3), ("bfloat16", 8e-3)])
def test_levels_16bit(dev, tname, tol):
    tdt = getattr(torch, tname)
    n = 1 << 12
    x = workloads.normal_batch(n, 2, seed=12)
    xt = to_gpu_16(x, dev, tdt)
    h = capi.fft_plan_ex([n], 2, 1, capi.FFT_C16F if tname == "float16" else capi.FFT_C16BF,
                         capi.FFT_FORWARD, LEVELS)
    try:
        out = torch.empty_like(xt)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        capi.fft_destroy(h)
    got = from_gpu_16(out).reshape(2, -1)
    assert rel_l2_rows(got, oracle.fft(quantised(x, tdt)), n).max() <= tol
