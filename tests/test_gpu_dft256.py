"""The one-kernel 256-point experiments (256 = 16 x 16, eq. 5) against the
FP64 oracle: the two radix-16 stages as 16 x 16 complex matrix products on
FP32 MFMA (method=mfma), and the exchange between the stages as cross-lane
moves, DPP and ds_swizzle (method=xlane) or ds_bpermute (xlane_bperm).
Ragged batches (whole and partial workgroups), both directions, caller
scale."""
import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import capi, workloads
from gpu_helpers import rel_l2_rows, require_gpu, tol_fp32, to_gpu_c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


METHODS = {"mfma": "mfma_dft256", "xlane": "xlane_dft256", "xlane_bperm": "xlane_bperm_dft256"}


def run(x, dev, method, inverse=False, scale=None):
    xt = to_gpu_c64(x, dev)
    batch = xt.numel() // 256
    h = capi.fft_plan_ex([256], batch, 1, capi.FFT_C64, capi.FFT_INVERSE if inverse else capi.FFT_FORWARD,
                         f"method={method}")
    try:
        assert capi.fft_plan_info(h)["pass_variant"] == [METHODS[method]]
        if scale is not None:
            capi.fft_set_scale(h, scale)
        out = torch.empty_like(xt)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("batch", [1, 3, 4, 5, 17, 1023, 65536])
@pytest.mark.parametrize("inverse", [False, True])
def test_dft256_parity(dev, method, batch, inverse):
    x = workloads.normal_batch(256, batch, seed=batch).astype(np.complex64)
    got = run(x, dev, method, inverse=inverse)
    ref = oracle.fft(x, inverse=inverse)
    err = rel_l2_rows(got, ref, 256)
    assert err.max() <= tol_fp32(256), float(err.max())


@pytest.mark.parametrize("method", list(METHODS))
def test_dft256_closed_forms_and_scale(dev, method):
    # impulses at every position: row n0 of the DFT matrix (eq. 1)
    x = np.eye(256, dtype=np.complex64)
    got = run(x, dev, method)
    k = np.arange(256)
    want = np.exp(-2j * np.pi * ((k[:, None] * k[None, :]) % 256) / 256)
    assert np.max(np.abs(got - want)) < 2e-6
    y = workloads.normal_batch(256, 7, seed=9).astype(np.complex64)
    got = run(y, dev, method, inverse=True, scale=1.0)
    assert rel_l2_rows(got, oracle.fft(y, inverse=True, scale=1.0), 256).max() <= tol_fp32(256)
