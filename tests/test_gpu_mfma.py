"""The matrix-core experiment: 256-point transforms whose two radix-16
stages are 16 x 16 complex matrix products on FP32 MFMA (method=mfma),
against the FP64 oracle: ragged batches (whole and partial workgroups),
both directions, caller scale."""
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


def run(x, dev, inverse=False, scale=None):
    xt = to_gpu_c64(x, dev)
    batch = xt.numel() // 256
    h = capi.fft_plan_ex([256], batch, 1, capi.FFT_C64, capi.FFT_INVERSE if inverse else capi.FFT_FORWARD,
                         "method=mfma")
    try:
        assert capi.fft_plan_info(h)["pass_variant"] == ["mfma_dft256"]
        if scale is not None:
            capi.fft_set_scale(h, scale)
        out = torch.empty_like(xt)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("batch", [1, 3, 4, 5, 1023, 65536])
@pytest.mark.parametrize("inverse", [False, True])
def test_mfma_256_parity(dev, batch, inverse):
    x = workloads.normal_batch(256, batch, seed=batch).astype(np.complex64)
    got = run(x, dev, inverse=inverse)
    ref = oracle.fft(x, inverse=inverse)
    err = rel_l2_rows(got, ref, 256)
    assert err.max() <= tol_fp32(256), float(err.max())


def test_mfma_256_closed_forms_and_scale(dev):
    # impulses at every position: row n0 of the DFT matrix (eq. 1)
    x = np.eye(256, dtype=np.complex64)
    got = run(x, dev)
    k = np.arange(256)
    want = np.exp(-2j * np.pi * ((k[:, None] * k[None, :]) % 256) / 256)
    assert np.max(np.abs(got - want)) < 2e-6
    y = workloads.normal_batch(256, 7, seed=9).astype(np.complex64)
    got = run(y, dev, inverse=True, scale=1.0)
    assert rel_l2_rows(got, oracle.fft(y, inverse=True, scale=1.0), 256).max() <= tol_fp32(256)
