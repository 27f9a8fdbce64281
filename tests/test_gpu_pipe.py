"""Host-to-host execution in chunks with overlapped transfers (the paper's
end-to-end regime, Sec. 3): results equal the device-resident plan's,
bitwise, and the oracle's within tolerance, for pinned and pageable host
memory, in place, 16-bit storage, several execs on one pipe."""
import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import capi, workloads
from gpu_helpers import from_gpu_16, quantised, rel_l2_rows, require_gpu, tol_fp32, to_gpu_16

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def device_reference(h, x_chunks, dev):
    """The same plan run chunk by chunk on device-resident data."""
    out = []
    st = torch.cuda.current_stream().cuda_stream
    for c in x_chunks:
        xi = c.to(dev)
        yi = torch.empty_like(xi)
        capi.fft_exec(h, xi.data_ptr(), yi.data_ptr(), st)
        torch.cuda.synchronize()
        out.append(yi.cpu())
    return torch.stack(out)


@pytest.mark.parametrize("n,batch,chunks,slots", [(4096, 4, 7, 3), (1 << 16, 2, 5, 2), (64, 128, 20, 2),
                                                  (1 << 20, 1, 3, 3)])
@pytest.mark.parametrize("pinned", [True, False])
def test_pipe_complex64(dev, n, batch, chunks, slots, pinned):
    x = workloads.normal_batch(n, batch * chunks, seed=n + chunks).astype(np.complex64)
    xt = torch.from_numpy(x).reshape(chunks, batch, n)
    if pinned:
        xt = xt.pin_memory()
    out = torch.empty_like(xt)
    if pinned:
        out = out.pin_memory()
    h = capi.fft_plan([n], batch, 1, capi.FFT_C64, capi.FFT_FORWARD)
    p = capi.fft_pipe_create(h, slots)
    try:
        capi.fft_pipe_exec(p, xt.data_ptr(), out.data_ptr(), chunks)
        capi.fft_pipe_wait(p)
        ref_dev = device_reference(h, list(xt), dev)
    finally:
        capi.fft_pipe_destroy(p)
        capi.fft_destroy(h)
    assert torch.equal(out, ref_dev)
    got = out.numpy().reshape(-1, n)
    assert rel_l2_rows(got, oracle.fft(x), n).max() <= tol_fp32(n)


def test_pipe_in_place_and_repeated_execs(dev):
    n, batch, chunks = 2048, 8, 9
    x = workloads.normal_batch(n, batch * chunks, seed=3).astype(np.complex64)
    ref = oracle.fft(x, inverse=True)
    h = capi.fft_plan([n], batch, 1, capi.FFT_C64, capi.FFT_INVERSE)
    p = capi.fft_pipe_create(h, 3)
    try:
        bufs = []
        for _ in range(3):  # three execs queued before one wait
            b = torch.from_numpy(x.copy()).pin_memory()
            capi.fft_pipe_exec(p, b.data_ptr(), b.data_ptr(), chunks)
            bufs.append(b)
        capi.fft_pipe_wait(p)
    finally:
        capi.fft_pipe_destroy(p)
        capi.fft_destroy(h)
    for b in bufs:
        assert rel_l2_rows(b.numpy().reshape(-1, n), ref, n).max() <= tol_fp32(n)
    assert torch.equal(bufs[0], bufs[1]) and torch.equal(bufs[1], bufs[2])


@pytest.mark.parametrize("tname,tol", [("float16", 1e-3), ("bfloat16", 8e-3)])
def test_pipe_16bit(dev, tname, tol):
    tdt = getattr(torch, tname)
    n, batch, chunks = 1024, 16, 6
    x = workloads.normal_batch(n, batch * chunks, seed=16)
    xt = to_gpu_16(x, dev, tdt).cpu().pin_memory()
    out = torch.empty_like(xt).pin_memory()
    h = capi.fft_plan([n], batch, 1, capi.FFT_C16F if tname == "float16" else capi.FFT_C16BF,
                      capi.FFT_FORWARD)
    p = capi.fft_pipe_create(h, 2)
    try:
        capi.fft_pipe_exec(p, xt.data_ptr(), out.data_ptr(), chunks)
        capi.fft_pipe_wait(p)
    finally:
        capi.fft_pipe_destroy(p)
        capi.fft_destroy(h)
    got = from_gpu_16(out).reshape(-1, n)
    assert rel_l2_rows(got, oracle.fft(quantised(x, tdt)), n).max() <= tol


def test_pipe_errors(dev):
    h = capi.fft_plan([256], 2, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        for slots in (0, 1, 65):
            with pytest.raises(capi.FFTError) as ei:
                capi.fft_pipe_create(h, slots)
            assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
        p = capi.fft_pipe_create(h, 2)
        with pytest.raises(capi.FFTError):
            capi.fft_pipe_exec(p, 0, 0, 1)
        with pytest.raises(capi.FFTError):
            capi.fft_pipe_exec(p, 1, 1, -1)
        capi.fft_pipe_exec(p, 0, 0, 0)  # nothing to do
        capi.fft_pipe_wait(p)
        capi.fft_pipe_destroy(p)
    finally:
        capi.fft_destroy(h)
