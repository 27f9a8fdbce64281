"""16-bit storage on the strided plans, the torch-facing wrappers, and
hipGraph capture/replay of strided plans."""
import math

import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import api, capi, workloads
from gpu_helpers import from_gpu_16, quantised, rel_l2_rows, require_gpu, tol_fp32, to_gpu_16, to_gpu_c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL16 = {"float16": 1e-3, "bfloat16": 8e-3}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.mark.parametrize("tname", ["float16", "bfloat16"])
@pytest.mark.parametrize("shape", [(256,), (4096,), (1 << 14,), (1 << 16,), (1 << 20,), (64, 512), (1024, 1024), (4096, 64)])
def test_16bit_storage(dev, tname, shape):
    tdt = getattr(torch, tname)
    n = int(np.prod(shape))
    b = 2
    x = workloads.normal_batch(n, b, seed=n % 1000).reshape((b,) + shape)
    xq = quantised(x, tdt)
    xt = to_gpu_16(x, dev, tdt)
    y = api.fft2(xt) if len(shape) == 2 else api.fft(xt)
    torch.cuda.synchronize()
    got = from_gpu_16(y).reshape(b, -1)
    ref = (oracle.fft2(xq) if len(shape) == 2 else oracle.fft(xq)).reshape(b, -1)
    err = rel_l2_rows(got, ref, n)
    print(f"{tname} {shape}: rel-L2 vs oracle on quantised input {err.max():.3e}")
    assert err.max() <= TOL16[tname], float(err.max())
    # inverse back to the input, same tolerance per direction
    z = api.ifft2(y) if len(shape) == 2 else api.ifft(y)
    torch.cuda.synchronize()
    ref_z = (oracle.fft2(from_gpu_16(y), inverse=True) if len(shape) == 2
             else oracle.ifft(from_gpu_16(y))).reshape(b, -1)
    assert rel_l2_rows(from_gpu_16(z).reshape(b, -1), ref_z, n).max() <= TOL16[tname]


@pytest.mark.parametrize("tname", ["float16", "bfloat16"])
@pytest.mark.parametrize("batch", [3, 16])
def test_16bit_first_pass_two_tiles_in_flight(dev, tname, batch):
    # 2^20 split 1024 x 1024, first pass with two tiles' loads in flight
    tdt = getattr(torch, tname)
    dt = "f16" if tname == "float16" else "bf16"
    sched = f"split=1024;a=a1024p32w16q2_{dt};b=c1024p32w16qx_{dt}"
    n = 1 << 20
    x = workloads.normal_batch(n, batch, seed=batch + 11)
    xq = quantised(x, tdt)
    y = api.fft(to_gpu_16(x, dev, tdt), schedule=sched)
    torch.cuda.synchronize()
    err = rel_l2_rows(from_gpu_16(y).reshape(batch, -1), oracle.fft(xq).reshape(batch, -1), n)
    assert err.max() <= TOL16[tname], float(err.max())


@pytest.mark.parametrize("tname", ["float16", "bfloat16"])
@pytest.mark.parametrize("shape", [(64, 512), (256, 32), (256, 16)])
def test_16bit_three_pass_2d(dev, tname, shape):
    # columns as two sub-passes, forced by the schedule
    tdt = getattr(torch, tname)
    # raises if the shape has no three-pass plan
    capi.fft_describe(list(shape), 3, 2, capi.FFT_C16F if tname == "float16" else capi.FFT_C16BF, "col3=1")
    n = int(np.prod(shape))
    x = workloads.normal_batch(n, 3, seed=7 + n).reshape((3,) + shape)
    xq = quantised(x, tdt)
    y = api.fft2(to_gpu_16(x, dev, tdt), schedule="col3=1")
    torch.cuda.synchronize()
    err = rel_l2_rows(from_gpu_16(y).reshape(3, -1), oracle.fft2(xq).reshape(3, -1), n)
    assert err.max() <= TOL16[tname], float(err.max())


def test_bf16_store_rounds_half_to_even(dev):
    # 2-point transforms X0 = x0 + x1, X1 = x0 - x1 of bf16 inputs: for these
    # pairs both are exact in FP32, so the only rounding is the store to
    # bf16, which must match torch's CPU conversion (nearest, ties to even)
    # bit for bit, halfway cases included
    u = 2.0 ** -8
    pairs = [(1.0, u),                 # 1 + 2^-8: halfway, to 1 (even)
             (1.0 + 2 * u, u),         # 1 + 3 2^-8: halfway, to 1 + 2^-6 (even)
             (1.0, 0.75 * u),          # below halfway: to 1
             (1.0, 1.5 * u),           # above halfway: to 1 + 2^-7
             (-1.0, -u),               # negative halfway
             (3.0, 3 * u),             # halfway at a larger exponent
             (0.5, 2.0 ** -9 + 2.0 ** -16), (1.5, -u), (0.0, 0.0), (-2.0, 3 * u)]
    x = np.array([[a + 1j * b, b - 1j * a] for a, b in pairs])  # rows: (x0, x1)
    xt = to_gpu_16(x, dev, torch.bfloat16)
    assert np.array_equal(from_gpu_16(xt), x)  # the inputs are bf16 values
    y = from_gpu_16(api.fft(xt))
    torch.cuda.synchronize()
    s32 = np.stack([x[:, 0] + x[:, 1], x[:, 0] - x[:, 1]], axis=1)
    pair = np.stack([s32.real, s32.imag], axis=-1)
    assert np.array_equal(pair.astype(np.float32).astype(np.float64), pair)  # exact in FP32
    ref = torch.from_numpy(pair.astype(np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(y, ref[..., 0] + 1j * ref[..., 1])
    assert y[0, 0].real == 1.0 and y[1, 0].real == 1.0 + 2.0 ** -6


def test_f16_store_rounds_half_to_even(dev):
    # as above for float16 (10 fraction bits): ties at 1 + 2^-11 and
    # 1 + 3 2^-11, both signs, and one overflow-free large value
    u = 2.0 ** -11
    pairs = [(1.0, u), (1.0 + 2 * u, u), (1.0, 0.75 * u), (1.0, 1.5 * u), (-1.0, -u),
             (1024.0, 0.5), (1024.0, 1.5), (0.0, 0.0), (-2.0, 3 * u), (0.25, 2.0 ** -14)]
    x = np.array([[a + 1j * b, b - 1j * a] for a, b in pairs])
    xt = to_gpu_16(x, dev, torch.float16)
    assert np.array_equal(from_gpu_16(xt), x)
    y = from_gpu_16(api.fft(xt))
    torch.cuda.synchronize()
    s32 = np.stack([x[:, 0] + x[:, 1], x[:, 0] - x[:, 1]], axis=1)
    pair = np.stack([s32.real, s32.imag], axis=-1)
    assert np.array_equal(pair.astype(np.float32).astype(np.float64), pair)
    ref = pair.astype(np.float16).astype(np.float64)  # numpy: nearest, ties to even
    assert np.array_equal(y, ref[..., 0] + 1j * ref[..., 1])
    assert y[0, 0].real == 1.0 and y[1, 0].real == 1.0 + 2.0 ** -9 and y[5, 0].real == 1024.0


def test_wrappers_match_capi(dev):
    x = workloads.normal_batch(4096, 5, seed=61).astype(np.complex64)
    xt = to_gpu_c64(x, dev)
    y = api.fft(xt)
    z = api.ifft(y)
    torch.cuda.synchronize()
    assert rel_l2_rows(y.cpu().numpy(), oracle.fft(x), 4096).max() <= tol_fp32(4096)
    assert rel_l2_rows(z.cpu().numpy(), x, 4096).max() <= 2 * tol_fp32(4096)
    img = workloads.normal_batch(128 * 256, 2, seed=62).astype(np.complex64).reshape(2, 128, 256)
    it = to_gpu_c64(img, dev)
    y2 = api.fft2(it)
    torch.cuda.synchronize()
    assert rel_l2_rows(y2.cpu().numpy().reshape(2, -1), oracle.fft2(img).reshape(2, -1),
                       128 * 256).max() <= tol_fp32(128 * 256)
    # in place through the wrapper (two-pass 1-D uses a torch-allocated workspace)
    big = to_gpu_c64(workloads.normal_batch(1 << 18, 2, seed=63), dev)
    ref = oracle.fft(big.cpu().numpy())
    api.fft(big, out=big)
    torch.cuda.synchronize()
    assert rel_l2_rows(big.cpu().numpy(), ref, 1 << 18).max() <= tol_fp32(1 << 18)
    with pytest.raises(ValueError):
        api.fft(torch.zeros(16, dtype=torch.complex64))  # CPU tensor: no CPU path


@pytest.mark.parametrize("shape", [(1 << 20,), (4096, 4096), (1024,)])
def test_graph_capture_replay_strided(dev, shape):
    n = int(np.prod(shape))
    b = 2 if n >= (1 << 20) else 16
    x = workloads.normal_batch(n, b, seed=71).astype(np.complex64)
    xt = to_gpu_c64(x, dev)
    out = torch.zeros_like(xt)
    eager = torch.empty_like(xt)
    h = capi.fft_plan(list(shape), b, len(shape), capi.FFT_C64, capi.FFT_FORWARD)
    try:
        capi.fft_exec(h, xt.data_ptr(), eager.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), s.cuda_stream)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(3):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep}"
            capi.fft_exec(h, xt.data_ptr(), eager.data_ptr(), torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
        del g
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("tname", ["float16", "bfloat16"])
def test_16bit_4096x4096_image(dev, tname):
    # the image workload in 16-bit storage (columns as two sub-passes)
    tdt = getattr(torch, tname)
    z = workloads.speckle_image(4096, 4096, seed=2)
    d = capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C16F if tname == "float16" else capi.FFT_C16BF)
    print(f"{tname} 4096x4096 passes: {d['names'][:d['passes']]}")
    y = api.fft2(to_gpu_16(z[None], dev, tdt))
    torch.cuda.synchronize()
    err = rel_l2_rows(from_gpu_16(y).reshape(1, -1), oracle.fft2(quantised(z[None], tdt)).reshape(1, -1),
                      4096 * 4096)
    print(f"{tname} 4096x4096 image rel-L2 {err.max():.3e}")
    assert err.max() <= TOL16[tname], float(err.max())


def test_profiling_skips_graph_capture(dev):
    # timing events stay out of captured graphs; eager execs are still timed
    n, b = 1 << 16, 4
    x = to_gpu_c64(workloads.normal_batch(n, b, seed=5).astype(np.complex64), dev)
    y = torch.empty_like(x)
    h = capi.fft_plan([n], b, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        capi.fft_profile_enable(h, 8)
        capi.fft_exec(h, x.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                capi.fft_exec(h, x.data_ptr(), y.data_ptr(), s.cuda_stream)
        torch.cuda.current_stream().wait_stream(s)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        capi.fft_profile_collect(h)
        ms, count = capi.fft_profile_read(h, 0)
        assert count == 1 and ms > 0
        ref = oracle.fft(x.cpu().numpy())
        assert rel_l2_rows(y.cpu().numpy(), ref, n).max() <= tol_fp32(n)
        del g
    finally:
        capi.fft_destroy(h)


def test_profiling_samples_one_exec_in_k(dev):
    # fft_profile_sample(plan, 3): of 10 execs, the 1st, 4th, 7th and 10th are
    # timed; every exec still computes the transform
    n, b = 1 << 12, 8
    x = to_gpu_c64(workloads.normal_batch(n, b, seed=6).astype(np.complex64), dev)
    h = capi.fft_plan([n], b, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        capi.fft_profile_enable(h, 8)
        capi.fft_profile_sample(h, 3)
        outs = []
        for _ in range(10):
            y = torch.empty_like(x)
            capi.fft_exec(h, x.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
            outs.append(y)
        torch.cuda.synchronize()
        capi.fft_profile_collect(h)
        ms, count = capi.fft_profile_read(h, 0)
        assert count == 4 and ms > 0
        ref = oracle.fft(x.cpu().numpy())
        for y in outs:
            assert rel_l2_rows(y.cpu().numpy(), ref, n).max() <= tol_fp32(n)
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_profile_sample(h, 0)
        assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
    finally:
        capi.fft_destroy(h)


def _variants_16(kind):
    return sorted(capi.fft_variant_name(i) for i in range(capi.fft_variant_count())
                  if capi.fft_variant_name(i).endswith("_" + kind) and "q" in capi.fft_variant_name(i).split("_")[0])


@pytest.mark.parametrize("name", _variants_16("f16") + _variants_16("bf16"))
def test_16bit_persistent_variants(dev, name):
    # every persistent 16-bit variant through a plan that uses it (more tiles
    # than resident workgroups), forward and inverse (the inverse with the
    # XCD remap), against the oracle on the quantised input
    tname = "float16" if name.endswith("_f16") else "bfloat16"
    code = capi.FFT_C16F if tname == "float16" else capi.FFT_C16BF
    tdt = getattr(torch, tname)
    i = [capi.fft_variant_name(k) for k in range(capi.fft_variant_count())].index(name)
    d = capi.fft_variant_describe(i)
    L = d["L"]
    if d["role"] == 1:
        n, sched = L * 512, f"split={L};a={name}"
    else:
        n, sched = 512 * L, f"split=512;b={name}"
    b = 3
    x = workloads.normal_batch(n, b, seed=L + 7)
    xq = quantised(x, tdt)
    xt = to_gpu_16(x, dev, tdt)
    st = torch.cuda.current_stream().cuda_stream
    for direction in (capi.FFT_FORWARD, capi.FFT_INVERSE):
        h = capi.fft_plan_ex([n], b, 1, code, direction,
                             sched + (";xcd=1" if direction == capi.FFT_INVERSE else ""))
        try:
            y = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), y.data_ptr(), st)
            torch.cuda.synchronize()
        finally:
            capi.fft_destroy(h)
        got = from_gpu_16(y).reshape(b, -1)
        ref = oracle.fft(xq, inverse=direction == capi.FFT_INVERSE).reshape(b, -1)
        err = rel_l2_rows(got, ref, n)
        assert err.max() <= TOL16[tname], (name, direction, float(err.max()))
