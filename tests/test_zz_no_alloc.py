"""fft_exec_static (the allocation-free exec: scratch from the library's static
device array) against fft_exec on the same plans, inputs and streams.

Each case runs two calls in a row through the C ABI, the second on a
smaller input than the first, and checks every output bit for bit against
fft_exec of the same plan (the same kernels run on the same values; only
where the scratch lives differs) and against the FP64 oracle within the
FP32 bound.  Also: an exec whose scratch would exceed the array is refused
with FFT_ERR_SCRATCH_LIMIT before anything is queued."""
import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import capi, workloads
from gpu_helpers import rel_l2_rows, require_gpu, to_gpu_c64, tol_fp32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def stream():
    return torch.cuda.current_stream().cuda_stream


def per_transform_max_err(got, ref, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    worst = 0.0
    for i, n in enumerate(sizes):
        g, r = got[off[i]:off[i + 1]], ref[off[i]:off[i + 1]]
        nr = np.linalg.norm(r)
        e = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g)
        worst = max(worst, e / tol_fp32(n))
    return worst


def test_batched_uneven_two_calls(dev):
    # the 512 uneven lengths 2^8..2^16 (queue and completion counters in the
    # static array), then a smaller batched plan; each against fft_exec
    cases = []
    sizes, packed = workloads.uneven_batch(512, 8, 16, seed=3)
    cases.append(([int(v) for v in sizes], packed))
    small = [1 << e for e in (13, 8, 15, 10, 14, 9, 16, 12, 11, 13)]
    cases.append((small, workloads.normal_batch(sum(small), 1, seed=71).reshape(-1)))
    for sizes, packed in cases:
        print(f"batched: {len(sizes)} transforms, {sum(sizes)} points", flush=True)
        xt = to_gpu_c64(packed, dev)
        h = capi.fft_plan_many(sizes, capi.FFT_C64, capi.FFT_FORWARD)
        try:
            ref_out = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), ref_out.data_ptr(), stream())
            torch.cuda.synchronize()
            assert capi.fft_many_watchdog(h) == capi.FFT_OK
            got = torch.full_like(xt, complex(7.0, -7.0))
            capi.fft_exec_static(h, xt.data_ptr(), got.data_ptr(), stream())
            torch.cuda.synchronize()
            assert capi.fft_many_watchdog(h) == capi.FFT_OK
        finally:
            capi.fft_destroy(h)
        g = got.cpu().numpy()
        assert np.array_equal(g, ref_out.cpu().numpy())
        ref = oracle.fft_many(np.asarray(packed, dtype=np.complex64), np.asarray(sizes))
        assert per_transform_max_err(g, ref, sizes) <= 1.0


def test_in_place_two_pass_two_calls(dev):
    # an in-place two-pass exec needs an intermediate of N * batch points:
    # here it lives in the static array; out of place, fft_exec needs none
    for n, batch, sched in ((1 << 16, 8, None), (1 << 13, 3, "split=128")):
        print(f"in place: N={n} batch={batch} {sched}", flush=True)
        x = workloads.normal_batch(n, batch, seed=n + batch).astype(np.complex64)
        h = capi.fft_plan_ex([n], batch, 1, capi.FFT_C64, capi.FFT_FORWARD, sched)
        try:
            assert capi.fft_plan_info(h)["passes"] == 2
            xt = to_gpu_c64(x, dev)
            ref_out = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), ref_out.data_ptr(), stream())
            buf = to_gpu_c64(x, dev)
            capi.fft_exec_static(h, buf.data_ptr(), buf.data_ptr(), stream())
            torch.cuda.synchronize()
        finally:
            capi.fft_destroy(h)
        g = buf.cpu().numpy()
        assert np.array_equal(g, ref_out.cpu().numpy())
        assert rel_l2_rows(g, oracle.fft(x), n).max() <= tol_fp32(n)


def test_three_pass_two_calls(dev):
    # a three-pass plan always writes its intermediate to a workspace: the
    # plan's own for fft_exec, the static array for fft_exec_static
    for n, batch, sched in ((1 << 18, 4, "split=1024;split2=16"), (1 << 14, 2, "split=64;split2=16")):
        print(f"three pass: N={n} batch={batch} {sched}", flush=True)
        x = workloads.normal_batch(n, batch, seed=n + 7).astype(np.complex64)
        h = capi.fft_plan_ex([n], batch, 1, capi.FFT_C64, capi.FFT_INVERSE, sched)
        try:
            assert capi.fft_plan_info(h)["passes"] == 3
            xt = to_gpu_c64(x, dev)
            ref_out = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), ref_out.data_ptr(), stream())
            got = torch.empty_like(xt)
            capi.fft_exec_static(h, xt.data_ptr(), got.data_ptr(), stream())
            torch.cuda.synchronize()
        finally:
            capi.fft_destroy(h)
        g = got.cpu().numpy()
        assert np.array_equal(g, ref_out.cpu().numpy())
        assert rel_l2_rows(g, oracle.fft(x, inverse=True), n).max() <= tol_fp32(n)


def test_no_scratch_needed_and_limit(dev):
    # a one-pass plan needs no scratch: the same results as fft_exec
    x = workloads.normal_batch(1024, 5, seed=73).astype(np.complex64)
    h = capi.fft_plan([1024], 5, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        xt = to_gpu_c64(x, dev)
        a, b = torch.empty_like(xt), torch.empty_like(xt)
        capi.fft_exec(h, xt.data_ptr(), a.data_ptr(), stream())
        capi.fft_exec_static(h, xt.data_ptr(), b.data_ptr(), stream())
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    finally:
        capi.fft_destroy(h)
    # in place, 2^20 x 8 complex64 would need 64 MiB of intermediate: refused
    # with nothing queued (the buffer keeps its values)
    n, batch = 1 << 20, 8
    assert n * batch * 8 > (32 << 20)
    h = capi.fft_plan([n], batch, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        buf = torch.ones(n * batch, dtype=torch.complex64, device=dev)
        rc = capi.fft_exec_static_status(h, buf.data_ptr(), buf.data_ptr(), stream())
        torch.cuda.synchronize()
        assert rc == capi.FFT_ERR_SCRATCH_LIMIT
        assert "scratch" in capi.error_string(rc)
        assert bool(torch.all(buf == 1))
    finally:
        capi.fft_destroy(h)
