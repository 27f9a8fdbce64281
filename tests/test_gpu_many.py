"""Batched uneven sizes in one persistent launch (fft_plan_many) vs the FP64
oracle, in complex64 and in FP16/BF16 storage; graph capture and replay;
the bounded wait; error paths."""
import math

import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import capi, workloads
from gpu_helpers import from_gpu_16, quantised, rel_l2_rows, require_gpu, to_gpu_16, to_gpu_c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DT16 = {"f16": (capi.FFT_C16F, "float16"), "bf16": (capi.FFT_C16BF, "bfloat16")}
TOL16 = {"f16": 1e-3, "bf16": 8e-3}


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def per_transform_errors(got, ref, sizes):
    off = offsets(sizes)
    errs = np.empty(len(sizes))
    for i in range(len(sizes)):
        g, r = got[off[i]:off[i + 1]], ref[off[i]:off[i + 1]]
        nr = np.linalg.norm(r)
        errs[i] = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g)
    return errs


def run_many_c64(packed, sizes, dev, inverse=False, schedule=None, scale=None):
    xt = to_gpu_c64(packed, dev)
    out = torch.empty_like(xt)
    h = capi.fft_plan_many_ex(list(sizes), capi.FFT_C64,
                              capi.FFT_INVERSE if inverse else capi.FFT_FORWARD, schedule)
    try:
        if scale is not None:
            capi.fft_set_scale(h, scale)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert capi.fft_many_watchdog(h) == capi.FFT_OK
    finally:
        capi.fft_destroy(h)
    return out.cpu().numpy()


def report(name, sizes, errs):
    lines = [f"{name}: per-size max rel-L2"]
    for lg in sorted(set(int(math.log2(s)) for s in sizes)):
        sel = [i for i, s in enumerate(sizes) if int(math.log2(s)) == lg]
        lines.append(f"  2^{lg}: n={len(sel)} max={errs[sel].max():.3e}")
    print("\n".join(lines))


@pytest.mark.parametrize("which", ["built-in", "tuned"])
def test_uneven_512_complex64(dev, which):
    from paper_1707_07263_amd import autotune
    sizes, packed = workloads.uneven_batch(512, 8, 16, seed=3)
    sched = autotune.many_schedule_for(sizes, capi.FFT_C64) if which == "tuned" else None
    xc = packed.astype(np.complex64)
    got = run_many_c64(xc, sizes, dev, schedule=sched)
    ref = oracle.fft_many(xc, sizes)
    errs = per_transform_errors(got, ref, sizes)
    report("512 uneven complex64", sizes, errs)
    tol = 1e-6 * np.log2(sizes.astype(np.float64))
    assert np.all(errs <= tol), float((errs / tol).max())
    inv = run_many_c64(got, sizes, dev, inverse=True)
    ref_inv = oracle.fft_many(got, sizes, inverse=True)
    assert np.all(per_transform_errors(inv, ref_inv, sizes) <= tol)


@pytest.mark.parametrize("pipe", [None, "pipe=1;threads=512", "pipe=1;threads=256", "pipe=2;threads=512",
                                  "pipe=2;threads=256;ntst=1", "pipe=2;threads=512;ntail=200"])
@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_uneven_512_16bit(dev, dt, pipe):
    code, tname = DT16[dt]
    tdt = getattr(torch, tname)
    sizes, packed = workloads.uneven_batch(512, 8, 16, seed=3)
    xq = quantised(packed, tdt)                      # the values the GPU actually holds
    xt = to_gpu_16(packed, dev, tdt)
    out = torch.empty_like(xt)
    from paper_1707_07263_amd import autotune
    h = capi.fft_plan_many_ex(list(sizes), code, capi.FFT_FORWARD,
                              pipe if pipe else autotune.many_schedule_for(sizes, code))
    try:
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert capi.fft_many_watchdog(h) == capi.FFT_OK  # no dependency wait ran out
    finally:
        capi.fft_destroy(h)
    got = from_gpu_16(out)
    ref = oracle.fft_many(xq, sizes)
    errs = per_transform_errors(got, ref, sizes)
    report(f"512 uneven {dt} (vs oracle on the quantised input)", sizes, errs)
    assert errs.max() <= TOL16[dt], float(errs.max())
    # end-to-end error against the unquantised input, reported only
    e2e = per_transform_errors(got, oracle.fft_many(packed, sizes), sizes)
    print(f"512 uneven {dt} end-to-end vs unquantised input: max {e2e.max():.3e}")


@pytest.mark.parametrize("schedule", [None, "pipe=0;threads=256;p=8", "pipe=0;threads=256;pass2=10",
                                      "pipe=0;threads=256;pass2=13;order=given", "pipe=0;threads=512",
                                      "pipe=0;threads=256;pass2=1", "pipe=0;threads=256;lag=1",
                                      "pipe=0;threads=256;lag=3;pass2=9",
                                      "pipe=1;threads=512", "pipe=1;threads=512;pass2=1",
                                      "pipe=1;threads=512;pass2=9;lag=2", "pipe=1;threads=256",
                                      "pipe=1;threads=256;pass2=3", "pipe=2;threads=512",
                                      "pipe=2;threads=512;pass2=1", "pipe=2;threads=512;pass2=9",
                                      "pipe=2;threads=512;pass.11=2;pass.12=2;n1.16=6;n1.15=9;n1.14=7",
                                      "pipe=2;threads=256", "pipe=2;threads=256;ntst=1;pass2=9",
                                      "pipe=2;threads=512;ntst=1", "pipe=2;threads=512;ntail=40",
                                      "pipe=0;threads=512;n1.16=10;pass.9=2;n1.5=2"])
def test_many_schedules_and_small_sizes(dev, schedule):
    # every length 2^0..2^16 twice, shuffled, under each compiled schedule
    g = workloads.rng(77)
    sizes = np.array([1 << e for e in list(range(0, 17)) * 2], dtype=np.int64)
    g.shuffle(sizes)
    packed = np.concatenate([workloads.normal_batch(int(n), 1, seed=int(n) + 5)[0] for n in sizes])
    xc = packed.astype(np.complex64)
    got = run_many_c64(xc, sizes, dev, schedule=schedule)
    ref = oracle.fft_many(xc, sizes)
    errs = per_transform_errors(got, ref, sizes)
    tol = 1e-6 * np.maximum(1.0, np.log2(sizes.astype(np.float64)))
    assert np.all(errs <= tol), (schedule, float((errs / tol).max()))


@pytest.mark.parametrize("schedule", ["pipe=0;threads=256;lag=0", "pipe=0;threads=256;lag=2",
                                      "pipe=0;threads=512;lag=1", "pipe=1;threads=512",
                                      "pipe=1;threads=256", "pipe=2;threads=512"])
def test_many_16x2p20_lagged_queue(dev, schedule):
    # sixteen 2^20-point transforms in one launch, second passes interleaved
    # with later first passes
    sizes = np.array([1 << 20] * 16, dtype=np.int64)
    x = workloads.normal_batch(1 << 20, 16, seed=88).astype(np.complex64)
    got = run_many_c64(x.reshape(-1), sizes, dev, schedule=schedule)
    ref = oracle.fft(x).reshape(-1)
    errs = per_transform_errors(got, ref, sizes)
    assert errs.max() <= 1e-6 * 20, (schedule, float(errs.max()))


def test_many_inverse_scale_and_repeat(dev):
    sizes, packed = workloads.uneven_batch(64, 6, 15, seed=21)
    xc = packed.astype(np.complex64)
    adj = run_many_c64(xc, sizes, dev, inverse=True, scale=1.0)
    ref = oracle.fft_many(xc, sizes, inverse=True, scale=1.0)
    tol = 1e-6 * np.log2(sizes.astype(np.float64))
    assert np.all(per_transform_errors(adj, ref, sizes) <= tol)
    # the queue state resets itself: repeated execs of one plan agree bitwise
    xt = to_gpu_c64(xc, dev)
    h = capi.fft_plan_many(list(sizes), capi.FFT_C64, capi.FFT_FORWARD)
    try:
        outs = []
        for _ in range(4):
            o = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), o.data_ptr(), torch.cuda.current_stream().cuda_stream)
            outs.append(o)
        torch.cuda.synchronize()
        for o in outs[1:]:
            assert torch.equal(o, outs[0])
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("schedule", [None, "pipe=1;threads=512", "pipe=1;threads=256", "pipe=2;threads=512",
                                      "pipe=2;threads=256;ntst=1"])
def test_many_graph_capture_replay(dev, schedule):
    sizes, packed = workloads.uneven_batch(128, 8, 16, seed=31)
    xt = to_gpu_c64(packed, dev)
    out = torch.zeros_like(xt)
    eager = torch.empty_like(xt)
    h = capi.fft_plan_many_ex(list(sizes), capi.FFT_C64, capi.FFT_FORWARD, schedule)
    try:
        st = torch.cuda.current_stream().cuda_stream
        capi.fft_exec(h, xt.data_ptr(), eager.data_ptr(), st)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), s.cuda_stream)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(4):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep} differs from eager"
            # eager work between replays
            capi.fft_exec(h, xt.data_ptr(), eager.data_ptr(), st)
            torch.cuda.synchronize()
        assert capi.fft_many_watchdog(h) == capi.FFT_OK
        del g
    finally:
        capi.fft_destroy(h)


@pytest.mark.parametrize("schedule", [None, "pipe=1;threads=512", "pipe=1;threads=256"])
def test_many_bounded_wait_forced_from_host(dev, schedule):
    # A wait bound of 1 us makes a second-pass tile give up early when its
    # first-pass tiles are still running; the kernel must still finish, the
    # flag must report it (when it happened) and a normal run afterwards must
    # be correct.
    sizes = np.array([1 << 16] * 64, dtype=np.int64)
    packed = workloads.normal_batch(1 << 16, 64, seed=41).reshape(-1)
    xt = to_gpu_c64(packed, dev)
    out = torch.empty_like(xt)
    h = capi.fft_plan_many_ex(list(sizes), capi.FFT_C64, capi.FFT_FORWARD, schedule)
    try:
        capi.fft_many_set_wait_limit(h, 1)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        st = capi.fft_many_watchdog(h, clear=True)
        assert st in (capi.FFT_OK, capi.FFT_ERR_WATCHDOG)
        print("forced short wait:", "expired" if st else "not needed")
        capi.fft_many_set_wait_limit(h, 2000000)
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert capi.fft_many_watchdog(h) == capi.FFT_OK
    finally:
        capi.fft_destroy(h)
    ref = oracle.fft_many(packed.astype(np.complex64), sizes)
    errs = per_transform_errors(out.cpu().numpy(), ref, sizes)
    assert errs.max() <= 1e-6 * 16


def test_many_errors(dev):
    xt = torch.zeros(1 << 16, dtype=torch.complex64, device=dev)
    h = capi.fft_plan_many([1 << 15, 1 << 15], capi.FFT_C64, capi.FFT_FORWARD)
    try:
        assert capi.fft_exec_status(h, xt.data_ptr(), xt.data_ptr(), 0) == capi.FFT_ERR_INPLACE
        # partially overlapping buffers are refused before any launch
        wide = torch.zeros((1 << 16) + 8, dtype=torch.complex64, device=dev)
        assert capi.fft_exec_status(h, wide.data_ptr(), wide.data_ptr() + 64, 0) == capi.FFT_ERR_INPLACE
    finally:
        capi.fft_destroy(h)
    for sizes, code in (([3], capi.FFT_ERR_UNSUPPORTED_SIZE), ([1 << 25], capi.FFT_ERR_UNSUPPORTED_SIZE)):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_plan_many(sizes, capi.FFT_C64, capi.FFT_FORWARD)
        assert ei.value.status == code
    with pytest.raises(capi.FFTError) as ei:
        capi.fft_plan_many_ex([16], capi.FFT_C64, capi.FFT_FORWARD, "p=7")
    assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
    # one-pass-only plans may run in place
    sizes = [256, 1024, 64]
    x = workloads.normal_batch(1344, 1, seed=3)[0]
    xt = to_gpu_c64(x, dev)
    h = capi.fft_plan_many(sizes, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        capi.fft_exec(h, xt.data_ptr(), xt.data_ptr(), 0)
        torch.cuda.synchronize()
    finally:
        capi.fft_destroy(h)
    ref = oracle.fft_many(x.astype(np.complex64), sizes)
    assert per_transform_errors(xt.cpu().numpy(), ref, np.array(sizes)).max() <= 1e-5


@pytest.mark.parametrize("schedule", ["pipe=2;threads=512", "pipe=2;threads=512;pass2=9",
                                      "pipe=2;threads=256;ntst=1", "pipe=2;threads=512;ntail=300"])
def test_many_two_launch_repeat_inverse_inplace(dev, schedule):
    # two launches per exec: repeated execs of one plan agree bitwise (each
    # launch resets its own queue head), the inverse with the default and a
    # caller scale matches the oracle, and a batch of one-pass lengths runs
    # in place (one launch)
    sizes, packed = workloads.uneven_batch(200, 4, 16, seed=23)
    xc = packed.astype(np.complex64)
    xt = to_gpu_c64(xc, dev)
    h = capi.fft_plan_many_ex(list(sizes), capi.FFT_C64, capi.FFT_FORWARD, schedule)
    try:
        outs = []
        for _ in range(3):
            o = torch.empty_like(xt)
            capi.fft_exec(h, xt.data_ptr(), o.data_ptr(), torch.cuda.current_stream().cuda_stream)
            outs.append(o)
        torch.cuda.synchronize()
        for o in outs[1:]:
            assert torch.equal(o, outs[0])
        got = outs[0].cpu().numpy()
    finally:
        capi.fft_destroy(h)
    tol = 1e-6 * np.maximum(1.0, np.log2(sizes.astype(np.float64)))
    assert np.all(per_transform_errors(got, oracle.fft_many(xc, sizes), sizes) <= tol)
    inv = run_many_c64(got, sizes, dev, inverse=True, schedule=schedule)
    assert np.all(per_transform_errors(inv, oracle.fft_many(got, sizes, inverse=True), sizes) <= tol)
    adj = run_many_c64(xc, sizes, dev, inverse=True, scale=1.0, schedule=schedule)
    assert np.all(per_transform_errors(adj, oracle.fft_many(xc, sizes, inverse=True, scale=1.0), sizes) <= tol)
    one = np.array([1 << e for e in (8, 6, 7, 3, 5, 1, 8, 4)], dtype=np.int64)  # one pass under both
    x1 = workloads.normal_batch(int(one.sum()), 1, seed=5)[0].astype(np.complex64)
    b = to_gpu_c64(x1, dev)
    h = capi.fft_plan_many_ex(list(one), capi.FFT_C64, capi.FFT_FORWARD, schedule)
    try:
        capi.fft_exec(h, b.data_ptr(), b.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        capi.fft_destroy(h)
    tol1 = 1e-6 * np.maximum(1.0, np.log2(one.astype(np.float64)))
    assert np.all(per_transform_errors(b.cpu().numpy(), oracle.fft_many(x1, one), one) <= tol1)
