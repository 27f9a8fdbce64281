"""GPU vs FP64-oracle parity for the strided (non-batched-uneven) plans.

Every case runs through the C ABI (fft_plan / fft_exec via ctypes) on seeded
inputs and compares each transform with the oracle: rel-L2 <= 1e-6*log2(N)
for the FP32 path.
"""
import math
import re

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


def run_c64(x, shape, inverse=False, schedule=None, scale=None, inplace=False, dev=None):
    """Plan + exec through the C ABI; returns the numpy result."""
    xt = to_gpu_c64(x, dev)
    n_total = int(np.prod(shape))
    batch = xt.numel() // n_total
    direction = capi.FFT_INVERSE if inverse else capi.FFT_FORWARD
    h = capi.fft_plan_ex(list(shape), batch, len(shape), capi.FFT_C64, direction, schedule)
    try:
        if scale is not None:
            capi.fft_set_scale(h, scale)
        out = xt if inplace else torch.empty_like(xt)
        ws = None
        if inplace:
            need = capi.fft_workspace_size(h)
            if need:
                ws = torch.empty(need, dtype=torch.uint8, device=dev)
                capi.fft_set_workspace(h, ws.data_ptr(), need)
        stream = torch.cuda.current_stream().cuda_stream
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), stream)
        torch.cuda.synchronize()
        res = out.cpu().numpy()
    finally:
        capi.fft_destroy(h)
    return res


def check_1d(x, n, inverse, dev, schedule=None):
    got = run_c64(x, [n], inverse=inverse, schedule=schedule, dev=dev)
    ref = oracle.fft(np.asarray(x, np.complex64), inverse=inverse)
    err = rel_l2_rows(got, ref, n)
    assert err.max() <= tol_fp32(n), (n, inverse, float(err.max()))
    return err


@pytest.mark.parametrize("lg", range(0, 15))
@pytest.mark.parametrize("inverse", [False, True])
def test_single_pass_sizes(dev, lg, inverse):
    # one-kernel sizes 2^0..2^14, ragged batch (not a multiple of the lines per workgroup)
    n = 1 << lg
    batch = 3 if n >= 4096 else 37
    x = workloads.normal_batch(n, batch, seed=1000 + lg)
    check_1d(x, n, inverse, dev)


@pytest.mark.parametrize("lg", range(15, 21))
@pytest.mark.parametrize("inverse", [False, True])
def test_two_pass_sizes(dev, lg, inverse):
    n = 1 << lg
    x = workloads.normal_batch(n, 3, seed=2000 + lg)
    check_1d(x, n, inverse, dev)


@pytest.mark.parametrize("split", [4, 64, 128, 256, 512, 2048, 4096])
def test_two_pass_all_splits(dev, split):
    # N = 2^16 with every split N1 x N2 that the variants allow (also forced
    # two-pass at N = 2^12 where one pass would do)
    n = 1 << 16
    if split == 4:
        n, split = 1 << 12, 64
    x = workloads.normal_batch(n, 2, seed=split)
    check_1d(x, n, False, dev, schedule=f"split={split}")
    check_1d(x, n, True, dev, schedule=f"split={split}")


@pytest.mark.parametrize("which", ["built-in", "tuned"])
def test_n1024_uniform_single(dev, which):
    # 1-D N=1024, batch 1, complex64, re/im ~ U[-1,1] seed 0; tolerance 1e-5
    x = workloads.uniform_1d(1024, 1, seed=0)
    err = check_1d(x, 1024, False, dev, schedule=tuned([1024], 1) if which == "tuned" else None)
    assert err.max() <= 1e-5


def test_n1024_batch32768_tuned(dev):
    # the 1024-point throughput shape under its tuned schedule
    x = workloads.uniform_1d(1024, 32768, seed=0)
    err = check_1d(x, 1024, False, dev, schedule=tuned([1024], 32768))
    assert err.max() <= 1e-5


def test_n2p16_batch64_tuned(dev):
    x = workloads.normal_batch(1 << 16, 64, seed=4)
    check_1d(x, 1 << 16, False, dev, schedule=tuned([1 << 16], 64))
    check_1d(x, 1 << 16, True, dev, schedule=tuned([1 << 16], 64))


def tuned(shape, batch):
    from paper_1707_07263_amd import autotune
    return autotune.schedule_for(shape, batch, capi.FFT_C64)


@pytest.mark.parametrize("which", ["built-in", "tuned"])
def test_n2p20_batch16_forward_inverse(dev, which):
    # N = 2^20, batch 16, N(0,1) seed 1: forward, then inverse of the GPU
    # output; "tuned" is the schedule the benchmark times
    n, b = 1 << 20, 16
    sched = tuned([n], b) if which == "tuned" else None
    x = workloads.normal_batch(n, b, seed=1)
    xc = x.astype(np.complex64)
    fwd = run_c64(xc, [n], schedule=sched, dev=dev)
    ref = oracle.fft(xc)
    e1 = rel_l2_rows(fwd, ref, n)
    assert e1.max() <= 2.0e-5, float(e1.max())
    inv = run_c64(fwd, [n], inverse=True, schedule=sched, dev=dev)
    ref_inv = oracle.ifft(fwd)
    e2 = rel_l2_rows(inv, ref_inv, n)
    assert e2.max() <= 2.0e-5, float(e2.max())
    rt = rel_l2_rows(inv, xc, n)
    assert rt.max() <= 4.0e-5, float(rt.max())
    # a typical FP32 FFT error at this size is ~2e-7; report a regression early
    assert e1.max() < 1e-6, float(e1.max())


@pytest.mark.parametrize("n,batch,sched", [
    # first pass with the loads of two tiles in flight: 1024 tiles on 256
    # workgroups (4 each), 768 (3 each: the walk ends on the first register
    # set), 320 (2 or 1 each), 64 (fewer tiles than workgroups)
    (1 << 20, 16, "split=1024;a=a1024p32w16q2_c64;b=c1024p32w16x_c64"),
    (1 << 20, 12, "split=1024;a=a1024p32w16q2_c64;b=c1024p32w16x_c64"),
    (1 << 20, 5, "split=1024;xcd=10;a=a1024p32w16q2_c64;b=c1024p32w16x_c64"),
    (1 << 20, 1, "split=1024;a=a1024p32w16q2_c64;b=c1024p32w16x_c64"),
    # two step-row entries per lane (W x P = 2 x lanes)
    (1 << 20, 12, "split=512;a=a512p32w32q2_c64"),
    (1 << 16, 3, "split=256;a=a256p16w16q2_c64"),
    (1 << 16, 64, "split=256;a=a256p16w16q2_c64"),
    (1 << 18, 7, "split=512;a=a512p16w8q2_c64"),
])
@pytest.mark.parametrize("inverse", [False, True])
def test_first_pass_two_tiles_in_flight(dev, n, batch, sched, inverse):
    names = capi.fft_describe([n], batch, 1, capi.FFT_C64, sched)["names"]
    assert names[0].endswith("q2_c64"), names
    x = workloads.normal_batch(n, batch, seed=batch + n % 97)
    check_1d(x, n, inverse, dev, schedule=sched)


@pytest.mark.parametrize("which", ["built-in", "tuned"])
def test_2d_4096x4096_speckle_image(dev, which):
    z = workloads.speckle_image(4096, 4096, seed=2)
    zc = z.astype(np.complex64)
    sched = tuned([4096, 4096], 1) if which == "tuned" else None
    got = run_c64(zc, [4096, 4096], schedule=sched, dev=dev)
    ref = oracle.fft2(zc)
    err = rel_l2_rows(got.reshape(1, -1), ref.reshape(1, -1), 4096 * 4096)
    assert err.max() <= 2.4e-5, float(err.max())
    assert err.max() < 1e-6, float(err.max())


@pytest.mark.parametrize("shape", [(1, 1), (1, 64), (64, 1), (2, 8), (8, 2), (16, 1024), (1024, 16),
                                   (256, 512), (512, 256), (4096, 8), (8, 4096), (128, 16384),
                                   (16384, 4)])
@pytest.mark.parametrize("inverse", [False, True])
def test_2d_shapes(dev, shape, inverse):
    r, c = shape
    b = 2
    x = workloads.normal_batch(r * c, b, seed=r * 7 + c).reshape(b, r, c)
    got = run_c64(x, [r, c], inverse=inverse, dev=dev)
    ref = oracle.fft2(x.astype(np.complex64), inverse=inverse)
    err = rel_l2_rows(got.reshape(b, -1), ref.reshape(b, -1), r * c)
    assert err.max() <= tol_fp32(r * c), (shape, float(err.max()))


@pytest.mark.slow
@pytest.mark.parametrize("lg", [22, 24])
def test_gpu_fp64_twiddles_large(dev, lg):
    # 1-D N >= 2^22: tables are generated on the GPU in FP64
    n = 1 << lg
    x = workloads.normal_batch(n, 1, seed=5)
    h = capi.fft_plan([n], 1, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        assert capi.fft_plan_info(h)["gpu_twiddles"] == 1
    finally:
        capi.fft_destroy(h)
    check_1d(x, n, False, dev)
    check_1d(x, n, True, dev)


def test_closed_forms_on_gpu(dev):
    for n in (16, 1024, 1 << 16):
        k = np.arange(n)
        x = np.zeros((3, n), complex)
        x[0, 0] = 1.0                        # impulse -> all ones
        x[1, :] = 0.5                        # constant -> N/2 at k = 0
        k0 = n // 3
        x[2, :] = np.exp(2j * np.pi * ((k0 * k) % n) / n)  # tone -> N at k0
        got = run_c64(x, [n], dev=dev)
        assert np.max(np.abs(got[0] - 1.0)) < 1e-6
        want1 = np.zeros(n)
        want1[0] = n / 2
        assert np.max(np.abs(got[1] - want1)) < 1e-6 * n
        want2 = np.zeros(n, complex)
        want2[k0] = n
        assert np.max(np.abs(got[2] - want2)) < 2e-6 * n


def test_impulse_batch_is_dft_matrix(dev):
    for n in (2, 8, 64, 256):
        eye = np.eye(n, dtype=complex)
        got = run_c64(eye, [n], dev=dev)
        j, k = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        want = np.exp(-2j * np.pi * ((j * k) % n) / n)
        assert np.max(np.abs(got - want)) < 2e-6


@pytest.mark.parametrize("n", [1024, 1 << 18])
def test_inplace(dev, n):
    x = workloads.normal_batch(n, 4, seed=9)
    got = run_c64(x, [n], inplace=True, dev=dev)
    ref = oracle.fft(x.astype(np.complex64))
    assert rel_l2_rows(got, ref, n).max() <= tol_fp32(n)
    got2 = run_c64(x.reshape(4, 32, n // 32), [32, n // 32], inplace=True, dev=dev)
    ref2 = oracle.fft2(x.astype(np.complex64).reshape(4, 32, n // 32))
    assert rel_l2_rows(got2.reshape(4, -1), ref2.reshape(4, -1), n).max() <= tol_fp32(n)


def test_scale_override_and_adjoint(dev):
    n = 1 << 16
    x = workloads.normal_batch(n, 2, seed=11).astype(np.complex64)
    y = workloads.normal_batch(n, 2, seed=12).astype(np.complex64)
    adj = run_c64(y, [n], inverse=True, scale=1.0, dev=dev)
    ref = oracle.adjoint(y)
    assert rel_l2_rows(adj, ref, n).max() <= tol_fp32(n)
    fx = run_c64(x, [n], dev=dev)
    # dot-product test <F x, y> = <x, F^H y>
    lhs = np.vdot(y.astype(np.complex128), fx.astype(np.complex128))
    rhs = np.vdot(adj.astype(np.complex128), x.astype(np.complex128))
    bound = 1e-6 * math.log2(n) * np.linalg.norm(fx) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= bound
    half = run_c64(x, [n], scale=0.5, dev=dev)
    assert rel_l2_rows(half, 0.5 * oracle.fft(x), n).max() <= tol_fp32(n)


def test_deterministic_repeats(dev):
    n = 1 << 20
    x = to_gpu_c64(workloads.normal_batch(n, 2, seed=13), dev)
    h = capi.fft_plan([n], 2, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        outs = []
        for _ in range(3):
            o = torch.empty_like(x)
            capi.fft_exec(h, x.data_ptr(), o.data_ptr(), torch.cuda.current_stream().cuda_stream)
            outs.append(o)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    finally:
        capi.fft_destroy(h)


def test_other_stream(dev):
    n = 4096
    x = workloads.normal_batch(n, 8, seed=14)
    xt = to_gpu_c64(x, dev)
    s = torch.cuda.Stream()
    out = torch.empty_like(xt)
    torch.cuda.synchronize()
    h = capi.fft_plan([n], 8, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        with torch.cuda.stream(s):
            capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), s.cuda_stream)
        s.synchronize()
    finally:
        capi.fft_destroy(h)
    assert rel_l2_rows(out.cpu().numpy(), oracle.fft(x.astype(np.complex64)), n).max() <= tol_fp32(n)


def test_error_codes(dev):
    n = 1 << 18
    x = torch.zeros(2 * n + 1, dtype=torch.complex64, device=dev)
    h = capi.fft_plan([n], 2, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        # misaligned pointer (4 bytes off an 8-byte element)
        st = capi.fft_exec_status(h, x.data_ptr() + 4, x.data_ptr(), 0)
        assert st == capi.FFT_ERR_ALIGNMENT
        # in place on a two-pass plan without a workspace
        assert capi.fft_exec_status(h, x.data_ptr(), x.data_ptr(), 0) == capi.FFT_ERR_INPLACE
        # partial overlap
        assert capi.fft_exec_status(h, x.data_ptr(), x.data_ptr() + 8, 0) == capi.FFT_ERR_INPLACE
        assert capi.fft_exec_status(h, 0, x.data_ptr(), 0) == capi.FFT_ERR_INVALID_ARGUMENT
    finally:
        capi.fft_destroy(h)
    for bad, code in (([12], capi.FFT_ERR_UNSUPPORTED_SIZE), ([1 << 29], capi.FFT_ERR_UNSUPPORTED_SIZE),
                      ([0], capi.FFT_ERR_UNSUPPORTED_SIZE)):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_plan(bad, 1, 1, capi.FFT_C64, capi.FFT_FORWARD)
        assert ei.value.status == code
    with pytest.raises(capi.FFTError) as ei:
        capi.fft_plan([16], 1, 1, 7, capi.FFT_FORWARD)
    assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
    with pytest.raises(capi.FFTError) as ei:
        capi.fft_plan([16], 1, 1, capi.FFT_C64, 0)
    assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
    with pytest.raises(capi.FFTError) as ei:
        capi.fft_plan_ex([1 << 16], 1, 1, capi.FFT_C64, -1, "a=nonexistent")
    assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT
    capi.fft_destroy(0)  # NULL is a no-op


def _variant_names(prefix_filter):
    from paper_1707_07263_amd import capi as c
    return [c.fft_variant_name(i) for i in range(c.fft_variant_count())
            if prefix_filter(c.fft_variant_name(i))]


PERSISTENT = sorted(n for n in _variant_names(lambda s: "q" in s.split("_")[0] and s.endswith("_c64")))


@pytest.mark.parametrize("name", PERSISTENT)
def test_persistent_variants(dev, name):
    # every persistent (software-pipelined) variant through a plan that uses
    # it, with more tiles than resident workgroups and a ragged last tile;
    # the inverse with the XCD remap (permuted start tiles)
    from paper_1707_07263_amd import capi as c
    i = [c.fft_variant_name(k) for k in range(c.fft_variant_count())].index(name)
    d = c.fft_variant_describe(i)
    L = d["L"]
    if d["role"] == 4:      # 2-D rows fused with a radix-W column step
        r, W = 1024, d["W"]
        batch = 3          # r / W * 3 tiles: more than resident workgroups
        sched = f"rowcol={W};row={name}"
        x = workloads.normal_batch(r * L, batch, seed=L + W).reshape(batch, r, L)
        for inv, sc in ((False, sched), (True, sched + ";xcd=1")):
            got = run_c64(x, [r, L], inverse=inv, schedule=sc, dev=dev)
            ref = oracle.fft2(x.astype(np.complex64), inverse=inv)
            err = rel_l2_rows(got.reshape(batch, -1), ref.reshape(batch, -1), r * L)
            assert err.max() <= tol_fp32(r * L), (name, inv, float(err.max()))
        return
    if d["role"] == 0:      # one-pass rows
        n, batch, sched = L, (1 << 22) // L + 3, f"single={name}"
    elif d["role"] == 1:    # first pass of a split
        n, batch, sched = L * 512, 5, f"split={L};a={name}"
    else:                   # strided columns (second pass of a split)
        n, batch, sched = 512 * L, 5, f"split=512;b={name}"
    x = workloads.normal_batch(n, batch, seed=L + batch)
    check_1d(x, n, False, dev, schedule=sched)
    check_1d(x, n, True, dev, schedule=sched + ";xcd=1")


# every shape here has a three-pass plan: rows R = Sq^2 (even log2 R), and a
# compiled row variant with at most R rows per tile (the smallest row tiles
# are 32 rows of 64 points, 128 of 16 and 256 of 8)
THREE_PASS_SHAPES = [(64, 64), (16, 1024), (256, 16), (256, 512), (1024, 16), (1024, 64), (4096, 8),
                     (4096, 256), (16384, 16), (256, 8)]


@pytest.mark.parametrize("shape", THREE_PASS_SHAPES)
@pytest.mark.parametrize("inverse", [False, True])
def test_2d_three_pass(dev, shape, inverse):
    # columns as two sub-passes of sqrt(rows) points, rows permuted in place
    r, c = shape
    capi.fft_describe([r, c], 2, 2, capi.FFT_C64, "col3=1")  # raises if the shape has no such plan
    b = 2
    x = workloads.normal_batch(r * c, b, seed=r + 3 * c).reshape(b, r, c)
    got = run_c64(x, [r, c], inverse=inverse, schedule="col3=1", dev=dev)
    ref = oracle.fft2(x.astype(np.complex64), inverse=inverse)
    err = rel_l2_rows(got.reshape(b, -1), ref.reshape(b, -1), r * c)
    assert err.max() <= tol_fp32(r * c), (shape, float(err.max()))


@pytest.mark.parametrize("col3", ["0", "1"])
def test_2d_4096x4096_image_both_column_plans(dev, col3):
    z = workloads.speckle_image(4096, 4096, seed=2).astype(np.complex64)
    got = run_c64(z, [4096, 4096], schedule=f"col3={col3}", dev=dev)
    ref = oracle.fft2(z)
    err = rel_l2_rows(got.reshape(1, -1), ref.reshape(1, -1), 4096 * 4096)
    assert err.max() <= 2.4e-5 and err.max() < 1e-6, float(err.max())
    # in place as well (no workspace needed for 2-D)
    got2 = run_c64(z, [4096, 4096], schedule=f"col3={col3}", inplace=True, dev=dev)
    assert np.array_equal(got, got2)


LONG_COLUMNS = sorted(n for n in _variant_names(
    lambda s: s.startswith("c") and "p32" in s and int(s[1:s.index("p")]) >= 2048))
COL_TWIDDLE = sorted(n for n in _variant_names(lambda s: s.startswith("t")))


@pytest.mark.parametrize("name", LONG_COLUMNS)
def test_long_column_variants(dev, name):
    # 32 points per lane down 2048- and 4096-long columns of a 2-D transform
    L = int(name[1:name.index("p")])
    dt = {"c64": capi.FFT_C64, "f16": capi.FFT_C16F, "bf16": capi.FFT_C16BF}[name.split("_")[1]]
    if dt != capi.FFT_C64:
        pytest.skip("complex64 variant test")
    for c, inverse in ((64, False), (4, True)):  # 4 columns: a partial tile
        x = workloads.normal_batch(L * c, 2, seed=L + c).reshape(2, L, c)
        got = run_c64(x, [L, c], inverse=inverse, schedule=f"col3=0;col={name}", dev=dev)
        ref = oracle.fft2(x.astype(np.complex64), inverse=inverse)
        assert rel_l2_rows(got.reshape(2, -1), ref.reshape(2, -1), L * c).max() <= tol_fp32(L * c)


@pytest.mark.parametrize("name", COL_TWIDDLE)
def test_column_twiddle_variants(dev, name):
    # every first column sub-pass variant in a three-pass 2-D plan, in its
    # storage type
    m = re.match(r"t(\d+)p(\d+)w(\d+)", name)
    sq, w = int(m.group(1)), int(m.group(3))
    dts = name.split("_")[1]
    dt = {"c64": capi.FFT_C64, "f16": capi.FFT_C16F, "bf16": capi.FFT_C16BF}[dts]
    r, c, sched = sq * sq, max(w, 16), f"col3=1;colt={name}"
    try:
        capi.fft_describe([r, c], 2, 2, dt, sched)
    except capi.FFTError:
        # few rows: long rows, so a row tile of two rows exists
        c, sched = 4096, sched + f";row=r4096p16w2_{dts}"
        try:
            capi.fft_describe([r, c], 2, 2, dt, sched)
        except capi.FFTError:
            pytest.skip("no three-pass plan with this variant")
    x = workloads.normal_batch(r * c, 2, seed=sq + w).reshape(2, r, c)
    if dt == capi.FFT_C64:
        got = run_c64(x, [r, c], schedule=sched, dev=dev)
        ref = oracle.fft2(x.astype(np.complex64))
        assert rel_l2_rows(got.reshape(2, -1), ref.reshape(2, -1), r * c).max() <= tol_fp32(r * c)
        return
    from gpu_helpers import from_gpu_16, quantised, to_gpu_16
    tdt = torch.float16 if dt == capi.FFT_C16F else torch.bfloat16
    xt = to_gpu_16(x, dev, tdt)
    out = torch.empty_like(xt)
    h = capi.fft_plan_ex([r, c], 2, 2, dt, capi.FFT_FORWARD, sched)
    try:
        capi.fft_exec(h, xt.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        capi.fft_destroy(h)
    ref = oracle.fft2(quantised(x, tdt))
    err = rel_l2_rows(from_gpu_16(out).reshape(2, -1), ref.reshape(2, -1), r * c)
    assert err.max() <= (1e-3 if dt == capi.FFT_C16F else 8e-3), float(err.max())


THREE_PASS_1D = [(1 << 12, "split=64;split2=16"), (1 << 16, "split=256;split2=8"),
                 (1 << 20, "split=1024;split2=128"), (1 << 18, "split=64;split2=2")]


@pytest.mark.parametrize("n,sched", THREE_PASS_1D)
@pytest.mark.parametrize("inverse", [False, True])
def test_three_pass_1d_forced(dev, n, sched, inverse):
    # N1 x N2 x N3 with a ragged batch of 3 (the last pass runs per transform)
    x = workloads.normal_batch(n, 3, seed=n % 9973)
    check_1d(x, n, inverse, dev, schedule=sched)
    got = run_c64(x, [n], inverse=inverse, schedule=sched, inplace=True, dev=dev)
    ref = oracle.fft(np.asarray(x, np.complex64), inverse=inverse)
    assert rel_l2_rows(got, ref, n).max() <= tol_fp32(n)


def test_three_pass_1d_2p25_full(dev):
    n = 1 << 25
    x = workloads.normal_batch(n, 1, seed=25).astype(np.complex64)
    assert capi.fft_describe([n], 1, 1, capi.FFT_C64)["passes"] == 3
    got = run_c64(x, [n], dev=dev)
    err = rel_l2_rows(got, oracle.fft(x), n)
    print(f"2^25 three-pass rel-L2 {err.max():.3e}")
    assert err.max() <= tol_fp32(n)


def test_three_pass_1d_2p28_sampled(dev):
    # 2^28 points: outputs sampled against the long-double sum, the round
    # trip and Parseval over the whole array
    n = 1 << 28
    g = np.random.default_rng(28)
    x = (g.standard_normal(n, dtype=np.float32) + 1j * g.standard_normal(n, dtype=np.float32)).astype(np.complex64)
    xt = to_gpu_c64(x, dev)
    fwd = capi.fft_plan([n], 1, 1, capi.FFT_C64, capi.FFT_FORWARD)
    inv = capi.fft_plan([n], 1, 1, capi.FFT_C64, capi.FFT_INVERSE)
    try:
        assert capi.fft_plan_info(fwd)["gpu_twiddles"] == 1
        y = torch.empty_like(xt)
        z = torch.empty_like(xt)
        st = torch.cuda.current_stream().cuda_stream
        capi.fft_exec(fwd, xt.data_ptr(), y.data_ptr(), st)
        capi.fft_exec(inv, y.data_ptr(), z.data_ptr(), st)
        torch.cuda.synchronize()
        rt = (torch.linalg.vector_norm(z - xt) / torch.linalg.vector_norm(xt)).item()
        ex = torch.linalg.vector_norm(xt.to(torch.complex128)).item() ** 2
        ey = torch.linalg.vector_norm(y.to(torch.complex128)).item() ** 2 / n
        ks = np.array([0, 1, 2, 12345, (1 << 27) + 3, n - 1, 98765432, 3 * (n // 4)])
        ys = y[torch.from_numpy(ks).to(dev)].cpu().numpy()
    finally:
        capi.fft_destroy(fwd)
        capi.fft_destroy(inv)
    del xt, y, z
    ref = oracle.dft_at(x, ks)
    rms = math.sqrt(n * 2.0)  # |X[k]| scale for unit-variance complex input
    worst = float(np.max(np.abs(ys - ref)) / rms)
    print(f"2^28: sampled |err|/rms {worst:.3e}, round trip {rt:.3e}, Parseval {abs(ey - ex) / ex:.3e}")
    assert worst <= tol_fp32(n)
    assert rt <= 2 * tol_fp32(n)
    assert abs(ey - ex) / ex <= 1e-5


@pytest.mark.parametrize("n,b", [(1024, 1 << 21), (1 << 20, 1 << 11)])
def test_batch_beyond_2p31_points(dev, n, b):
    # 2^31 points in one plan (16 GiB each way): element offsets past the
    # 32-bit range; sampled rows, the last included, against the oracle
    print(f"batch of 2^31 points: n={n} batch={b}", flush=True)
    g = torch.Generator(device=dev)
    g.manual_seed(31)
    xt = torch.randn(b, n, dtype=torch.complex64, device=dev, generator=g)
    y = torch.empty_like(xt)
    h = capi.fft_plan([n], b, 1, capi.FFT_C64, capi.FFT_FORWARD)
    try:
        capi.fft_exec(h, xt.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        capi.fft_destroy(h)
    rows = torch.tensor([0, 1, b // 2 - 1, b // 2, b - 2, b - 1, 12345 % b, (b * 7) // 9], device=dev)
    xs = xt[rows].cpu().numpy()
    ys = y[rows].cpu().numpy()
    del xt, y
    torch.cuda.empty_cache()
    err = rel_l2_rows(ys, oracle.fft(xs), n)
    print(f"n={n} batch={b}: sampled rows rel-L2 max {err.max():.3e}")
    assert err.max() <= tol_fp32(n), float(err.max())


BLOCKED_2D = [((256, 512), 3, "blk=8"), ((1024, 1024), 2, "blk=8;xcd=01"), ((512, 4096), 1, "blk=8"),
              ((4096, 256), 2, "blk=16"), ((128, 2048), 2, "blk=32"),
              ((4096, 4096), 1, "blk=8;row=r4096p16w1q_c64;col=c4096p32w8x_c64;xcd=01")]


@pytest.mark.parametrize("shape,batch,sched", BLOCKED_2D)
@pytest.mark.parametrize("inverse", [False, True])
def test_2d_blocked_intermediate(dev, shape, batch, sched, inverse):
    # rows into column blocks of a workspace, then columns reading whole
    # blocks: out of place and in place, against the oracle
    r, c = shape
    x = workloads.normal_batch(r * c, batch, seed=r + c + batch).reshape(batch, r, c)
    got = run_c64(x, [r, c], inverse=inverse, schedule=sched, dev=dev)
    ref = oracle.fft2(x.astype(np.complex64), inverse=inverse)
    err = rel_l2_rows(got.reshape(batch, -1), ref.reshape(batch, -1), r * c)
    assert err.max() <= tol_fp32(r * c), (shape, sched, float(err.max()))
    got2 = run_c64(x, [r, c], inverse=inverse, schedule=sched, inplace=True, dev=dev)
    assert np.array_equal(got, got2)


# rows fused with the first radix-4 step of the columns (R = 4 M), then
# M-point columns in place: shapes down to M = 2, several column widths,
# batched images (one column launch per image), every fused row length
ROWCOL_2D = [((4096, 4096), 1, "rowcol=4"), ((4096, 4096), 1, "rowcol=4;col=c1024p32w32x_c64;xcd=11"),
             ((1024, 1024), 2, "rowcol=4"), ((64, 256), 3, "rowcol=4"), ((8, 512), 2, "rowcol=4"),
             ((256, 2048), 2, "rowcol=4;xcd=10"), ((2048, 4096), 1, "rowcol=4;col=c512p16w16q_c64"),
             ((16, 1024), 5, "rowcol=4"), ((4096, 4096), 1, "rowcol=4;row=f4096p32w4qx_c64"),
             ((1024, 4096), 2, "rowcol=2"), ((64, 2048), 3, "rowcol=2;xcd=11"),
             # stage twiddles from two factor tables of W_4096, one-round exchanges
             ((4096, 4096), 1, "rowcol=4;row=f4096p16w4q_c64;col=c1024p32w16x_c64"),
             ((16, 4096), 3, "rowcol=4;row=f4096p32w4q_c64"),
             ((4096, 4096), 1, "rowcol=2;row=f4096p16w2q_c64;col=c2048p32w16x_c64"),
             ((32, 4096), 2, "rowcol=2;row=f4096p32w2q_c64"),
             ((4096, 4096), 1, "rowcol=2;row=f4096p16w2q_c64;col=c2048p32w8q_c64;xcd=01")]


@pytest.mark.parametrize("shape,batch,sched", ROWCOL_2D)
@pytest.mark.parametrize("inverse", [False, True])
def test_2d_rows_fused_with_column_step(dev, shape, batch, sched, inverse):
    r, c = shape
    names = capi.fft_describe([r, c], batch, 2, capi.FFT_C64, sched)["names"]
    assert names[0].startswith("f") and names[0].endswith("_c64"), names
    x = workloads.normal_batch(r * c, batch, seed=3 * r + c + batch).reshape(batch, r, c)
    got = run_c64(x, [r, c], inverse=inverse, schedule=sched, dev=dev)
    ref = oracle.fft2(x.astype(np.complex64), inverse=inverse)
    err = rel_l2_rows(got.reshape(batch, -1), ref.reshape(batch, -1), r * c)
    assert err.max() <= tol_fp32(r * c), (shape, sched, float(err.max()))
    # in place: the rows go through the workspace; same kernels, same bits
    got2 = run_c64(x, [r, c], inverse=inverse, schedule=sched, inplace=True, dev=dev)
    assert np.array_equal(got, got2)


def test_2d_rows_fused_scale_and_closed_form(dev):
    # a caller scale is applied once, by the last pass; an impulse at (a, b)
    # gives W_R^{a k} W_C^{b l} (eq. 1 along both axes)
    r, c = 64, 256
    x = np.zeros((1, r, c), np.complex64)
    x[0, 5, 17] = 1
    got = run_c64(x, [r, c], schedule="rowcol=4", scale=0.5, dev=dev).reshape(r, c)
    k = np.arange(r)[:, None]
    l = np.arange(c)[None, :]
    want = 0.5 * np.exp(-2j * np.pi * ((5 * k) % r) / r) * np.exp(-2j * np.pi * ((17 * l) % c) / c)
    assert np.max(np.abs(got - want)) < 2e-6
