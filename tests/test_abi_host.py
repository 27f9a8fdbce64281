"""CPU-side checks of the C-ABI library: it loads, exports every function
declared in include/mi355fft.h, plans schedules on the host, reports errors
for bad arguments, and its host twiddle generator rounds W_M^e correctly.
No kernel is launched here."""
import os
import re

import mpmath
import numpy as np
import pytest

from paper_1707_07263_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355fft.h")


@pytest.fixture(scope="module")
def lib():
    return capi.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.EXPORTED)


def test_error_strings(lib):
    for code in range(0, -9, -1):
        s = capi.error_string(code)
        assert s and s != "unknown status"
    assert capi.error_string(-99) == "unknown status"


def test_variant_registry(lib):
    n = capi.fft_variant_count()
    assert n > 100
    seen = set()
    for i in range(n):
        name = capi.fft_variant_name(i)
        d = capi.fft_variant_describe(i)
        assert name not in seen
        seen.add(name)
        m = re.match(r"([ractf])(\d+)p(\d+)w(\d+)(q2|q)?(x?)_(c64|f16|bf16)$", name)
        assert m, name
        assert int(m.group(2)) == d["L"] and int(m.group(3)) == d["P"] and int(m.group(4)) == d["W"]
        assert {"r": 0, "a": 1, "c": 2, "t": 3, "f": 4}[m.group(1)] == d["role"]
        assert {"c64": 0, "f16": 1, "bf16": 2}[m.group(7)] == d["dtype"]
        assert d["threads"] == d["W"] * d["L"] // d["P"] and d["threads"] <= 1024
    assert capi.fft_variant_name(n) is None


@pytest.mark.parametrize("n,dims,batch,passes,split", [
    ([1024], 1, 1, 1, [0, 0]),                 # one pass fits a workgroup
    ([1 << 14], 1, 4, 1, [0, 0]),
    ([1 << 15], 1, 4, 2, [256, 128]),          # first length that needs the split
    ([1 << 20], 1, 16, 2, [1024, 1024]),
    ([1 << 24], 1, 1, 2, [4096, 4096]),
    ([4096, 4096], 2, 1, 3, [0, 0]),           # rows, then columns as two sub-passes
    ([2048, 4096], 2, 1, 2, [0, 0]),           # rows, then columns
    ([1, 64], 2, 3, 1, [0, 0]),                # a length-1 axis needs no pass
    ([64, 1], 2, 3, 1, [0, 0]),
    ([1], 1, 5, 1, [0, 0]),
])
def test_describe_schedules(lib, n, dims, batch, passes, split):
    d = capi.fft_describe(n, batch, dims, capi.FFT_C64)
    assert d["passes"] == passes
    assert d["split"] == split
    if dims == 1 and n[0] > 1 and passes == 2:
        assert d["names"][0].startswith(f"a{split[0]}p") and d["names"][1].startswith(f"c{split[1]}p")


def test_describe_schedule_overrides(lib):
    d = capi.fft_describe([1 << 16], 2, 1, capi.FFT_C64, "split=512")
    assert d["split"] == [512, 128]
    d = capi.fft_describe([1 << 20], 2, 1, capi.FFT_C64, "a=a1024p16w8_c64;b=c1024p16w8_c64")
    assert d["names"] == ["a1024p16w8_c64", "c1024p16w8_c64"]
    for bad in ("split=3", "split=1048576", "a=c1024p16w8_c64", "a=a512p16w16_c64", "bogus=1", "split"):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_describe([1 << 20], 2, 1, capi.FFT_C64, bad)
        assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT, bad


@pytest.mark.parametrize("n,dims,dtype,code", [
    ([12], 1, 0, capi.FFT_ERR_UNSUPPORTED_SIZE),
    ([0], 1, 0, capi.FFT_ERR_UNSUPPORTED_SIZE),
    ([1 << 29], 1, 0, capi.FFT_ERR_UNSUPPORTED_SIZE),
    ([1 << 15, 4], 2, 0, capi.FFT_ERR_UNSUPPORTED_SIZE),
    ([16], 3, 0, capi.FFT_ERR_INVALID_ARGUMENT),
    ([16], 1, 9, capi.FFT_ERR_INVALID_ARGUMENT),
])
def test_describe_errors(lib, n, dims, dtype, code):
    with pytest.raises(capi.FFTError) as ei:
        capi.fft_describe(n, 1, dims, dtype)
    assert ei.value.status == code


def test_describe_16bit(lib):
    for dt in (capi.FFT_C16F, capi.FFT_C16BF):
        for n in ([256], [1 << 20], [512, 512]):
            d = capi.fft_describe(n, 2, len(n), dt)
            suffix = "_f16" if dt == capi.FFT_C16F else "_bf16"
            assert all(v.endswith(suffix) for v in d["names"])


@pytest.mark.parametrize("M,R,mul,count", [(16, 0, 1, 16), (1024, 0, 1, 1024), (1 << 20, 0, 1024, 1024),
                                          (1 << 20, 0, 1, 2048), (1024, 16, 1, 1024), (1 << 22, 0, 2047, 512),
                                          (1 << 24, 16, 4096, 4096)])
def test_host_twiddles_correctly_rounded(lib, M, R, mul, count):
    # every entry is W_M^e = exp(-2 pi i e / M) rounded to float32; compared
    # with the value computed to 30 digits by mpmath and rounded once
    got = capi.fft_twiddle_host(count, R, M, mul)
    mpmath.mp.dps = 30
    want = np.empty(count, np.complex64)
    for i in range(count):
        e = (i // R) * (i % R) * mul if R else i * mul
        ang = 2 * mpmath.pi * mpmath.mpf(e % M) / M
        c, s = mpmath.cos(ang), mpmath.sin(ang)
        # cos/sin of exact multiples of pi/2 are exactly 0; at 30 digits they
        # come out as ~1e-31, below any float32 table entry
        c = 0 if abs(c) < mpmath.mpf(10) ** -25 else c
        s = 0 if abs(s) < mpmath.mpf(10) ** -25 else s
        want[i] = np.float32(float(c)) + 1j * np.float32(-float(s))
    mism = np.nonzero(got != want)[0]
    # float64 -> float32 double rounding can only differ at exact ties, which
    # these arguments do not hit
    assert mism.size == 0, [(int(i), got[i], want[i]) for i in mism[:5]]


def test_host_twiddle_symmetries(lib):
    M = 4096
    w = capi.fft_twiddle_host(M, 0, M, 1).astype(np.complex128)
    k = np.arange(M)
    # eq. 4: W^{-k} = conj(W^k), read as W^{M-k}
    assert np.array_equal(w[(M - k) % M], np.conj(w))
    # quarter-turn symmetry of the reduction: W^{k + M/4} = -i W^k exactly
    assert np.array_equal(w[(k + M // 4) % M], -1j * w)
    # eq. 5 reducibility: W_M^{2k} = W_{M/2}^k
    half = capi.fft_twiddle_host(M // 2, 0, M // 2, 1)
    assert np.array_equal(w[0::2].astype(np.complex64), half)


def test_package_imports_without_gpu():
    import paper_1707_07263_amd as pkg
    from paper_1707_07263_amd import api  # noqa: F401
    assert callable(pkg.fft) and callable(pkg.fft2) and callable(pkg.fft_many)
    assert pkg.FFTFunction is api.FFTFunction


def test_describe_three_pass_2d(lib):
    d = capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64)
    assert d["passes"] == 3
    assert d["names"][0].startswith("t64p") and d["names"][1].startswith("c64p")
    assert d["names"][2].startswith("r4096p")
    assert capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, "col3=0")["passes"] == 2
    d = capi.fft_describe([1024, 64], 3, 2, capi.FFT_C64, "col3=1")
    assert d["passes"] == 3 and d["names"][0].startswith("t32p")
    # rows not a power of four, or a single column: refused when asked for,
    # and the automatic choice falls back to two passes
    for shape in ([2048, 64], [4096, 1]):
        with pytest.raises(capi.FFTError):
            capi.fft_describe(shape, 1, 2, capi.FFT_C64, "col3=1")
        assert capi.fft_describe(shape, 1, 2, capi.FFT_C64)["passes"] <= 2
    # a row variant with an odd number of rows per tile cannot pair rows
    assert capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, "row=r4096p16w1q_c64")["passes"] == 2
    # a column tile never takes more columns than the image has when a
    # narrower variant exists (8 columns: 8-column tiles, not 16)
    d = capi.fft_describe([4096, 8], 2, 2, capi.FFT_C64, "col3=1")
    assert d["passes"] == 3
    assert all(int(re.search(r"w(\d+)", nm).group(1)) <= 8 for nm in d["names"][:2]), d["names"]


def test_describe_blocked_2d(lib):
    d = capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, "blk=8")
    assert d["passes"] == 2 and d["names"][0].startswith("r4096") and d["names"][1].startswith("c4096")
    # a column tile never spans two blocks; a row lane must stay in one block column
    assert int(re.search(r"w(\d+)", d["names"][1]).group(1)) <= 8
    for shape, sched in (([64, 64], "blk=16"), ([16, 8], "blk=8"), ([4096, 4096], "blk=8;col3=1"),
                         ([4096, 4096], "blk=12"), ([1, 4096], "blk=8")):
        with pytest.raises(capi.FFTError):
            capi.fft_describe(shape, 1, 2, capi.FFT_C64, sched)


def test_describe_levels_method(lib):
    d = capi.fft_describe([1 << 20], 16, 1, capi.FFT_C64, "method=levels")
    assert d["passes"] == 1 and d["names"][0] == "levels_radix2"
    assert capi.fft_describe([1 << 20], 16, 1, capi.FFT_C64, "method=lds")["passes"] == 2
    # a length-1 transform is a copy under either method
    assert capi.fft_describe([1], 3, 1, capi.FFT_C64, "method=levels")["names"][0] == "copy_scale"
    for bad, dims, n in (("method=levels", 2, [64, 64]), ("method=radix2", 1, [64])):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_describe(n, 1, dims, capi.FFT_C64, bad)
        assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT


def test_describe_rows_fused_with_column_step(lib):
    # rowcol=4: the row pass takes the first radix-4 step of the columns,
    # leaving columns of R/4 points
    for (r, c), col_len in (((4096, 4096), 1024), ((64, 256), 16), ((8, 1024), 2)):
        d = capi.fft_describe([r, c], 2, 2, capi.FFT_C64, "rowcol=4")
        assert d["passes"] == 2 and re.match(rf"f{c}p\d+w4qx?_c64$", d["names"][0]), d
        assert re.match(rf"c{col_len}p\d+w\d+", d["names"][1]), d
    d = capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, "rowcol=2")
    assert d["names"][0] == "f4096p32w2qx_c64" and d["names"][1].startswith("c2048")
    for bad in ("rowcol=8", "rowcol=4;col3=1", "rowcol=4;blk=8", "rowcol=x", "rowcol=2;row=f4096p16w4qx_c64"):
        with pytest.raises(capi.FFTError):
            capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, bad)
    # no fused variant for this row length, too few rows, or 1-D
    for shape, dims in (([64, 128], 2), ([4, 1024], 2), ([1 << 20], 1)):
        with pytest.raises(capi.FFTError):
            capi.fft_describe(shape, 1, dims, capi.FFT_C64, "rowcol=4")


def test_describe_dft256_experiments(lib):
    for method, name in (("mfma", "mfma_dft256"), ("xlane", "xlane_dft256"),
                         ("xlane_bperm", "xlane_bperm_dft256")):
        d = capi.fft_describe([256], 5, 1, capi.FFT_C64, f"method={method}")
        assert d["passes"] == 1 and d["names"][0] == name
        # 256-point complex64 batches only
        for n, dims, dt in (([512], 1, capi.FFT_C64), ([256], 1, capi.FFT_C16F),
                            ([16, 16], 2, capi.FFT_C64)):
            with pytest.raises(capi.FFTError) as ei:
                capi.fft_describe(n, 1, dims, dt, f"method={method}")
            assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT


def test_describe_xcd_masks(lib):
    for ok in ("xcd=0", "xcd=1", "xcd=01", "xcd=10"):
        assert capi.fft_describe([1 << 20], 16, 1, capi.FFT_C64, ok)["passes"] == 2
    assert capi.fft_describe([4096, 4096], 1, 2, capi.FFT_C64, "col3=1;xcd=101")["passes"] == 3
    for bad in ("xcd=011", "xcd=2", "xcd=", "xcd=00000"):
        with pytest.raises(capi.FFTError):
            capi.fft_describe([1 << 20], 16, 1, capi.FFT_C64, bad)



def test_describe_three_pass_1d(lib):
    # beyond two passes of 2^12: N1 x N2 x N3 = 2^10 x 2^7 x 2^(l-17)
    for l in (25, 26, 27, 28):
        d = capi.fft_describe([1 << l], 1, 1, capi.FFT_C64)
        assert d["passes"] == 3 and d["split"] == [1024, 1 << (l - 10)]
        assert d["names"][0].startswith("a1024p") and d["names"][1].startswith("t128p")
        assert d["names"][2].startswith(f"c{1 << (l - 17)}p")
    # forced at smaller sizes
    for n, sched in ((1 << 12, "split=64;split2=16"), (1 << 16, "split=256;split2=8"),
                     (1 << 20, "split=1024;split2=128"), (1 << 18, "split=64;split2=2")):
        assert capi.fft_describe([n], 3, 1, capi.FFT_C64, sched)["passes"] == 3
    d = capi.fft_describe([1 << 16], 3, 1, capi.FFT_C64, "split=256;split2=8")
    assert d["passes"] == 3 and d["names"][1].startswith("t8p") and d["names"][2].startswith("c32p")
    for bad in ("split2=256", "split=8192;split2=4", "split2=3", "split2=65536"):
        with pytest.raises(capi.FFTError):
            capi.fft_describe([1 << 26], 1, 1, capi.FFT_C64, bad)


def test_pipe_argument_errors(lib):
    import ctypes
    h = ctypes.c_void_p()
    assert lib.fft_pipe_create(None, 3, ctypes.byref(h)) == capi.FFT_ERR_INVALID_ARGUMENT
    assert lib.fft_pipe_create(None, 3, None) == capi.FFT_ERR_INVALID_ARGUMENT
    assert lib.fft_pipe_exec(None, None, None, 1) == capi.FFT_ERR_INVALID_ARGUMENT
    assert lib.fft_pipe_wait(None) == capi.FFT_ERR_INVALID_ARGUMENT
    assert lib.fft_pipe_destroy(None) == capi.FFT_OK


def test_tuned_cache_is_valid_for_the_compiled_variants(lib):
    # every committed tuned schedule plans on the host, and the passes it
    # names are the passes the planner builds (no GPU needed)
    import json
    from paper_1707_07263_amd import autotune, workloads
    with open(autotune.CACHE_PATH) as f:
        cache = json.load(f)
    uneven = [int(s) for s in workloads.uneven_sizes(512, 8, 16, seed=3)]
    plans = many = 0
    for key, entry in cache.items():
        arch, kind, shape, batch, dtype = key.split("|")
        sched = entry["schedule"]
        if kind == "plan":
            dims = [int(v) for v in shape.split("x")]
            d = capi.fft_describe(dims, int(batch), len(dims), int(dtype), sched)
            named = [v.split("=", 1)[1] for v in sched.split(";")
                     if v.split("=", 1)[0] in ("single", "a", "b", "row", "col", "colt")]
            assert set(named) <= set(d["names"]), (key, named, d["names"])
            plans += 1
        else:
            assert kind == "many" and autotune._many_key(uneven, int(dtype)) == key, key
            items, _, _ = capi.fft_describe_many(uneven, int(dtype), sched)
            assert len(items) > 0
            many += 1
    assert plans >= 8 and many == 3


def test_committed_variant_sources_match_generator():
    # the variants_*.hip instantiation tables are generated from the registry
    # in gen_variants.py at every build; the committed copies must be exactly
    # what it generates
    import importlib.util
    path = os.path.join(ROOT, "paper_1707_07263_amd", "csrc", "gen_variants.py")
    spec = importlib.util.spec_from_file_location("gen_variants_check", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert mod.check() == []
