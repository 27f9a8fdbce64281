"""Host logic of bench.py: argument handling, the rocprofv3 summary parsers
and the traffic lookup, on synthetic CSV files (no GPU needed)."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

PIPE_A = "void mfft::k_pipe<1024, 32, 16, 1, 0, true, 0, HIP_vector_type<float, 2u>, 1>(mfft::PassArgs)"
STRIP_B = "void mfft::k_strip<1024, 32, 16, 1, 1, false, 1, HIP_vector_type<float, 2u> >(mfft::PassArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_defaults_and_multi_gpu_refusal(capsys):
    a = bench.parse_args([])
    assert (a.gpus, a.mode) == (1, "bench") and a.steps > 0 and a.warmup >= 0
    assert bench.main(["--gpus", "2"]) == 2
    err = capsys.readouterr().err
    assert "one GPU" in err


def test_no_gpu_visible_is_an_error(capsys):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    assert bench.main(["--steps", "1", "--warmup", "0"]) == 1
    assert "no GPU" in capsys.readouterr().err


@pytest.mark.parametrize("variant,sig", [
    ("a1024p32w16q_c64", "k_pipe<1024, 32, 16, 1, 0, true, 0, HIP_vector_type<float, 2u>, 1>"),
    ("a1024p32w16q2_c64", "k_pipe<1024, 32, 16, 1, 0, true, 0, HIP_vector_type<float, 2u>, 2>"),
    ("c1024p32w16x_c64", "k_strip<1024, 32, 16, 1, 1, false, 1, HIP_vector_type<float, 2u> >"),
    ("r256p16w16_f16", "k_strip<256, 16, 16, 0, 0, false, 0, __half2 >"),
    ("a256p16w16q_bf16", "k_pipe<256, 16, 16, 1, 0, true, 0, mfft::c16bf, 1>"),
    ("not-a-variant", "not-a-variant"),
])
def test_variant_kernel_signature(variant, sig):
    assert bench.variant_kernel_signature(variant) == sig


def test_source_hash_is_stable_and_scoped():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
    int(h, 16)
    # every source the hash skips belongs to a kernel family the step never runs
    csrc = os.path.join(ROOT, "paper_1707_07263_amd", "csrc")
    skipped = [f for f in os.listdir(csrc) if f.startswith(bench.NOT_IN_STEP)]
    assert not any(f.startswith(("fft_device", "fft_host", "strip")) for f in skipped)


def test_summarize_trace_orders_by_total(tmp_path):
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]
    _write_csv(str(tmp_path / "a" / "run_kernel_stats.csv"), hdr, [
        [STRIP_B, 6, 300000, 50000, 40.0],
        [PIPE_A, 6, 360000, 60000, 48.0],
        [COPY, 1, 90000, 90000, 12.0],
    ])
    out = bench.summarize_trace(str(tmp_path)).splitlines()
    assert out[0].startswith("kernel | calls")
    assert PIPE_A in out[1] and "| 6 | 60.00 | 0.360 | 48.00" in out[1]
    assert STRIP_B in out[2] and COPY in out[3]
    with pytest.raises(SystemExit):
        bench.summarize_trace(str(tmp_path / "empty"))


def _pmc_dirs(tmp_path, copy_fetch_kib, copy_write_kib, a_fetch, a_write):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    df, dw = tmp_path / "fetch", tmp_path / "write"
    _write_csv(str(df / "x" / "run_counter_collection.csv"), hdr, [
        [COPY, "FETCH_SIZE", copy_fetch_kib],
        [PIPE_A, "FETCH_SIZE", a_fetch[0]],
        [PIPE_A, "FETCH_SIZE", a_fetch[1]],
        [PIPE_A, "GRBM_COUNT", 7],
    ])
    _write_csv(str(dw / "x" / "run_counter_collection.csv"), hdr, [
        [COPY, "WRITE_SIZE", copy_write_kib],
        [PIPE_A, "WRITE_SIZE", a_write[0]],
        [PIPE_A, "WRITE_SIZE", a_write[1]],
    ])
    return str(df), str(dw)


def test_summarize_pmc_scales_by_copy_calibration(tmp_path):
    kib = bench.COPY_BYTES / 1024
    # the copy's fetch counter reads half its size, its write counter the whole
    df, dw = _pmc_dirs(tmp_path, kib / 2, kib, (1000.0, 3000.0), (4096.0, 4096.0))
    out = bench.summarize_pmc(df, dw).splitlines()
    assert out[0] == "source_hash=" + bench.kernel_source_hash()
    assert "fetch_scale=2.0000 write_scale=1.0000" in out[1]
    line = [l for l in out if PIPE_A in l][0]
    assert "dispatches=2" in line and "fetch_kib_avg=2000.0" in line and "write_kib_avg=4096.0" in line
    assert line.endswith(f"hbm_bytes_per_launch={(2000 * 2 + 4096) * 1024}")


def test_read_traffic_checks_the_source_hash(tmp_path, monkeypatch):
    kib = bench.COPY_BYTES / 1024
    df, dw = _pmc_dirs(tmp_path, kib / 2, kib, (1000.0, 1000.0), (512.0, 512.0))
    f = tmp_path / "traffic.txt"
    f.write_text("# header\n" + bench.summarize_pmc(df, dw) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic("a1024p32w16q_c64") == (1000 * 2 + 512) * 1024
    assert bench.read_traffic("c1024p32w16x_c64") is None  # not in the file
    # measured on other kernel sources: no figure
    f.write_text(f.read_text().replace("source_hash=", "source_hash=0"))
    assert bench.read_traffic("a1024p32w16q_c64") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic("a1024p32w16q_c64") is None


def test_committed_traffic_summary_parses():
    # the committed summary names the step's kernels with a per-launch figure
    with open(bench.TRAFFIC_FILE) as f:
        lines = f.read().splitlines()
    assert any(l.startswith("source_hash=") for l in lines)
    kern = [l for l in lines if l.startswith("kernel=") and ("k_pipe" in l or "k_strip" in l)]
    assert kern
    for l in kern:
        v = float(l.rsplit("hbm_bytes_per_launch=", 1)[1])
        assert v > 0


def test_stats_helper():
    s = bench._stats([3.0, 1.0, 2.0, 10.0])
    assert s == {"min": 1.0, "median": 2.0, "p90": 10.0}
    assert bench._stats([5.0]) == {"min": 5.0, "median": 5.0, "p90": 5.0}


def test_cpu_model_names_the_host():
    name = bench.cpu_model()
    assert isinstance(name, str) and name


def test_summarize_counters_averages_per_kernel(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(str(tmp_path / "c" / "run_counter_collection.csv"), hdr, [
        [PIPE_A, "SQ_LDS_BANK_CONFLICT", 10], [PIPE_A, "SQ_LDS_BANK_CONFLICT", 30],
        [PIPE_A, "SQ_INSTS_LDS", 100], [PIPE_A, "SQ_INSTS_LDS", 100], [COPY, "SQ_INSTS_LDS", 0],
    ])
    out = bench.summarize_counters(str(tmp_path)).splitlines()
    line = [l for l in out if PIPE_A in l][0]
    assert "dispatches=2" in line and "SQ_LDS_BANK_CONFLICT=20" in line and "SQ_INSTS_LDS=100" in line
    assert any(COPY in l and "SQ_INSTS_LDS=0" in l for l in out)
    with pytest.raises(SystemExit):
        bench.summarize_counters(str(tmp_path / "none"))
