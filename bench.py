#!/usr/bin/env python3
"""Benchmark of the FFT hot path on one MI355X.

Workload (one "step"): the 1-D complex-to-complex FFT of 16 signals of
N = 2^20 points (complex64, re/im ~ N(0,1), seed 1), forward then inverse.
N = 2^20 exceeds one workgroup's LDS, so each direction is the two-pass
N1 x N2 = 1024 x 1024 split (pass A: 1024-point column transforms with the
fused W_N^{n2*k1} twiddle; pass B: 1024-point column transforms).

metric  GFLOP/s = sum over transforms of 5*N*log2(N) / step time.
roofline  the dominant kernel's algorithmic bytes per launch (every point
          read once and written once: 2 * 16 * 2^20 * 8 B) over its average
          launch time, timed live with HIP events recorded by the library on
          the exec stream, against MI355X peak HBM (8 TB/s).
cpu_baseline  the FP64 oracle on the host's cores on a bounded sample of the
          same step.

Buffers rotate over >= 1 GiB so that the 256 MB Infinity Cache cannot hold a
step's working set between steps: every step reads its input from HBM.

Other modes (used to make the rocprofv3 summaries under profiles/):
  --mode profile     run warmup + steps only (no CPU baseline), for
                     `rocprofv3 --kernel-trace --stats` and `--pmc` runs;
                     also runs one plain 256 MiB device copy (calibration);
                     --profile-workload image2d|many|dft256 profiles the 4096^2
                     image, the 512 uneven transforms or 65536 x 256 under each
                     one-kernel 256-point method instead of the step
  --mode configs     every benchmarked workload (1024 single, 1024 x 32768,
                     16 x 2^20 forward and inverse, the 4096^2 image, the
                     512 uneven batch in three storage types, 64 x 2^16
                     forward + adjoint), one JSON line of per-workload rates
  --mode transfer    host-to-host: the Table 1 sizes (16 .. 65536, one
                     transform) with the copies included, and a 1 GiB batch
                     through the chunked pipe (copy in, transform, copy out
                     overlapped) against the same chunks run one after another
  --mode ablation    the method the paper improves on (Sec. 2.2: one global
                     radix-2 kernel per butterfly level) against the LDS
                     passes, forward 16 x 2^20, one JSON line
  --summarize-trace DIR         print the kernel-time summary of a trace run
  --summarize-pmc DIR_FETCH DIR_WRITE  print per-kernel HBM traffic
  --summarize-counters DIR      print per-kernel averages of any counters
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 1 << 20
BATCH = 16
SEED = 1
PEAK_HBM_GBS = 8000.0
ROT_BYTES = 1 << 30
COPY_BYTES = 256 << 20
# HIP events are recorded on one step in PROFILE_EVERY of the timed region:
# each recorded event costs a few microseconds of queue time, which would
# otherwise be charged to every step of the wall-clock rate
PROFILE_EVERY = 5
# one-kernel 256-point methods compared in the dft256 profile: the fastest
# LDS butterfly variant, matrix-core stages, cross-lane exchanges
DFT256_SCHEDULES = ("single=r256p8w8_c64", "method=mfma", "method=xlane", "method=xlane_bperm")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_fft_n2p20_b16.txt")


# sources of other kernel families, which the benchmarked step never runs
NOT_IN_STEP = ("many.", "levels.", "mfma.", "xlane.", "variants_c16.")


def kernel_source_hash() -> str:
    """Hash of the sources the benchmarked step's kernels and launches are
    built from; a traffic figure is only valid for the kernels it was
    measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1707_07263_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.startswith(NOT_IN_STEP):
            continue
        if f.endswith((".hpp", ".hip", ".cpp", ".py")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", choices=["bench", "profile", "ablation", "configs", "transfer"],
                    default="bench")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other forms (2-D image, uneven batch in three storage types, "
                         "forward + adjoint pair) after the headline step")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("DIR_FETCH", "DIR_WRITE"))
    ap.add_argument("--summarize-counters", metavar="DIR")
    ap.add_argument("--profile-workload", choices=["step", "image2d", "many", "dft256"], default="step",
                    help="profile mode: the benchmarked step, the 4096x4096 2-D image forward "
                         "transform (tuned schedule, four rotating buffers), the 512 uneven "
                         "complex64 transforms in one exec (tuned schedule: two launches, rotating "
                         "buffers of >= 1 GiB), or 65536 x 256 complex64 forward under each "
                         "one-kernel 256-point method (LDS butterflies, matrix cores, cross-lane)")
    return ap.parse_args(argv)


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------
def _csv_rows(root, suffix):
    rows = []
    for path in glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name: str) -> str:
    name = name.strip()
    for key in ("k_strip", "k_many", "k_scale_copy", "k_twiddle_fp64"):
        if key in name:
            return name
    return name[:120]


def summarize_trace(d: str) -> str:
    rows = _csv_rows(d, "kernel_stats.csv")
    if not rows:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    lines = ["kernel | calls | avg_us | total_ms | pct"]
    for r in sorted(rows, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        calls = int(r["Calls"])
        avg = float(r["AverageNs"]) / 1e3
        tot = float(r["TotalDurationNs"]) / 1e6
        pct = float(r.get("Percentage", 0))
        lines.append(f"{_short(r['Name'])} | {calls} | {avg:.2f} | {tot:.3f} | {pct:.2f}")
    return "\n".join(lines)


def _pmc_per_kernel(d: str, counter: str):
    rows = _csv_rows(d, "counter_collection.csv")
    per = {}
    for r in rows:
        if r.get("Counter_Name", "").strip() != counter:
            continue
        k = _short(r["Kernel_Name"])
        per.setdefault(k, []).append(float(r["Counter_Value"]))
    return per


def summarize_pmc(dfetch: str, dwrite: str) -> str:
    fetch = _pmc_per_kernel(dfetch, "FETCH_SIZE")
    write = _pmc_per_kernel(dwrite, "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    copy_w = [v for k, vs in write.items() if "copy" in k.lower() or "elementwise" in k.lower() for v in vs]
    lines = [f"source_hash={kernel_source_hash()}"]
    if copy_f and copy_w:
        kib = COPY_BYTES / 1024.0
        cf = kib / max(copy_f)
        cw = kib / max(copy_w)
        lines.append(f"copy_calibration fetch_kib={max(copy_f):.1f} write_kib={max(copy_w):.1f} "
                     f"expected_kib={kib:.1f} fetch_scale={cf:.4f} write_scale={cw:.4f}")
    else:
        cf = cw = 1.0
        lines.append("copy_calibration missing fetch_scale=1 write_scale=1")
    for k in sorted(set(fetch) | set(write)):
        f = fetch.get(k, [])
        w = write.get(k, [])
        if not f or not w:
            continue
        af = sum(f) / len(f)
        aw = sum(w) / len(w)
        lines.append(f"kernel={k} dispatches={len(f)} fetch_kib_avg={af:.1f} write_kib_avg={aw:.1f} "
                     f"hbm_bytes_per_launch={(af * cf + aw * cw) * 1024:.0f}")
    return "\n".join(lines)


def summarize_counters(d: str) -> str:
    """Per-kernel average of every counter in a `rocprofv3 --pmc` run."""
    rows = _csv_rows(d, "counter_collection.csv")
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    per = {}
    for r in rows:
        k = _short(r["Kernel_Name"])
        per.setdefault(k, {}).setdefault(r["Counter_Name"].strip(), []).append(float(r["Counter_Value"]))
    lines = []
    for k in sorted(per):
        cs = per[k]
        n = max(len(v) for v in cs.values())
        vals = " ".join(f"{c}={sum(v) / len(v):.0f}" for c, v in sorted(cs.items()))
        lines.append(f"kernel={k} dispatches={n} {vals}")
    return "\n".join(lines)


def variant_kernel_signature(variant: str) -> str:
    """Template arguments of the strip kernel a variant name stands for, as
    rocprofv3 prints them (e.g. a1024p32w16x_c64 ->
    k_strip<1024, 32, 16, 1, 0, true, 1, HIP_vector_type<float, 2u> >,
    a1024p32w16q2_c64 -> k_pipe<1024, 32, 16, 1, 0, true, 0, HIP_vector_type<float, 2u>, 2>)."""
    import re
    m = re.match(r"([rac])(\d+)p(\d+)w(\d+)(q2|q)?(x?)_(c64|f16|bf16)$", variant)
    if not m:
        return variant
    role, L, P, W, q, x, dt = m.groups()
    lm, sm, tw = {"r": (0, 0, "false"), "a": (1, 0, "true"), "c": (1, 1, "false")}[role]
    ts = {"c64": "HIP_vector_type<float, 2u>", "f16": "__half2", "bf16": "mfft::c16bf"}[dt]
    if q:
        return f"k_pipe<{L}, {P}, {W}, {lm}, {sm}, {tw}, {1 if x else 0}, {ts}, {2 if q == 'q2' else 1}>"
    return f"k_strip<{L}, {P}, {W}, {lm}, {sm}, {tw}, {1 if x else 0}, {ts} >"


def read_traffic(kernel_name: str):
    """Scaled HBM bytes per launch of `kernel_name` from the committed pmc
    summary, or None if absent or measured on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        text = f.read().splitlines()
    kv = [l for l in text if l.startswith("source_hash=")]
    if not kv or kv[0].split("=", 1)[1].strip() != kernel_source_hash():
        return None
    sig = variant_kernel_signature(kernel_name)
    for line in text:
        if line.startswith("kernel=") and sig in line:
            for tok in line.split():
                if tok.startswith("hbm_bytes_per_launch="):
                    return float(tok.split("=", 1)[1])
    return None


# ---------------------------------------------------------------------------
# GPU benchmark
# ---------------------------------------------------------------------------
def timing_oracle():
    """The oracle built for this host's CPU (gcc -O3 -march=native, in a
    temporary directory, removed once loaded), or the portable in-tree build
    if that compile fails.  Returns (oracle functions, build description)."""
    import tempfile

    import oracle as portable
    try:
        with tempfile.TemporaryDirectory(prefix="oracle_native_") as d:
            return portable.native(d), "gcc -O3 -march=native -fopenmp"
    except Exception as e:  # no compiler on this host: the portable build
        print(f"[bench] native oracle build failed ({e}); timing the portable build", file=sys.stderr)
        return portable, "gcc -O3 -fopenmp (portable)"


def cpu_baseline(x_np, seconds: float):
    """FP64 oracle on the host cores: forward + inverse of the same 16 x 2^20
    batch, repeated until `seconds` have passed (at least once)."""
    oracle, build = timing_oracle()
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    reps, t0 = 0, time.perf_counter()
    while True:
        y = oracle.fft(x_np)
        oracle.fft(y, inverse=True)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 100:
            break
    flops = reps * 2 * BATCH * 5.0 * N * math.log2(N)
    out = {"value": round(flops / el / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{reps} x (forward + inverse of 16 x 2^20 complex, FP64 radix-2) in {el:.1f} s"}
    # the same oracle on one thread, over single transforms of the batch (a
    # bounded sample of about a quarter of the time above)
    oracle.set_threads(1)
    reps1, t0 = 0, time.perf_counter()
    while True:
        row = x_np[reps1 % BATCH:reps1 % BATCH + 1]
        oracle.fft(oracle.fft(row), inverse=True)
        reps1 += 1
        el1 = time.perf_counter() - t0
        if el1 >= seconds / 4 or reps1 >= 400:
            break
    oracle.set_threads(cores)
    out["single_thread"] = {"value": round(reps1 * 2 * 5.0 * N * math.log2(N) / el1 / 1e9, 3),
                            "sample": f"{reps1} x (forward + inverse of one 2^20 transform) in {el1:.1f} s"}
    out["cpu_model"] = cpu_model()
    out["build"] = build
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _stats(v):
    """min, median and 90th percentile of per-repetition times."""
    v = sorted(v)
    q = lambda f: v[min(len(v) - 1, int(math.ceil(f * len(v))) - 1)]
    return {"min": round(v[0], 2), "median": round(q(0.5), 2), "p90": round(q(0.9), 2)}


def _time_plans(capi, torch, plans, nbytes_io, reps):
    """Device time of running `plans` (each (handle, in/out byte count)) back
    to back, over rotating buffers of >= 1 GiB; per-launch HIP events
    recorded by the library on the exec stream.  Returns the mean and the
    per-repetition times (each repetition synchronised and read on its own)."""
    stream = torch.cuda.current_stream().cuda_stream
    # >= 1 GiB of rotating buffers (at most 64 sets: the latency-bound case
    # is tiny and its working set stays cache-resident regardless)
    nsets = min(64, max(2, math.ceil(ROT_BYTES / max(nbytes_io, 1))))
    bufs = []
    for _ in range(nsets):
        bufs.append([(torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1),
                      torch.empty(n, dtype=torch.uint8, device="cuda")) for _, n in plans])
    for i in range(3):
        for (h, _), (x, y) in zip(plans, bufs[i % nsets]):
            capi.fft_exec(h, x.data_ptr(), y.data_ptr(), stream)
    torch.cuda.synchronize()
    for h, _ in plans:
        capi.fft_profile_enable(h, 1)
    passes = [capi.fft_plan_info(h)["passes"] for h, _ in plans]
    per_rep, total = [], 0.0
    for i in range(reps):
        for (h, _), (x, y) in zip(plans, bufs[i % nsets]):
            capi.fft_exec(h, x.data_ptr(), y.data_ptr(), stream)
        torch.cuda.synchronize()
        cum = 0.0
        for (h, _), np_ in zip(plans, passes):
            capi.fft_profile_collect(h)
            cum += sum(1e3 * capi.fft_profile_read(h, p)[0] for p in range(np_))
        per_rep.append(cum - total)
        total = cum
    for h, _ in plans:
        capi.fft_profile_enable(h, 0)
    del bufs
    torch.cuda.empty_cache()
    return total / reps, per_rep


def _time_torch_fft(torch, fn, shapes, reps):
    """Context only: the vendor FFT that torch calls on this GPU (hipFFT /
    rocFFT), timed with torch's events on the same shapes over rotating
    inputs of >= 1 GiB.  Returns per-repetition microseconds, or an error."""
    try:
        nbytes = sum(8 * math.prod(sh) for sh in shapes)
        nsets = min(16, max(2, math.ceil(ROT_BYTES / max(2 * nbytes, 1))))
        sets = [[torch.randn(*sh, dtype=torch.complex64, device="cuda") for sh in shapes] for _ in range(nsets)]
        for i in range(3):
            fn(*sets[i % nsets])
        torch.cuda.synchronize()
        out = []
        for i in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(*sets[i % nsets])
            e1.record()
            torch.cuda.synchronize()
            out.append(1e3 * e0.elapsed_time(e1))
        del sets
        torch.cuda.empty_cache()
        return out
    except Exception as ex:  # context only: a vendor failure is reported, not raised
        torch.cuda.empty_cache()
        return str(ex)[:200]


def configs_report(capi, torch, reps):
    """Rates of every benchmarked workload with its tuned schedule (inputs'
    values do not change the timing; shapes and sizes are the workloads')."""
    from paper_1707_07263_amd import autotune, workloads
    out = {"mode": "configs", "reps": reps, "peak_GBps": PEAK_HBM_GBS, "configs": []}

    def add(name, plans, dtype_bytes, note="", vendor=None):
        nbytes = sum(n for _, n in plans)
        us, per_rep = _time_plans(capi, torch, plans, 2 * nbytes, reps)
        flops = sum(capi.fft_plan_info(h)["flops"] for h, _ in plans)
        moved = sum(sum(capi.fft_plan_info(h)["bytes_pass"]) for h, _ in plans)
        minimum = sum(capi.fft_plan_info(h)["bytes_min"] for h, _ in plans)
        out["configs"].append({
            "workload": name, "us": round(us, 2), "GFLOPs": round(flops / (us * 1e-6) / 1e9, 1),
            "method_GBps": round(moved / (us * 1e-6) / 1e9, 1),
            "method_frac": round(moved / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
            "min_GBps": round(minimum / (us * 1e-6) / 1e9, 1),
            "us_reps": _stats(per_rep),
            "schedules": [capi.fft_plan_info(h)["pass_variant"] for h, _ in plans], "note": note})
        for h, _ in plans:
            capi.fft_destroy(h)
        print(f"[bench] {name}: {us:.2f} us", file=sys.stderr, flush=True)
        if vendor is not None:
            fn, shapes, what = vendor
            t = _time_torch_fft(torch, fn, shapes, reps)
            out["configs"][-1]["torch_fft"] = ({"what": what, "us": _stats(t)} if isinstance(t, list)
                                               else {"what": what, "error": t})
            print(f"[bench]   torch.fft context: {out['configs'][-1]['torch_fft']}", file=sys.stderr, flush=True)

    def plan(shape, batch, dtype, direction, scale=None):
        h = capi.fft_plan_ex(list(shape), batch, len(shape), dtype, direction,
                             autotune.schedule_for(list(shape), batch, dtype))
        if scale is not None:
            capi.fft_set_scale(h, scale)
        n = batch
        for s_ in shape:
            n *= s_
        return h, n * (8 if dtype == capi.FFT_C64 else 4)

    C64 = capi.FFT_C64
    tf = torch.fft
    add("1-D N=1024 batch 1, forward (latency-bound)", [plan([1024], 1, C64, capi.FFT_FORWARD)], 8,
        vendor=(lambda x: tf.fft(x), [(1024,)], "fft"))
    add("1-D N=1024 batch 32768, forward", [plan([1024], 32768, C64, capi.FFT_FORWARD)], 8,
        vendor=(lambda x: tf.fft(x), [(32768, 1024)], "fft"))
    add("1-D N=2^20 batch 16, forward then inverse",
        [plan([N], BATCH, C64, capi.FFT_FORWARD), plan([N], BATCH, C64, capi.FFT_INVERSE)], 8,
        vendor=(lambda x: tf.ifft(tf.fft(x)), [(BATCH, N)], "ifft(fft(x))"))
    for dt, name in ((capi.FFT_C16F, "fp16 pairs"), (capi.FFT_C16BF, "bf16 pairs")):
        add(f"1-D N=2^20 batch 16, forward then inverse, {name}",
            [plan([N], BATCH, dt, capi.FFT_FORWARD), plan([N], BATCH, dt, capi.FFT_INVERSE)], 4)
    add("2-D 4096x4096 image, forward", [plan([4096, 4096], 1, C64, capi.FFT_FORWARD)], 8,
        vendor=(lambda x: tf.fft2(x), [(4096, 4096)], "fft2"))
    add("1-D N=2^28 batch 1, forward (three passes, GPU FP64 twiddles)",
        [plan([1 << 28], 1, C64, capi.FFT_FORWARD)], 8,
        vendor=(lambda x: tf.fft(x), [(1 << 28,)], "fft"))
    sizes = [int(v) for v in workloads.uneven_sizes(512, 8, 16, seed=3)]
    counts = {}
    for v in sizes:
        counts[v] = counts.get(v, 0) + 1
    grouped = [(c, n) for n, c in sorted(counts.items())]
    for dt, name in ((C64, "complex64"), (capi.FFT_C16F, "fp16 pairs"), (capi.FFT_C16BF, "bf16 pairs")):
        h = capi.fft_plan_many_ex(sizes, dt, capi.FFT_FORWARD, autotune.many_schedule_for(sizes, dt))
        add(f"512 uneven 2^8..2^16 in one exec (persistent kernel, two launches), {name}", [(h, sum(sizes) * (8 if dt == C64 else 4))],
            8 if dt == C64 else 4,
            vendor=((lambda *xs: [tf.fft(x) for x in xs]), grouped, "fft per length (9 batched calls)")
            if dt == C64 else None)
    add("64 x 2^16 forward + adjoint backward (autograd pair)",
        [plan([1 << 16], 64, C64, capi.FFT_FORWARD), plan([1 << 16], 64, C64, capi.FFT_INVERSE, 1.0)], 8,
        vendor=(lambda x: tf.ifft(tf.fft(x), norm="forward"), [(64, 1 << 16)], "ifft(fft(x), norm=forward)"))
    return out


def _rel_l2(got, ref):
    """||got - ref|| / ||ref|| in FP64 (an exactly zero reference needs a zero output)."""
    import numpy as np
    g = np.asarray(got, dtype=np.complex128).reshape(-1)
    r = np.asarray(ref, dtype=np.complex128).reshape(-1)
    nr = np.linalg.norm(r)
    return float(np.linalg.norm(g - r) / nr) if nr > 0 else float(np.linalg.norm(g))


def _to_c128(t):
    """A device tensor of complex64, or of 16-bit pairs [..., 2], as numpy complex128."""
    import numpy as np
    import torch
    a = t.detach().cpu()
    if a.dtype in (torch.float16, torch.bfloat16):
        f = a.float().numpy()
        return f[..., 0].astype(np.float64) + 1j * f[..., 1].astype(np.float64)
    return a.numpy().astype(np.complex128)


def forms_report(capi, torch, reps):
    """Every form of the method beside the headline step, each on its own
    workload: device time (per-launch HIP events over rotating buffers of
    >= 1 GiB), method bytes and fraction of peak HBM, and the error of the
    same plan's output against the FP64 oracle on that workload's seeded
    input (per length for the uneven batch).  The oracle runs after the GPU
    timing, on the host."""
    import numpy as np

    import oracle
    from paper_1707_07263_amd import autotune, workloads
    C64, F16, BF16 = capi.FFT_C64, capi.FFT_C16F, capi.FFT_C16BF
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    out = {}

    def rate(plans, nbytes_io):
        us, per_rep = _time_plans(capi, torch, plans, nbytes_io, reps)
        moved = sum(sum(capi.fft_plan_info(h)["bytes_pass"]) for h, _ in plans)
        flops = sum(capi.fft_plan_info(h)["flops"] for h, _ in plans)
        return {"us": round(us, 2), "us_reps": _stats(per_rep),
                "GFLOPs": round(flops / (us * 1e-6) / 1e9, 1),
                "method_bytes": moved, "method_GBps": round(moved / (us * 1e-6) / 1e9, 1),
                "frac_of_peak": round(moved / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                "kernels": [capi.fft_plan_info(h)["pass_variant"] for h, _ in plans]}

    def run(h, x):
        y = torch.empty_like(x)
        capi.fft_exec(h, x.data_ptr(), y.data_ptr(), st)
        torch.cuda.synchronize()
        return y

    # the 4096 x 4096 image, rows then columns (Sec. 2.3.2)
    shape = [4096, 4096]
    h = capi.fft_plan_ex(shape, 1, 2, C64, capi.FFT_FORWARD, autotune.schedule_for(shape, 1, C64))
    z = workloads.speckle_image(4096, 4096, seed=2).astype(np.complex64)
    got = _to_c128(run(h, torch.from_numpy(z).to(dev)))
    r = rate([(h, z.nbytes)], 2 * z.nbytes)
    capi.fft_destroy(h)
    r["rel_l2_vs_oracle"] = _rel_l2(got, oracle.fft2(z))
    r["tolerance"] = 2.4e-5
    out["image_4096x4096_c64"] = r
    print(f"[bench] form image 4096^2: {r['us']} us, rel-L2 {r['rel_l2_vs_oracle']:.2e}",
          file=sys.stderr, flush=True)

    # 512 uneven lengths 2^8..2^16 in one launch, three storage types
    sizes, packed = workloads.uneven_batch(512, 8, 16, seed=3)
    sl = [int(v) for v in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    for dt, name, tol in ((C64, "c64", None), (F16, "f16", 1e-3), (BF16, "bf16", 8e-3)):
        h = capi.fft_plan_many_ex(sl, dt, capi.FFT_FORWARD, autotune.many_schedule_for(sl, dt))
        if dt == C64:
            xin = packed.astype(np.complex64)
            xt = torch.from_numpy(xin).to(dev)
        else:
            tdt = torch.float16 if dt == F16 else torch.bfloat16
            pairs = np.stack([packed.real, packed.imag], -1).astype(np.float32)
            xt = torch.from_numpy(pairs).to(tdt).to(dev)
            xin = _to_c128(xt)  # the values the GPU holds: the oracle's input
        got = _to_c128(run(h, xt))
        wd = capi.fft_many_watchdog(h, 1)
        esz = 8 if dt == C64 else 4
        r = rate([(h, sum(sl) * esz)], 2 * sum(sl) * esz)
        capi.fft_destroy(h)
        ref = oracle.fft_many(xin, sizes)
        per = {}
        for lg in range(8, 17):
            sel = [i for i in range(len(sl)) if sl[i] == 1 << lg]
            if sel:
                per[f"2^{lg}"] = max(_rel_l2(got[off[i]:off[i + 1]], ref[off[i]:off[i + 1]]) for i in sel)
        r["rel_l2_vs_oracle_max_per_length"] = per
        r["rel_l2_vs_oracle_max"] = max(per.values())
        r["tolerance"] = "1e-6*log2(N) per transform" if tol is None else tol
        r["watchdog"] = "ok" if wd == capi.FFT_OK else "expired"
        r["points"] = sum(sl)
        out[f"uneven512_{name}"] = r
        print(f"[bench] form 512 uneven {name}: {r['us']} us, max rel-L2 {r['rel_l2_vs_oracle_max']:.2e}",
              file=sys.stderr, flush=True)

    # differentiable pair: 64 x 2^16 forward, then the adjoint (inverse
    # direction, scale 1) of g = 2 W^2 (F x), the gradient of sum |W F x|^2
    x, w, _ = workloads.autograd_case(64, 1 << 16, seed=4)
    x64 = x.astype(np.complex64)
    hf = capi.fft_plan_ex([1 << 16], 64, 1, C64, capi.FFT_FORWARD, autotune.schedule_for([1 << 16], 64, C64))
    ha = capi.fft_plan_ex([1 << 16], 64, 1, C64, capi.FFT_INVERSE, autotune.schedule_for([1 << 16], 64, C64))
    capi.fft_set_scale(ha, 1.0)
    y = run(hf, torch.from_numpy(x64).to(dev))
    g = (2.0 * torch.from_numpy(w.astype(np.float32)).to(dev) ** 2) * y
    grad = _to_c128(run(ha, g))
    yc = _to_c128(y)
    nb = x64.nbytes
    r = rate([(hf, nb), (ha, nb)], 4 * nb)
    capi.fft_destroy(hf)
    capi.fft_destroy(ha)
    ref_y = oracle.fft(x64)
    r["rel_l2_forward_vs_oracle"] = _rel_l2(yc, ref_y)
    r["rel_l2_gradient_vs_oracle"] = _rel_l2(grad, oracle.adjoint(2.0 * w ** 2 * ref_y))
    r["tolerance"] = {"forward": 1.6e-5, "gradient": 5e-5}
    out["autograd_64x2^16_fwd_adjoint"] = r
    print(f"[bench] form 64 x 2^16 forward + adjoint: {r['us']} us, forward rel-L2 "
          f"{r['rel_l2_forward_vs_oracle']:.2e}, gradient {r['rel_l2_gradient_vs_oracle']:.2e}",
          file=sys.stderr, flush=True)
    return out


def transfer_report(capi, torch, reps):
    """End-to-end host-to-host timings (pinned host memory)."""
    import statistics
    out = {"mode": "transfer", "reps": reps, "table1": [], "pipe": {}}
    st = torch.cuda.current_stream().cuda_stream
    for lg in (4, 6, 8, 10, 12, 14, 16):
        n = 1 << lg
        h = capi.fft_plan([n], 1, 1, capi.FFT_C64, capi.FFT_FORWARD)
        xh = torch.randn(n, dtype=torch.complex64).pin_memory()
        yh = torch.empty_like(xh).pin_memory()
        xd = torch.empty(n, dtype=torch.complex64, device="cuda")
        yd = torch.empty_like(xd)
        e2e, dev_only = [], []
        for i in range(reps + 5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xd.copy_(xh, non_blocking=True)
            capi.fft_exec(h, xd.data_ptr(), yd.data_ptr(), st)
            yh.copy_(yd, non_blocking=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            capi.fft_exec(h, xd.data_ptr(), yd.data_ptr(), st)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if i >= 5:
                e2e.append((t1 - t0) * 1e6)
                dev_only.append((t2 - t1) * 1e6)
        capi.fft_destroy(h)
        out["table1"].append({"n": n, "end_to_end_us": round(statistics.median(e2e), 2),
                              "transform_only_us": round(statistics.median(dev_only), 2)})
        print(f"[bench] host-to-host N={n}: {statistics.median(e2e):.1f} us", file=sys.stderr, flush=True)
    # 1 GiB of 2^16-point signals through the pipe, 32 MiB chunks
    n, batch, chunks = 1 << 16, 64, 32
    h = capi.fft_plan([n], batch, 1, capi.FFT_C64, capi.FFT_FORWARD)
    xh = torch.randn(chunks, batch, n, dtype=torch.complex64).pin_memory()
    yh = torch.empty_like(xh).pin_memory()
    total_bytes = 2 * xh.numel() * 8
    res = {}
    for slots in (1, 3):
        if slots == 1:
            # one after another: copy in, transform, copy out per chunk
            xd = torch.empty(batch, n, dtype=torch.complex64, device="cuda")
            yd = torch.empty_like(xd)
            ts = []
            for r in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for c in range(chunks):
                    xd.copy_(xh[c], non_blocking=True)
                    capi.fft_exec(h, xd.data_ptr(), yd.data_ptr(), st)
                    yh[c].copy_(yd, non_blocking=True)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
        else:
            p = capi.fft_pipe_create(h, slots)
            ts = []
            for r in range(3):
                t0 = time.perf_counter()
                capi.fft_pipe_exec(p, xh.data_ptr(), yh.data_ptr(), chunks)
                capi.fft_pipe_wait(p)
                ts.append(time.perf_counter() - t0)
            capi.fft_pipe_destroy(p)
        t = min(ts)
        res["serial" if slots == 1 else f"pipe_{slots}_slots"] = {
            "ms": round(t * 1e3, 3), "host_GBps": round(total_bytes / t / 1e9, 2),
            "GFLOPs": round(5.0 * n * 16 * batch * chunks / t / 1e9, 1)}
    capi.fft_destroy(h)
    out["pipe"] = {"workload": "32 chunks of 64 x 2^16 complex64 (1 GiB in, 1 GiB out), pinned", **res}
    return out


def ablation(capi, torch, lds_plan, sets, nsets, stream, reps):
    """Forward 16 x 2^20 with the LDS passes and with one radix-2 kernel per
    level (log2 N = 20 launches, each moving every point), timed alike."""
    lev = capi.fft_plan_ex([N], BATCH, 1, capi.FFT_C64, capi.FFT_FORWARD, "method=levels")
    out = {"ablation": "per-level global-memory radix-2 (paper Sec. 2.2) vs LDS-resident passes",
           "workload": "1-D C2C forward, N=2^20, batch 16, complex64, N(0,1) seed 1",
           "reps": reps}
    res = {}
    for name, plan in (("lds", lds_plan), ("levels", lev)):
        info = capi.fft_plan_info(plan)
        for i in range(3):
            xi, yi, _ = sets[i % nsets]
            capi.fft_exec(plan, xi.data_ptr(), yi.data_ptr(), stream)
        torch.cuda.synchronize()
        capi.fft_profile_enable(plan, reps)
        for i in range(reps):
            xi, yi, _ = sets[i % nsets]
            capi.fft_exec(plan, xi.data_ptr(), yi.data_ptr(), stream)
        torch.cuda.synchronize()
        capi.fft_profile_collect(plan)
        us = sum(1e3 * capi.fft_profile_read(plan, p)[0] / reps for p in range(info["passes"]))
        moved = sum(info["bytes_pass"])
        res[name] = yi.clone()
        out[name] = {"us": round(us, 2), "launches": N.bit_length() - 1 if name == "levels" else info["passes"],
                     "GFLOPs": round(info["flops"] / (us * 1e-6) / 1e9, 1),
                     "bytes_moved": moved, "GBps": round(moved / (us * 1e-6) / 1e9, 1)}
        capi.fft_profile_enable(plan, 0)
    out["speedup_lds_over_levels"] = round(out["levels"]["us"] / out["lds"]["us"], 2)
    out["rel_l2_levels_vs_lds"] = (torch.linalg.vector_norm(res["levels"] - res["lds"]) /
                                   torch.linalg.vector_norm(res["lds"])).item()
    capi.fft_destroy(lev)
    out["matrix_cores"] = mfma_report(capi, torch, reps)
    return out


def mfma_report(capi, torch, reps):
    """256-point transforms: radix-16 stages as matrix-core products, and the
    exchange between them as cross-lane moves (DPP/ds_swizzle, ds_bpermute),
    against the fastest one-kernel butterfly variant for the same batch, with data
    from HBM (65536 signals, rotating buffers), resident in the 256 MB
    Infinity Cache (16384 signals, 64 MB in and out) and in L2 (2048
    signals, one buffer pair)."""
    names = [capi.fft_variant_name(i) for i in range(capi.fft_variant_count())]
    butterflies = [n for n in names if n.startswith("r256p") and n.endswith("_c64")]
    res = {}
    for batch, label, rotate in ((65536, "hbm", True), (16384, "infinity_cache_resident", False),
                                 (2048, "cache_resident", False)):
        nb = batch * 256 * 8
        nsets = max(2, math.ceil(ROT_BYTES / (2 * nb))) if rotate else 1
        bufs = [(torch.randn(batch * 256, dtype=torch.complex64, device="cuda"),
                 torch.empty(batch * 256, dtype=torch.complex64, device="cuda")) for _ in range(nsets)]
        st = torch.cuda.current_stream().cuda_stream

        def timed(sched):
            h = capi.fft_plan_ex([256], batch, 1, capi.FFT_C64, capi.FFT_FORWARD, sched)
            for i in range(3):
                capi.fft_exec(h, bufs[i % nsets][0].data_ptr(), bufs[i % nsets][1].data_ptr(), st)
            torch.cuda.synchronize()
            capi.fft_profile_enable(h, reps)
            for i in range(reps):
                capi.fft_exec(h, bufs[i % nsets][0].data_ptr(), bufs[i % nsets][1].data_ptr(), st)
            torch.cuda.synchronize()
            capi.fft_profile_collect(h)
            us = 1e3 * capi.fft_profile_read(h, 0)[0] / reps
            capi.fft_destroy(h)
            return us

        best = min((timed(f"single={v}"), v) for v in butterflies)
        row = {"butterflies": {"us": round(best[0], 2), "variant": best[1],
                               "GBps": round(2 * nb / (best[0] * 1e-6) / 1e9, 1), "of": len(butterflies)}}
        for key, method, variant in (("matrix_cores", "mfma", "mfma_dft256"),
                                     ("cross_lane_dpp", "xlane", "xlane_dft256"),
                                     ("cross_lane_bpermute", "xlane_bperm", "xlane_bperm_dft256")):
            t = timed(f"method={method}")
            row[key] = {"us": round(t, 2), "variant": variant, "GBps": round(2 * nb / (t * 1e-6) / 1e9, 1)}
            row[f"{key}_over_butterflies_time"] = round(t / best[0], 3)
        res[f"{batch}x256_{label}"] = row
        del bufs
    return res


def main(argv=None) -> int:
    args = parse_args(argv)
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return 0
    if args.summarize_pmc:
        print(summarize_pmc(*args.summarize_pmc))
        return 0
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters))
        return 0
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus N > 1 is not supported. The batch of "
              "independent transforms would shard by rows with no communication.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1707_07263_amd import capi, workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    capi.load()
    print(f"[bench] generating 16 x 2^20 complex64 input (seed {SEED})", file=sys.stderr, flush=True)
    x_np = workloads.normal_batch(N, BATCH, seed=SEED).astype(np.complex64)
    x = torch.from_numpy(x_np).to(dev)
    set_bytes = 3 * x.numel() * 8
    nsets = max(1, math.ceil(ROT_BYTES / set_bytes))
    sets = []
    for _ in range(nsets):
        sets.append((x.clone(), torch.empty_like(x), torch.empty_like(x)))
    del x
    from paper_1707_07263_amd import autotune
    sched = autotune.schedule_for([N], BATCH, capi.FFT_C64)  # committed tuner result, else built-in
    fwd = capi.fft_plan_ex([N], BATCH, 1, capi.FFT_C64, capi.FFT_FORWARD, sched)
    inv = capi.fft_plan_ex([N], BATCH, 1, capi.FFT_C64, capi.FFT_INVERSE, sched)
    info_f = capi.fft_plan_info(fwd)
    info_i = capi.fft_plan_info(inv)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step(i):
        xi, yi, zi = sets[i % nsets]
        capi.fft_exec(fwd, xi.data_ptr(), yi.data_ptr(), stream)
        capi.fft_exec(inv, yi.data_ptr(), zi.data_ptr(), stream)

    image_only = args.mode == "profile" and args.profile_workload in ("image2d", "many", "dft256")
    for i in range(0 if image_only else args.warmup):
        step(i)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    if args.mode == "ablation":
        print(json.dumps(ablation(capi, torch, fwd, sets, nsets, stream, args.steps)))
        return 0
    if args.mode == "configs":
        del sets
        torch.cuda.empty_cache()
        print(json.dumps(configs_report(capi, torch, args.steps)))
        return 0
    if args.mode == "transfer":
        del sets
        torch.cuda.empty_cache()
        print(json.dumps(transfer_report(capi, torch, args.steps)))
        return 0

    if args.mode == "profile":
        if args.profile_workload == "image2d":
            del sets
            torch.cuda.empty_cache()
            shape = [4096, 4096]
            h2 = capi.fft_plan_ex(shape, 1, 2, capi.FFT_C64, capi.FFT_FORWARD,
                                  autotune.schedule_for(shape, 1, capi.FFT_C64))
            imgs = [(torch.randn(4096 * 4096, dtype=torch.complex64, device=dev),
                     torch.empty(4096 * 4096, dtype=torch.complex64, device=dev)) for _ in range(4)]
            for i in range(args.warmup + args.steps):
                xi, yi = imgs[i % 4]
                capi.fft_exec(h2, xi.data_ptr(), yi.data_ptr(), stream)
            torch.cuda.synchronize()
            capi.fft_destroy(h2)
            del imgs
        elif args.profile_workload == "many":
            del sets
            torch.cuda.empty_cache()
            sizes = [int(v) for v in workloads.uneven_sizes(512, 8, 16, seed=3)]
            hm = capi.fft_plan_many_ex(sizes, capi.FFT_C64, capi.FFT_FORWARD,
                                       autotune.many_schedule_for(sizes, capi.FFT_C64))
            pts = sum(sizes)
            nm = max(2, math.ceil(ROT_BYTES / (16 * pts)))
            bufs = [(torch.randn(pts, dtype=torch.complex64, device=dev),
                     torch.empty(pts, dtype=torch.complex64, device=dev)) for _ in range(nm)]
            for i in range(args.warmup + args.steps):
                xi, yi = bufs[i % nm]
                capi.fft_exec(hm, xi.data_ptr(), yi.data_ptr(), stream)
            torch.cuda.synchronize()
            capi.fft_destroy(hm)
            del bufs
        elif args.profile_workload == "dft256":
            del sets
            torch.cuda.empty_cache()
            batch = 65536
            nb = batch * 256 * 8
            nd = max(2, math.ceil(ROT_BYTES / (2 * nb)))
            bufs = [(torch.randn(batch * 256, dtype=torch.complex64, device=dev),
                     torch.empty(batch * 256, dtype=torch.complex64, device=dev)) for _ in range(nd)]
            for sched in DFT256_SCHEDULES:
                hd = capi.fft_plan_ex([256], batch, 1, capi.FFT_C64, capi.FFT_FORWARD, sched)
                for i in range(args.warmup + args.steps):
                    xi, yi = bufs[i % nd]
                    capi.fft_exec(hd, xi.data_ptr(), yi.data_ptr(), stream)
                torch.cuda.synchronize()
                capi.fft_destroy(hd)
            del bufs
        else:
            for i in range(args.steps):
                step(i)
        torch.cuda.synchronize()
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] profile mode: {args.steps} steps + one {COPY_BYTES >> 20} MiB copy", file=sys.stderr)
        return 0

    timed_execs = (args.steps + PROFILE_EVERY - 1) // PROFILE_EVERY
    for plan in (fwd, inv):
        capi.fft_profile_enable(plan, timed_execs)
        capi.fft_profile_sample(plan, PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    capi.fft_profile_collect(fwd)
    capi.fft_profile_collect(inv)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)

    # per-kernel launch times from the library's HIP events
    kernels = []
    for plan, info, dname in ((fwd, info_f, "forward"), (inv, info_i, "inverse")):
        for p in range(info["passes"]):
            ms, cnt = capi.fft_profile_read(plan, p)
            kernels.append({"direction": dname, "pass": p, "variant": info["pass_variant"][p],
                            "avg_us": 1e3 * ms / max(cnt, 1), "launches": cnt,
                            "bytes": info["bytes_pass"][p], "total_ms": ms})
    # the dominant kernel: the variant with the largest total time over every
    # launch in the timed region (both directions), as rocprofv3 groups them
    per_kernel = {}
    for k in kernels:
        e = per_kernel.setdefault(k["variant"], {"variant": k["variant"], "total_ms": 0.0,
                                                 "launches": 0, "bytes": k["bytes"]})
        e["total_ms"] += k["total_ms"]
        e["launches"] += k["launches"]
    dom = max(per_kernel.values(), key=lambda k: k["total_ms"])
    dom["avg_us"] = 1e3 * dom["total_ms"] / max(dom["launches"], 1)
    achieved = dom["bytes"] / (dom["avg_us"] * 1e-6) / 1e9
    traffic = read_traffic(dom["variant"])

    # round trip of the last step's buffers as a sanity check
    xi, yi, zi = sets[(args.warmup + args.steps - 1) % nsets]
    rt = (torch.linalg.vector_norm(zi - xi) / torch.linalg.vector_norm(xi)).item()
    y_gpu = yi.cpu().numpy()
    z_gpu = zi.cpu().numpy()

    flops_step = info_f["flops"] + info_i["flops"]
    value = flops_step / (ms_per_step * 1e-3) / 1e9
    result = {
        "metric": "GFLOP/s (5N log2N/t), 1-D C2C FFT forward+inverse",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1-D C2C FFT forward then inverse, N=2^20 (four-step 1024x1024), "
                               "batch 16, complex64, N(0,1) seed 1",
                   "n": N, "batch": BATCH, "passes_per_direction": info_f["passes"],
                   "schedule": sched or "built-in", "variants": info_f["pass_variant"],
                   "hbm_bytes_moved_per_step": 2 * sum(info_f["bytes_pass"]),
                   "effective_GBps": round(2 * sum(info_f["bytes_pass"]) / (ms_per_step * 1e-3) / 1e9, 1),
                   "rotating_sets": nsets, "round_trip_rel_l2": rt},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": dom["variant"], "kernel_avg_us": round(dom["avg_us"], 3),
                     "kernel_launches": dom["launches"], "kernel_bytes_per_launch": dom["bytes"],
                     "timed_steps": f"HIP events on 1 step in {PROFILE_EVERY} of the {args.steps} timed steps",
                     "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT),
                     "kernels": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in kk.items()}
                                 for kk in kernels]},
    }
    capi.fft_destroy(fwd)
    capi.fft_destroy(inv)
    del sets
    torch.cuda.empty_cache()
    # error of the step's results against the FP64 oracle: the forward output
    # against eq. 1 of the input, the inverse output against eq. 2 of the GPU
    # forward output (per transform; the batch maximum)
    import oracle
    ref_y = oracle.fft(x_np)
    ref_z = oracle.fft(y_gpu, inverse=True)
    result["config"]["rel_l2_vs_oracle"] = {
        "forward_max": max(_rel_l2(y_gpu[b], ref_y[b]) for b in range(BATCH)),
        "inverse_max": max(_rel_l2(z_gpu[b], ref_z[b]) for b in range(BATCH)),
        "tolerance": 2.0e-5}
    del ref_y, ref_z
    if not args.no_forms:
        result["forms"] = forms_report(capi, torch, max(10, min(args.steps, 20)))
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(x_np, args.cpu_seconds)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
