"""Schedule autotuner for the FFT plans.

A plan's schedule is a string understood by fft_plan_ex / fft_plan_many_ex
(the split N1, and the kernel variant of each pass; or, for batched uneven
sizes, points per lane, workgroup size, two-pass threshold and queue order).
The tuner times candidates on the GPU with the library's own per-launch HIP
events and keeps the fastest:

* one-pass and 2-D plans: every compiled variant of each pass, one pass at a
  time with the others fixed (coordinate descent, two sweeps);
* 1-D two-pass plans: every split N1 x N2 whose halves have variants, then
  coordinate descent over the first- and second-pass variants of the best
  splits;
* batched plans: the cross product of the compiled persistent-kernel
  variants, two-pass thresholds and queue orders.

Inputs rotate over >= 1 GiB of buffers so each timed launch reads HBM, not
the Infinity Cache.  Results go to a JSON cache keyed by GPU architecture and
problem; `schedule_for` / `many_schedule_for` look them up for the API.
"""
from __future__ import annotations

import json
import math
import re
import os
import threading
import time

from . import capi

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_PATH = os.environ.get("MI355FFT_TUNE_CACHE", os.path.join(HERE, "tuned_schedules.json"))
ARCH = "gfx950"
_lock = threading.Lock()
_cache = None

ROLE_ROW, ROLE_A, ROLE_COL, ROLE_COL_TW, ROLE_ROWCOL = 0, 1, 2, 3, 4


def _load_cache() -> dict:
    global _cache
    if _cache is None:
        try:
            with open(CACHE_PATH) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def _key(kind, shape, batch, dtype):
    return f"{ARCH}|{kind}|{'x'.join(str(int(s)) for s in shape)}|{int(batch)}|{int(dtype)}"


def _many_key(sizes, dtype):
    import hashlib
    h = hashlib.sha1(",".join(str(int(s)) for s in sizes).encode()).hexdigest()[:16]
    return f"{ARCH}|many|{len(sizes)}|{h}|{int(dtype)}"


def schedule_for(shape, batch, dtype):
    """Tuned schedule string for a strided plan, or None."""
    with _lock:
        e = _load_cache().get(_key("plan", shape, batch, dtype))
    return None if e is None else e["schedule"]


def many_schedule_for(sizes, dtype):
    with _lock:
        e = _load_cache().get(_many_key(sizes, dtype))
    return None if e is None else e["schedule"]


def save(entries: dict, path: str | None = None) -> None:
    path = path or CACHE_PATH
    with _lock:
        c = dict(_load_cache())
        c.update(entries)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        global _cache
        _cache = c


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------
class _Buffers:
    """Rotating input/output sets of >= 1 GiB in total."""

    def __init__(self, elems: int, esize: int, torch):
        self.torch = torch
        set_bytes = 2 * elems * esize
        self.n = max(2, math.ceil((1 << 30) / set_bytes))
        words = elems * esize // 4
        self.sets = [(torch.randn(words, device="cuda"), torch.empty(words, device="cuda"))
                     for _ in range(self.n)]

    def ptrs(self, i):
        a, b = self.sets[i % self.n]
        return a.data_ptr(), b.data_ptr()


def _time_handle(h, bufs, reps, warm=2):
    import torch
    st = torch.cuda.current_stream().cuda_stream
    for i in range(warm):
        capi.fft_exec(h, *bufs.ptrs(i), st)
    torch.cuda.synchronize()
    capi.fft_profile_enable(h, reps)
    for i in range(reps):
        capi.fft_exec(h, *bufs.ptrs(warm + i), st)
    torch.cuda.synchronize()
    capi.fft_profile_collect(h)
    info = capi.fft_plan_info(h)
    per = []
    for p in range(info["passes"]):
        ms, n = capi.fft_profile_read(h, p)
        per.append(1e3 * ms / max(n, 1))
    capi.fft_profile_enable(h, 0)
    return per, info


def _variants():
    out = []
    for i in range(capi.fft_variant_count()):
        d = capi.fft_variant_describe(i)
        d["name"] = capi.fft_variant_name(i)
        out.append(d)
    return out


def _time_schedule(shape, batch, dtype, sched, bufs, reps):
    try:
        h = capi.fft_plan_ex(list(shape), batch, len(shape), dtype, capi.FFT_FORWARD, sched)
    except capi.FFTError:
        return None
    try:
        per, info = _time_handle(h, bufs, reps)
    finally:
        capi.fft_destroy(h)
    return per, info


def tune_plan(shape, batch, dtype=capi.FFT_C64, reps=10, verbose=False):
    """Tune a strided plan; returns (schedule string, per-pass microseconds)."""
    import torch
    shape = [int(s) for s in shape]
    n = 1
    for s in shape:
        n *= s
    esize = 8 if dtype == capi.FFT_C64 else 4
    bufs = _Buffers(n * batch, esize, torch)
    var = [v for v in _variants() if v["dtype"] == dtype]

    def names(role, L, W=None):
        return [v["name"] for v in var if v["role"] == role and v["L"] == L and (W is None or v["W"] == W)]

    results = []

    def run(sched):
        r = _time_schedule(shape, batch, dtype, sched, bufs, reps)
        if r is None:
            return None
        per, info = r
        results.append((sum(per), sched, per, info["pass_variant"]))
        if verbose:
            print(f"  {sum(per):9.2f} us  {sched}  {['%.1f' % x for x in per]}", flush=True)
        return sum(per), per, info

    base = run(None)
    if base is None:
        raise capi.FFTError(capi.FFT_ERR_UNSUPPORTED_SIZE, "tune_plan")
    info = base[2]
    keys = []
    starts = [{}]
    if len(shape) == 2:
        if shape[1] > 1:
            keys.append(("row", ROLE_ROW, shape[1]))
        if shape[0] > 1:
            keys.append(("col", ROLE_COL, shape[0]))
        splits = [None]
        lg_r = int(math.log2(shape[0]))
        if lg_r % 2 == 0 and lg_r >= 2 and shape[1] >= 2 and run("col3=1") is not None:
            # columns as two sub-passes of sqrt(rows) points, tuned separately
            sq = 1 << (lg_r // 2)
            keys3 = [("colt", ROLE_COL_TW, sq), ("col", ROLE_COL, sq), ("row", ROLE_ROW, shape[1])]
            starts = [{"col3": 0}, ({"col3": 1}, keys3)]
        for r in (4, 2):
            # rows fused with the first radix-r step of the columns, then
            # columns of R/r points
            if shape[0] >= 2 * r and run(f"rowcol={r}") is not None:
                keysf = [("row", ROLE_ROWCOL, shape[1]), ("col", ROLE_COL, shape[0] // r)]
                starts.append(({"rowcol": r}, keysf))
    elif info["passes"] == 1 and shape[0] > 1:
        keys.append(("single", ROLE_ROW, shape[0]))
        splits = [None]
    elif info["passes"] == 2:
        lg = int(math.log2(shape[0]))
        splits = [1 << a for a in range(6, 13) if 6 <= lg - a <= 12]
    elif info["passes"] == 3 and len(shape) == 1:
        # N1 x N2 x N3: first-pass lengths 2^8..2^12, second-pass 2^5..2^7
        lg = int(math.log2(shape[0]))
        splits = [(1 << a, 1 << b) for a in range(8, 13) for b in range(5, 8) if 1 <= lg - a - b <= 14]
    else:
        return "", base[1]

    def sched_of(d):
        return ";".join(f"{k}={v}" for k, v in d.items())

    def xcd_search(cur):
        # per-pass XCD remap: every mask over the plan's passes
        base = run(sched_of(cur))
        if base is None:
            return cur
        npass = base[2]["passes"]
        best = (base[0], cur.get("xcd"))
        for m in range(1 << npass):
            mask = "".join("1" if (m >> i) & 1 else "0" for i in range(npass))
            trial = dict(cur)
            trial["xcd"] = mask
            r = run(sched_of(trial))
            if r is not None and r[0] < best[0]:
                best = (r[0], mask)
        out = dict(cur)
        if best[1] is not None:
            out["xcd"] = best[1]
        return out

    def descend(prefix, keys, start):
        cur = xcd_search(dict(start))
        for _ in range(2):
            for key, role, L in keys:
                best = None
                # a fused row pass must match the plan's column radix
                for nm in names(role, L, cur.get("rowcol") if role == ROLE_ROWCOL else None):
                    trial = dict(cur)
                    trial[key] = nm
                    s = ";".join(f"{k}={v}" for k, v in trial.items())
                    r = run(s)
                    if r is not None and (best is None or r[0] < best[0]):
                        best = (r[0], nm)
                if best is not None:
                    cur[key] = best[1]
        return xcd_search(cur)

    if splits == [None]:
        for st in starts:
            if isinstance(st, tuple):
                descend("", st[1], st[0])
            else:
                descend("", keys, st)
    elif isinstance(splits[0], tuple):
        ranked = []
        for sp, sp2 in splits:
            r = run(f"split={sp};split2={sp2}")
            if r is not None:
                ranked.append((r[0], sp, sp2))
        ranked.sort()
        for _, sp, sp2 in ranked[:2]:
            n3 = shape[0] // (sp * sp2)
            descend("", [("a", ROLE_A, sp), ("colt", ROLE_COL_TW, sp2), ("b", ROLE_COL, n3)],
                    {"split": sp, "split2": sp2})
    else:
        # rank splits by their default variants, then refine the two best
        ranked = []
        for sp in splits:
            r = run(f"split={sp}")
            if r is not None:
                ranked.append((r[0], sp))
        ranked.sort()
        for _, sp in ranked[:2]:
            N1, N2 = sp, shape[0] // sp
            descend("", [("a", ROLE_A, N1), ("b", ROLE_COL, N2)], {"split": sp})
    best = min(results, key=lambda r: r[0])
    return best[1] or "", best[2]


def tune_many(sizes, dtype=capi.FFT_C64, reps=10, verbose=False):
    """Tune a batched-uneven plan; returns (schedule string, microseconds)."""
    import torch
    total = int(sum(int(s) for s in sizes))
    esize = 8 if dtype == capi.FFT_C64 else 4
    bufs = _Buffers(total, esize, torch)

    def timed(s):
        try:
            h = capi.fft_plan_many_ex(list(sizes), dtype, capi.FFT_FORWARD, s)
        except capi.FFTError:
            return None
        try:
            per, _ = _time_handle(h, bufs, reps)
        finally:
            capi.fft_destroy(h)
        if verbose:
            print(f"  {per[0]:9.2f} us  {s}", flush=True)
        return per[0]

    grid = []
    for P in (8, 16):
        for threads in (256, 512):
            for pipe in (0, 1):
                # the pipelined kernel keeps tiles up to 2^12 (512 lanes) or 2^11
                max_tile = min(12 if (not pipe or threads == 512) else 11, int(math.log2(threads * P)))
                for pass2 in range(max(8, max_tile - 3), max_tile + 2):
                    for order in ("bigfirst", "given"):
                        grid.append(f"p={P};threads={threads};pass2={pass2};order={order}"
                                    + (";pipe=1" if pipe else ";pipe=0"))
    # the two-launch kernel (512 lanes, tiles up to 2^12)
    for pass2 in range(9, 14):
        grid.append(f"p=16;threads=512;pipe=2;pass2={pass2}")
    best = None
    for s in grid:
        us = timed(s)
        if us is not None and (best is None or us < best[0]):
            best = (us, s)
    if best is not None and "pipe=2" not in best[1]:
        # queue order: second passes lagging the first passes by k transforms
        base = best[1]
        for lag in (1, 2, 4, 8):
            us = timed(f"{base};lag={lag}")
            if us is not None and us < best[0]:
                best = (us, f"{base};lag={lag}")
    if best is not None:
        best = _tune_per_length(sizes, best, timed)
    if best is not None and "pipe=2" in best[1]:
        # nontemporal stores for the last items of each launch
        base = best[1]
        for k in (64, 128, 256, 400):
            us = timed(f"{base};ntail={k}")
            if us is not None and us < best[0] * 0.995:
                best = (us, f"{base};ntail={k}")
    return best[1], [best[0]]


def _tune_per_length(sizes, best, timed):
    """Per-length choices on top of the best global schedule: for every
    length present, one pass or two (where both are possible) and, for two
    passes, the first-pass length N1 (coordinate descent, two sweeps, each
    change kept only if the whole launch gets faster)."""
    lgs = sorted({int(math.log2(int(n))) for n in sizes}, reverse=True)
    def opt(key, default):
        m = re.search(r"(?:^|;)" + key + r"=(\d+)", best[1])
        return int(m.group(1)) if m else default
    threads, P, pipe = opt("threads", 256), opt("p", 16), opt("pipe", 0)
    base = best[1]
    max_tile = min(12 if (pipe != 1 or threads == 512) else 11, int(math.log2(threads * P)))
    pass2 = opt("pass2", max_tile + 1)
    cur = dict()
    for _ in range(2):
        for lg in lgs:
            two_default = lg >= pass2 or lg > max_tile
            options = []
            if lg <= max_tile and lg >= 2:
                options.append(("pass", 1 if two_default else 2))
            for l1 in range(max(1, lg - max_tile), min(max_tile, lg - 1) + 1):
                options.append(("n1", l1))
            for key, val in options:
                trial = dict(cur)
                trial.pop(("pass", lg), None)
                trial.pop(("n1", lg), None)
                trial[(key, lg)] = val
                s = base + "".join(f";{k}.{L}={v}" for (k, L), v in sorted(trial.items()))
                us = timed(s)
                if us is not None and us < best[0] * 0.995:
                    best = (us, s)
                    cur = trial
    return best


def tune_and_store(problems, many=(), reps=10, path=None, verbose=True):
    """Tune a list of (shape, batch, dtype) and of (sizes, dtype); store."""
    entries = {}
    for shape, batch, dtype in problems:
        t0 = time.time()
        s, per = tune_plan(shape, batch, dtype, reps, verbose)
        entries[_key("plan", shape, batch, dtype)] = {"schedule": s, "us": per,
                                                      "tuned_s": round(time.time() - t0, 1)}
        if verbose:
            print(f"tuned {shape} x{batch} dtype {dtype}: {s} {per}", flush=True)
    for sizes, dtype in many:
        s, per = tune_many(sizes, dtype, reps, verbose)
        entries[_many_key(sizes, dtype)] = {"schedule": s, "us": per, "count": len(sizes)}
        if verbose:
            print(f"tuned many({len(sizes)}) dtype {dtype}: {s} {per}", flush=True)
    save(entries, path)
    return entries


def standard_problems():
    """The workloads this package is benchmarked on (1-D 2^10 and 2^20, the
    latter also in 16-bit storage, 2-D 4096^2, batched 2^16, 1-D 2^28,
    batched uneven sizes in three storage types)."""
    from . import workloads
    plans = [([1024], 1, capi.FFT_C64), ([1024], 32768, capi.FFT_C64),
             ([1 << 20], 16, capi.FFT_C64), ([4096, 4096], 1, capi.FFT_C64),
             ([1 << 16], 64, capi.FFT_C64), ([1 << 28], 1, capi.FFT_C64),
             ([1 << 20], 16, capi.FFT_C16F), ([1 << 20], 16, capi.FFT_C16BF)]
    sizes = workloads.uneven_sizes(512, 8, 16, seed=3)
    many = [(list(int(s) for s in sizes), dt) for dt in (capi.FFT_C64, capi.FFT_C16F, capi.FFT_C16BF)]
    return plans, many


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the standard workloads and write the cache")
    ap.add_argument("--out", default=CACHE_PATH)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--only", choices=["plans", "many", "all"], default="all")
    ap.add_argument("--match", default=None,
                    help="tune only the problems whose cache key contains this text")
    args = ap.parse_args()
    plans, many = standard_problems()
    if args.match:
        plans = [p for p in plans if args.match in _key("plan", p[0], p[1], p[2])]
        many = [m for m in many if args.match in _many_key(m[0], m[1])]
    if args.only == "plans":
        many = []
    if args.only == "many":
        plans = []
    tune_and_store(plans, many, reps=args.reps, path=args.out)
