"""Writes the kernel-instantiation sources (variants_*.hip).

Run by the package build before compiling; the list below is the registry of
compiled strip-pass variants: role (row = contiguous lines, a = first pass of
a 1-D split with the inter-pass twiddle, col = strided columns), sub-transform
length L, points per lane P and lines per workgroup W.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LDS_MAX = 160 * 1024
DT = {"c64": "float2", "f16": "__half2", "bf16": "c16bf"}
ROLE = {"r": "ROLE_ROW", "a": "ROLE_SPLIT_A", "c": "ROLE_COL", "t": "ROLE_COL_TW"}


def lds_bytes(L, W, ex=0):
    # the kernels' padded layout needs W * (L + L/32 + 2) slots: this is an
    # upper bound of it for L >= 16 (shorter lines, whose tiles are far below
    # the limit, need one or two slots more), kept so that the registry stays
    # the set of variants measured and tested
    return W * (L + (L >> 4) + 1) * (4 if ex else 8)


def threads(L, P, W):
    pp = min(P, L)
    return W * (L // pp)


def ok(L, P, W, ex=0, min_threads=64):
    t = threads(L, P, W)
    return t <= 1024 and t >= min(min_threads, 1024) and lds_bytes(L, W, ex) <= LDS_MAX


def row_set():
    out = []
    for lg in range(1, 15):
        L = 1 << lg
        for P in (8, 16, 32):
            if P > L and P != 8:
                continue
            if P == 32 and (L < 512 or L > 1024):
                continue
            pp = min(P, L)
            T = L // pp
            for target in (256, 512):
                W = max(1, target // T)
                for ex in (0, 1):
                    if ex and lds_bytes(L, W) <= 64 * 1024:
                        continue
                    if ok(L, P, W, ex) and (L, P, W, ex) not in out:
                        out.append((L, P, W, ex))
    return out


def strided_set(lo_lg, hi_lg, role):
    out = []
    for lg in range(lo_lg, hi_lg + 1):
        L = 1 << lg
        for P in (8, 16, 32):
            if P > L and P != 8:
                continue
            # 32 points per lane: up to 1024 points, and for the long 2-D
            # column passes (2048, 4096) with 8-16 columns per tile
            if P == 32 and (L < 256 or L > (4096 if role == "c" else 1024)):
                continue
            for W in (1, 2, 4, 8, 16, 32, 64):
                if P == 32 and L > 1024 and W > 16:
                    continue
                if role == "a" and W < 4:
                    continue
                if P == 32 and W < 8:
                    continue
                for ex in (0, 1):
                    if ex and lds_bytes(L, W) <= 64 * 1024:
                        continue
                    if ok(L, P, W, ex, min_threads=64 if L >= 64 else 1):
                        out.append((L, P, W, ex))
    return out


def a_set():
    return strided_set(6, 12, "a")


def col_set():
    return strided_set(1, 14, "c")


def coltw_set():
    """Columns with a twiddle (first column sub-pass of the three-pass 2-D
    plan): lengths 2..128, wide strips."""
    out = []
    for lg in range(1, 8):
        L = 1 << lg
        for P in (8, 16):
            if P > L and P != 8:
                continue
            for W in (8, 16, 32, 64):
                if ok(L, P, W, 0, min_threads=64 if L >= 64 else 1):
                    out.append((L, P, W, 0))
    return out


def c16_set():
    # one variant per (role, L) for the 16-bit storage types
    out = []
    for lg in range(1, 15):
        L = 1 << lg
        P = 16
        T = L // min(P, L)
        W = max(1, 256 // T)
        while not ok(L, P, W) and W > 1:
            W //= 2
        out.append(("r", L, P, W, 0))
    for lg in range(6, 13):
        L = 1 << lg
        W = 16
        while not ok(L, 16, W) and W > 1:
            W //= 2
        out.append(("a", L, 16, W, 0))
    for lg in range(1, 15):
        L = 1 << lg
        W = 16
        while not ok(L, 16, W, min_threads=1) and W > 1:
            W //= 2
        out.append(("c", L, 16, W, 0))
    for lg in range(1, 8):
        out.append(("t", 1 << lg, 16, 16, 0))
    # three-pass 2-D: wide column tiles for the two short column passes, and
    # rows paired with their transposes (an even number of rows per tile)
    for lg in range(4, 8):
        L = 1 << lg
        for role in ("t", "c"):
            if ok(L, 16, 64):
                out.append((role, L, 16, 64, 0))
    for lg in range(11, 13):
        if ok(1 << lg, 16, 2):
            out.append(("r", 1 << lg, 16, 2, 0))
    # the split passes of 2^16 and 2^20 with the next tile prefetched (a
    # sixth entry 1: persistent; the prefetch holds 16-bit pairs, one register
    # each) or 128 B row segments (32 pairs per row)
    out += [("a", 1024, 32, 16, 0, 1), ("a", 1024, 32, 16, 0, 2), ("c", 1024, 32, 16, 1, 1),
            ("a", 256, 16, 32, 0, 1), ("c", 256, 16, 32, 0, 1), ("c", 256, 16, 32, 0)]
    return list(dict.fromkeys(out))


def rowcol_set():
    """2-D row passes fused with a radix-4 column step (k_rowcol): row
    lengths 256 .. 4096, four rows per tile; the two-round exchange where
    the one-round one would not fit in LDS beside the stage table."""
    out = []
    for lg in range(8, 13):
        L = 1 << lg
        P = 16 if L <= 512 else 32
        ex = 1 if L >= 4096 else 0
        out.append((L, P, 4, ex))
    # 4096-point rows: 1024 lanes of 16 points (more waves per CU), and a
    # radix-2 column step (two rows per tile: half the LDS)
    out += [(4096, 16, 4, 1), (4096, 32, 2, 1), (2048, 32, 2, 0)]
    return [v + (1,) for v in out] + SPLIT_TW_ROWCOL


# fused row passes whose stage twiddles come from two factor tables of W_L
# (TWP 2): the LDS then holds a one-round exchange of four (or two) 4096-point
# rows; two rows of 16 points per lane take 128 registers and 69 KB of LDS,
# so two workgroups share a CU
SPLIT_TW_ROWCOL = [(4096, 16, 4, 0, 2), (4096, 32, 4, 0, 2), (4096, 16, 2, 0, 2), (4096, 32, 2, 0, 2)]


def name(role, L, P, W, ex, dt, persist=0):
    # q: persistent with the next tile in flight; q2: the next two tiles
    q = {0: "", 1: "q", 2: "q2"}[persist]
    return f"{role}{L}p{min(P, L)}w{W}{q}{'x' if ex else ''}_{dt}"


def pipe_lds_bytes(L, P, W, ex, twid):
    pp = min(P, L)
    xn = W * (L + (L >> 4) + 1) if ex == 0 else (W * (L + (L >> 4) + 1) + 1) // 2
    # padded stage tables: rows of R + 2 for every stage after the first
    lg, lp = L.bit_length() - 1, pp.bit_length() - 1
    S = (lg + lp - 1) // lp if lg > lp else 1
    first = L >> ((S - 1) * lp)
    tw, ns = 0, first
    for _ in range(1, S):
        tw += ns * ((pp + 2) if pp >= 4 else pp)
        ns *= pp
    return 8 * (xn + max(tw, 1) + (W * pp if twid else 0))


def pipe_set():
    """Persistent pipelined variants: one workgroup of 256..1024 lanes per CU."""
    out = []
    for role in ("a", "c", "r"):
        for lg in range(8, 13):
            L = 1 << lg
            for P in (16, 32):
                if P == 32 and L > 1024 and role != "c":
                    continue
                for W in ((1, 2, 4) if role == "r" else (8, 16, 32)):
                    for ex in (0, 1):
                        # 1024 lanes leave 128 registers per lane: too few for
                        # a tile in flight plus the next one (they spill)
                        t = threads(L, P, W)
                        if t < 256 or t > 512:
                            continue
                        # the first pass's step rows: at most two entries per lane
                        if role == "a" and W * min(P, L) > 2 * t:
                            continue
                        if pipe_lds_bytes(L, P, W, ex, role == "a") > LDS_MAX:
                            continue
                        if ex and pipe_lds_bytes(L, P, W, 0, role == "a") <= LDS_MAX:
                            continue
                        out.append((role, L, P, W, ex))
    return out


# check mode: emit() records the files whose committed text differs from what
# the registry generates instead of writing them
_CHECK = None


def emit(fname, func, items):
    lines = ['#include "variants.hpp"', "", "namespace mfft {", "",
             f"void {func}(void (*add)(const Variant&)) {{"]
    for it in items:
        role, L, P, W, ex, dt = it[:6]
        persist = it[6] if len(it) > 6 else 0
        lines.append(f'  add(make_variant<{ROLE[role]}, {L}, {P}, {W}, {ex}, {DT[dt]}, {persist}>'
                     f'("{name(role, L, P, W, ex, dt, persist)}"));')
    lines += ["}", "", "}  // namespace mfft", ""]
    emit_text(fname, "\n".join(lines))


def emit_text(fname, text):
    path = os.path.join(HERE, fname)
    if not os.path.exists(path) or open(path).read() != text:
        if _CHECK is not None:
            _CHECK.append(fname)
            return
        with open(path, "w") as f:
            f.write(text)


def check():
    """Names of the committed variants_*.hip files that differ from what the
    registry below generates (empty when they match); writes nothing."""
    global _CHECK
    _CHECK = []
    try:
        main()
        return list(_CHECK)
    finally:
        _CHECK = None


def main():
    emit("variants_c64_row.hip", "add_variants_c64_row", [("r",) + v + ("c64",) for v in row_set()])
    emit("variants_c64_a.hip", "add_variants_c64_a", [("a",) + v + ("c64",) for v in a_set()])
    cols = [("c",) + v + ("c64",) for v in col_set()]
    half = len(cols) // 2
    emit("variants_c64_col.hip", "add_variants_c64_col", cols[:half])
    emit("variants_c64_col2.hip", "add_variants_c64_col2", cols[half:])
    items = []
    for dt in ("f16", "bf16"):
        items += [v[:5] + (dt,) + v[5:] for v in c16_set()]
    emit("variants_c16.hip", "add_variants_c16", items)
    # the first passes also with two tiles in flight
    pipe = [v + ("c64", 1) for v in pipe_set()]
    pipe += [v + ("c64", 2) for v in pipe_set() if v[0] == "a"]
    emit("variants_c64_pipe.hip", "add_variants_c64_pipe",
         pipe + [("t",) + v + ("c64",) for v in coltw_set()])
    lines = ['#include "variants.hpp"', "", "namespace mfft {", "",
             "void add_variants_c64_rowcol(void (*add)(const Variant&)) {"]
    for L, P, W, ex, twp in rowcol_set():
        lines.append(f'  add(make_rowcol_variant<{L}, {P}, {W}, {ex}, {twp}, float2>'
                     f'("{name("f", L, P, W, ex, "c64", 1)}"));')
    lines += ["}", "", "}  // namespace mfft", ""]
    emit_text("variants_c64_rowcol.hip", "\n".join(lines))


if __name__ == "__main__":
    main()
