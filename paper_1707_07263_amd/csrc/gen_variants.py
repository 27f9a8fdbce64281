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
ROLE = {"r": "ROLE_ROW", "a": "ROLE_SPLIT_A", "c": "ROLE_COL"}


def lds_bytes(L, W):
    return W * (L + (L >> 4) + 1) * 8


def threads(L, P, W):
    pp = min(P, L)
    return W * (L // pp)


def ok(L, P, W, min_threads=64):
    t = threads(L, P, W)
    return t <= 1024 and t >= min(min_threads, 1024) and lds_bytes(L, W) <= LDS_MAX


def row_set():
    out = []
    for lg in range(1, 15):
        L = 1 << lg
        for P in (8, 16):
            if P > L and P != 8:
                continue
            pp = min(P, L)
            T = L // pp
            for target in (256, 512):
                W = max(1, target // T)
                if ok(L, P, W) and (L, P, W) not in out:
                    out.append((L, P, W))
    return out


def a_set():
    out = []
    for lg in range(6, 13):
        L = 1 << lg
        for W in (4, 8, 16, 32):
            for P in (8, 16):
                if ok(L, P, W):
                    out.append((L, P, W))
    return out


def col_set():
    out = []
    for lg in range(1, 15):
        L = 1 << lg
        for W in (1, 2, 4, 8, 16, 32, 64):
            for P in (8, 16):
                if P > L and P != 8:
                    continue
                if ok(L, P, W, min_threads=64 if L >= 64 else 1):
                    out.append((L, P, W))
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
        out.append(("r", L, P, W))
    for lg in range(6, 13):
        L = 1 << lg
        W = 16
        while not ok(L, 16, W) and W > 1:
            W //= 2
        out.append(("a", L, 16, W))
    for lg in range(1, 15):
        L = 1 << lg
        W = 16
        while not ok(L, 16, W, min_threads=1) and W > 1:
            W //= 2
        out.append(("c", L, 16, W))
    return out


def name(role, L, P, W, dt):
    return f"{role}{L}p{min(P, L)}w{W}_{dt}"


def emit(fname, func, items):
    lines = ['#include "variants.hpp"', "", "namespace mfft {", "",
             f"void {func}(void (*add)(const Variant&)) {{"]
    for role, L, P, W, dt in items:
        lines.append(f'  add(make_variant<{ROLE[role]}, {L}, {P}, {W}, {DT[dt]}>("{name(role, L, P, W, dt)}"));')
    lines += ["}", "", "}  // namespace mfft", ""]
    text = "\n".join(lines)
    path = os.path.join(HERE, fname)
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as f:
            f.write(text)


def main():
    emit("variants_c64_row.hip", "add_variants_c64_row", [("r", L, P, W, "c64") for L, P, W in row_set()])
    emit("variants_c64_a.hip", "add_variants_c64_a", [("a", L, P, W, "c64") for L, P, W in a_set()])
    emit("variants_c64_col.hip", "add_variants_c64_col", [("c", L, P, W, "c64") for L, P, W in col_set()])
    items = []
    for dt in ("f16", "bf16"):
        items += [(r, L, P, W, dt) for r, L, P, W in c16_set()]
    emit("variants_c16.hip", "add_variants_c16", items)


if __name__ == "__main__":
    main()
