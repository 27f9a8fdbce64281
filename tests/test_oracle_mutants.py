"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of oracle.c (on the CPU), builds it, and checks that the
pin checks of test_oracle.py reject it; the unmodified source must pass."""
import cmath
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1707_07263_amd import workloads

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "twiddle_sign": ("w[2 * j + 1] = (double)sign * sin(ang);", "w[2 * j + 1] = -(double)sign * sin(ang);"),
    "no_bit_reversal": ("    if (i < r) {", "    if (0) {"),
    "butterfly_plus": ("RE(q) = ur - tr;", "RE(q) = ur + tr;"),
    "twiddle_index": ("ORACLE_TWO_PI * (double)j / (double)len", "ORACLE_TWO_PI * (double)(j + 1) / (double)len"),
    "half_angle": ("ORACLE_TWO_PI * (double)j / (double)len", "ORACLE_TWO_PI * (double)j / (double)half"),
    "cross_term_sign": ("const double ti = wr * IM(q) + wi * RE(q);", "const double ti = wr * IM(q) - wi * RE(q);"),
    "no_inverse_scale": ("return sign > 0 ? 1.0 / (double)n : 1.0;", "return 1.0;"),
    "columns_wrong_stride": ("fft1d_strided(img + 2 * c, rows, cols, sign, sc, w);",
                             "fft1d_strided(img + 2 * c, rows, rows, sign, sc, w);"),
    "packed_skips_last": ("#pragma omp for schedule(dynamic, 1)\n      for (int64_t i = 0; i < count; ++i) {\n        const double sc",
                          "#pragma omp for schedule(dynamic, 1)\n      for (int64_t i = 0; i < count - 1; ++i) {\n        const double sc"),
    "packed_first_scale": ("default_scale(sizes[i], sign)", "default_scale(sizes[0], sign)"),
    "direct_sign": ("(long double)sign * sinl(ang)", "sinl(ang)"),
    "direct_no_scale": ("      sr /= (long double)n;\n", ""),
    "sampled_outer_index": ("(unsigned __int128)(a * Sb) * (unsigned __int128)k", "(unsigned __int128)a * (unsigned __int128)k"),
    "sampled_cross_sign": ("pi += xr * tb[2 * b + 1] + xi * tb[2 * b];", "pi += xr * tb[2 * b + 1] - xi * tb[2 * b];"),
    "sampled_no_scale": ("out[2 * i] = (double)(sr * sc);", "out[2 * i] = (double)sr;"),
}


def brute(x, sign):
    n = len(x)
    return np.array([sum(complex(x[t]) * cmath.exp(sign * 2j * math.pi * ((t * k) % n) / n)
                         for t in range(n)) for k in range(n)])


def pins_pass(o) -> bool:
    """A compact run of the pins; False as soon as one fails."""
    def close(a, b, tol=1e-12):
        a, b = np.asarray(a), np.asarray(b)
        return np.linalg.norm(a - b) <= tol * max(1.0, np.linalg.norm(b))
    for n in (8, 16):
        x = workloads.normal_batch(n, 1, seed=n)[0]
        if not close(o.fft(x), brute(x, -1)):
            return False
        if not close(o.ifft(x), brute(x, +1) / n):
            return False
        if not close(o.dft_direct(x), brute(x, -1)):
            return False
        if not close(o.dft_direct(x, inverse=True), brute(x, +1) / n):
            return False
    for n in (16, 64):
        x = workloads.normal_batch(n, 1, seed=n + 1)[0]
        ks = np.arange(n)
        if not close(o.dft_at(x, ks), brute(x, -1)):
            return False
        if not close(o.dft_at(x, ks, inverse=True), brute(x, +1) / n):
            return False
    img = workloads.normal_batch(4 * 8, 1, seed=3).reshape(4, 8)
    if not close(o.fft2(img), np.fft.fft2(img)):
        return False
    sizes, packed = workloads.uneven_batch(5, 1, 5, seed=4)
    segs = np.split(packed, np.cumsum(sizes)[:-1])
    if not close(o.fft_many(packed, sizes), np.concatenate([np.fft.fft(s) for s in segs])):
        return False
    if not close(o.fft_many(packed, sizes, inverse=True), np.concatenate([np.fft.ifft(s) for s in segs])):
        return False
    return True


def build_variant(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", str(src),
                           "-o", str(lib), "-lm"])
    return oracle.Oracle(str(lib))


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmodified_source_passes(tmp_path, source):
    assert pins_pass(build_variant(tmp_path, "clean", source))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, source, name):
    old, new = MUTANTS[name]
    assert old in source, f"mutation site for {name} not found"
    assert not pins_pass(build_variant(tmp_path, name, source.replace(old, new, 1))), name
