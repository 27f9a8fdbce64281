"""FP64 CPU oracle for the complex DFT (eq. 1 forward, eq. 2 inverse).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library and its Python
binding never do.  It shares no code with the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, FP64): the iterative radix-2
Cooley-Tukey method the paper describes as the serial CPU method (Sec. 2.2),
and eq. 1 / eq. 2 evaluated directly in long double for small N.  This module
only marshals numpy arrays to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


_FLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math", "-ffp-contract=off"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, no fast-math, no
    FMA contraction).  The in-tree library is built for any x86-64 host, since
    it may run on another machine than the one that built it."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + _FLAGS + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def native(directory: str) -> "Oracle":
    """The oracle compiled for the CPU it runs on (-march=native), into
    `directory`, for timing the CPU baseline on that host.  Same source,
    same FP64 arithmetic without fast-math or FMA contraction."""
    path = os.path.join(directory, "liboracle_native.so")
    subprocess.check_call(["gcc", "-march=native"] + _FLAGS + [_SRC, "-o", path, "-lm"])
    return Oracle(path)


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_fft1d.argtypes = [dp, i64, i64, ctypes.c_int, ctypes.c_double]
    lib.oracle_fft2d.argtypes = [dp, i64, i64, i64, ctypes.c_int, ctypes.c_double]
    lib.oracle_fft_many.argtypes = [dp, ctypes.POINTER(i64), i64, ctypes.c_int, ctypes.c_double]
    lib.oracle_dft_direct.argtypes = [dp, dp, i64, ctypes.c_int]
    lib.oracle_dft_at.argtypes = [dp, i64, ctypes.POINTER(i64), i64, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    for f in (lib.oracle_fft1d, lib.oracle_fft2d, lib.oracle_fft_many, lib.oracle_dft_direct,
              lib.oracle_dft_at):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _as_c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _sign(inverse: bool) -> int:
    return 1 if inverse else -1


def fft(x, inverse: bool = False, scale: float | None = None) -> np.ndarray:
    """1-D transform along the last axis (length a power of two).

    Forward: eq. 1, unscaled.  Inverse: eq. 2, times 1/N.  ``scale`` overrides
    the factor (inverse with scale=1 is the adjoint of the forward transform).
    """
    a = _as_c128(x)
    n = a.shape[-1]
    batch = a.size // n if n else 0
    _check(_load().oracle_fft1d(_ptr(a), n, batch, _sign(inverse),
                                -1.0 if scale is None else float(scale)), "fft1d")
    return a


def ifft(x) -> np.ndarray:
    return fft(x, inverse=True)


def adjoint(g) -> np.ndarray:
    """F^H g for the forward transform F: the inverse direction, unscaled."""
    return fft(g, inverse=True, scale=1.0)


def fft2(x, inverse: bool = False, scale: float | None = None) -> np.ndarray:
    """2-D transform over the last two axes: rows first, then columns."""
    a = _as_c128(x)
    r, c = a.shape[-2], a.shape[-1]
    batch = a.size // (r * c)
    _check(_load().oracle_fft2d(_ptr(a), r, c, batch, _sign(inverse),
                                -1.0 if scale is None else float(scale)), "fft2d")
    return a


def fft_many(packed, sizes, inverse: bool = False, scale: float | None = None) -> np.ndarray:
    """Independent 1-D transforms of lengths ``sizes`` packed back to back."""
    a = _as_c128(packed).reshape(-1)
    s = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    if int(s.sum()) != a.size:
        raise ValueError("sizes do not add up to the packed length")
    _check(_load().oracle_fft_many(_ptr(a), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   s.size, _sign(inverse),
                                   -1.0 if scale is None else float(scale)), "fft_many")
    return a


def dft_at(x, ks, inverse: bool = False, scale: float | None = None) -> np.ndarray:
    """Selected outputs X[ks] of one transform of x (1-D, length a power of
    two), each summed term by term in long double; O(N) per output."""
    a = _as_c128(x)
    if a.ndim != 1:
        raise ValueError("dft_at takes one transform")
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    out = np.empty(len(ks), dtype=np.complex128)
    _check(_load().oracle_dft_at(_ptr(a), a.shape[0], ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 len(ks), _sign(inverse), -1.0 if scale is None else float(scale),
                                 _ptr(out)), "dft_at")
    return out


def dft_direct(x, inverse: bool = False) -> np.ndarray:
    """Eq. 1 / eq. 2 term by term in long double (any N >= 1, O(N^2))."""
    a = _as_c128(x)
    n = a.shape[-1]
    out = np.empty_like(a)
    lib = _load()
    flat_in = a.reshape(-1, n)
    flat_out = out.reshape(-1, n)
    for i in range(flat_in.shape[0]):
        row = np.ascontiguousarray(flat_in[i])
        res = np.empty_like(row)
        _check(lib.oracle_dft_direct(_ptr(row), _ptr(res), n, _sign(inverse)), "dft_direct")
        flat_out[i] = res
    return out


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


class Oracle:
    """The same functions bound to another build of oracle.c (used by the
    tests that plant mistakes in a copy of the source and check that the
    pins catch them)."""

    def __init__(self, lib_path: str):
        self._lib = _declare(ctypes.CDLL(lib_path))

    def _swap(self, fn, *a, **k):
        global _lib
        saved = _lib
        _lib = self._lib
        try:
            return fn(*a, **k)
        finally:
            _lib = saved

    def fft(self, *a, **k):
        return self._swap(fft, *a, **k)

    def ifft(self, *a, **k):
        return self._swap(ifft, *a, **k)

    def adjoint(self, *a, **k):
        return self._swap(adjoint, *a, **k)

    def fft2(self, *a, **k):
        return self._swap(fft2, *a, **k)

    def fft_many(self, *a, **k):
        return self._swap(fft_many, *a, **k)

    def dft_direct(self, *a, **k):
        return self._swap(dft_direct, *a, **k)

    def dft_at(self, *a, **k):
        return self._swap(dft_at, *a, **k)

    def max_threads(self):
        return self._swap(max_threads)

    def set_threads(self, n):
        return self._swap(set_threads, n)
