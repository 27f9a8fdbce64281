"""ctypes binding of libmi355fft.so under the C names of include/mi355fft.h.

Argument marshalling only: every function here forwards to the library and
turns a negative status into ``FFTError``.  Device pointers and streams are
plain integers (``tensor.data_ptr()``, ``torch.cuda.Stream.cuda_stream``).

The library links against the HIP runtime by its soname; ``torch`` is
imported first so that the runtime torch already loaded is the one the
library binds to (one HIP runtime per process, shared streams and memory).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355fft.so")

FFT_C64, FFT_C16F, FFT_C16BF = 0, 1, 2
FFT_FORWARD, FFT_INVERSE = -1, 1
FFT_OK = 0
FFT_ERR_INVALID_ARGUMENT = -1
FFT_ERR_UNSUPPORTED_SIZE = -2
FFT_ERR_ALIGNMENT = -3
FFT_ERR_INPLACE = -4
FFT_ERR_HIP = -5
FFT_ERR_NO_MEMORY = -6
FFT_ERR_WATCHDOG = -7
FFT_ERR_SCRATCH_LIMIT = -8

EXPORTED = (
    "fft_plan", "fft_plan_ex", "fft_plan_many", "fft_plan_many_ex", "fft_many_watchdog",
    "fft_many_set_wait_limit", "fft_exec", "fft_exec_static", "fft_set_scale", "fft_workspace_size",
    "fft_set_workspace", "fft_plan_info", "fft_destroy", "fft_error_string",
    "fft_last_hip_error", "fft_variant_count", "fft_variant_name", "fft_variant_describe",
    "fft_describe", "fft_profile_enable", "fft_profile_sample", "fft_profile_collect", "fft_profile_read",
    "fft_twiddle_host", "fft_describe_many", "fft_pipe_create", "fft_pipe_exec", "fft_pipe_wait",
    "fft_pipe_destroy", "fft_describe_many_launches",
)


class fft_plan_info_t(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64 * 2),
        ("batch", ctypes.c_int64),
        ("dims", ctypes.c_int),
        ("dtype", ctypes.c_int),
        ("direction", ctypes.c_int),
        ("passes", ctypes.c_int),
        ("split", ctypes.c_int64 * 2),
        ("pass_variant", (ctypes.c_char * 32) * 4),
        ("points", ctypes.c_int64),
        ("flops", ctypes.c_double),
        ("bytes_min", ctypes.c_double),
        ("bytes_pass", ctypes.c_double * 4),
        ("gpu_twiddles", ctypes.c_int),
    ]


class FFTError(RuntimeError):
    def __init__(self, status: int, what: str, hip: int = 0):
        self.status = status
        self.hip = hip
        msg = f"{what}: {error_string(status)} (status {status}"
        msg += f", hipError {hip})" if status == FFT_ERR_HIP else ")"
        super().__init__(msg)


_lib = None


def library_path() -> str:
    return LIB_PATH


def load():
    """Load the library (after torch), declaring every prototype."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "fft_plan": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, pp], ctypes.c_int),
        "fft_plan_ex": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                         ctypes.c_char_p, pp], ctypes.c_int),
        "fft_plan_many": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, pp], ctypes.c_int),
        "fft_plan_many_ex": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, pp],
                             ctypes.c_int),
        "fft_many_watchdog": ([vp, ctypes.c_int], ctypes.c_int),
        "fft_many_set_wait_limit": ([vp, ctypes.c_int64], ctypes.c_int),
        "fft_exec": ([vp, vp, vp, vp], ctypes.c_int),
        "fft_exec_static": ([vp, vp, vp, vp], ctypes.c_int),
        "fft_set_scale": ([vp, ctypes.c_double], ctypes.c_int),
        "fft_workspace_size": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "fft_set_workspace": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "fft_plan_info": ([vp, ctypes.POINTER(fft_plan_info_t)], ctypes.c_int),
        "fft_destroy": ([vp], ctypes.c_int),
        "fft_error_string": ([ctypes.c_int], ctypes.c_char_p),
        "fft_last_hip_error": ([], ctypes.c_int),
        "fft_variant_count": ([], ctypes.c_int),
        "fft_variant_name": ([ctypes.c_int], ctypes.c_char_p),
        "fft_variant_describe": ([ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 6, ctypes.c_int),
        "fft_describe": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER((ctypes.c_char * 32) * 4),
                          i64p], ctypes.c_int),
        "fft_profile_enable": ([vp, ctypes.c_int], ctypes.c_int),
        "fft_profile_sample": ([vp, ctypes.c_int], ctypes.c_int),
        "fft_profile_collect": ([vp], ctypes.c_int),
        "fft_profile_read": ([vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), i64p], ctypes.c_int),
        "fft_describe_many": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_char_p,
                               ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, i64p,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                              ctypes.c_int),
        "fft_describe_many_launches": ([i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_char_p,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, i64p], ctypes.c_int),
        "fft_twiddle_host": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                              ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "fft_pipe_create": ([vp, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "fft_pipe_exec": ([vp, vp, vp, ctypes.c_int64], ctypes.c_int),
        "fft_pipe_wait": ([vp], ctypes.c_int),
        "fft_pipe_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != FFT_OK:
        raise FFTError(rc, what, load().fft_last_hip_error() if rc == FFT_ERR_HIP else 0)


def _i64(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(1, len(vals)))(*vals)


def _sched(s):
    return None if s is None else s.encode()


def error_string(status: int) -> str:
    return load().fft_error_string(int(status)).decode()


def fft_plan(n, batch, dims, dtype, direction) -> int:
    h = ctypes.c_void_p()
    _check(load().fft_plan(_i64(n), int(batch), int(dims), int(dtype), int(direction),
                           ctypes.byref(h)), "fft_plan")
    return h.value


def fft_plan_ex(n, batch, dims, dtype, direction, schedule) -> int:
    h = ctypes.c_void_p()
    _check(load().fft_plan_ex(_i64(n), int(batch), int(dims), int(dtype), int(direction),
                              _sched(schedule), ctypes.byref(h)), "fft_plan_ex")
    return h.value


def fft_plan_many(sizes, dtype, direction) -> int:
    h = ctypes.c_void_p()
    _check(load().fft_plan_many(_i64(sizes), len(sizes), int(dtype), int(direction),
                                ctypes.byref(h)), "fft_plan_many")
    return h.value


def fft_plan_many_ex(sizes, dtype, direction, schedule) -> int:
    h = ctypes.c_void_p()
    _check(load().fft_plan_many_ex(_i64(sizes), len(sizes), int(dtype), int(direction),
                                   _sched(schedule), ctypes.byref(h)), "fft_plan_many_ex")
    return h.value


def fft_many_watchdog(plan: int, clear: bool = True) -> int:
    rc = load().fft_many_watchdog(plan, 1 if clear else 0)
    if rc not in (FFT_OK, FFT_ERR_WATCHDOG):
        _check(rc, "fft_many_watchdog")
    return rc


def fft_many_set_wait_limit(plan: int, microseconds: int) -> None:
    _check(load().fft_many_set_wait_limit(plan, int(microseconds)), "fft_many_set_wait_limit")


def fft_exec(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _check(load().fft_exec(plan, in_ptr, out_ptr, stream), "fft_exec")


def fft_exec_status(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> int:
    """fft_exec returning the raw status (for tests of the error codes)."""
    return load().fft_exec(plan, in_ptr, out_ptr, stream)


def fft_exec_static(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
    _check(load().fft_exec_static(plan, in_ptr, out_ptr, stream), "fft_exec_static")


def fft_exec_static_status(plan: int, in_ptr: int, out_ptr: int, stream: int = 0) -> int:
    """fft_exec_static returning the raw status (for tests of the error codes)."""
    return load().fft_exec_static(plan, in_ptr, out_ptr, stream)


def fft_set_scale(plan: int, scale: float) -> None:
    _check(load().fft_set_scale(plan, float(scale)), "fft_set_scale")


def fft_workspace_size(plan: int) -> int:
    b = ctypes.c_size_t()
    _check(load().fft_workspace_size(plan, ctypes.byref(b)), "fft_workspace_size")
    return b.value


def fft_set_workspace(plan: int, ptr: int, nbytes: int) -> None:
    _check(load().fft_set_workspace(plan, ptr, int(nbytes)), "fft_set_workspace")


def fft_plan_info(plan: int) -> dict:
    info = fft_plan_info_t()
    _check(load().fft_plan_info(plan, ctypes.byref(info)), "fft_plan_info")
    return {
        "n": list(info.n), "batch": info.batch, "dims": info.dims, "dtype": info.dtype,
        "direction": info.direction, "passes": info.passes, "split": list(info.split),
        "pass_variant": [bytes(v.value).decode() for v in info.pass_variant][:info.passes],
        "points": info.points, "flops": info.flops, "bytes_min": info.bytes_min,
        "bytes_pass": list(info.bytes_pass)[:info.passes], "gpu_twiddles": info.gpu_twiddles,
    }


def fft_pipe_create(plan: int, slots: int = 3) -> int:
    h = ctypes.c_void_p()
    _check(load().fft_pipe_create(plan, int(slots), ctypes.byref(h)), "fft_pipe_create")
    return h.value


def fft_pipe_exec(pipe: int, host_in: int, host_out: int, chunks: int) -> None:
    _check(load().fft_pipe_exec(pipe, host_in, host_out, int(chunks)), "fft_pipe_exec")


def fft_pipe_wait(pipe: int) -> None:
    _check(load().fft_pipe_wait(pipe), "fft_pipe_wait")


def fft_pipe_destroy(pipe: int) -> None:
    _check(load().fft_pipe_destroy(pipe), "fft_pipe_destroy")


def fft_destroy(plan: int) -> None:
    if plan:
        load().fft_destroy(plan)


def fft_last_hip_error() -> int:
    return load().fft_last_hip_error()


def fft_variant_count() -> int:
    return load().fft_variant_count()


def fft_variant_name(i: int):
    r = load().fft_variant_name(int(i))
    return None if r is None else r.decode()


def fft_variant_describe(i: int) -> dict:
    vals = [ctypes.c_int() for _ in range(6)]
    _check(load().fft_variant_describe(int(i), *[ctypes.byref(v) for v in vals]),
           "fft_variant_describe")
    keys = ("L", "P", "W", "threads", "role", "dtype")
    return {k: v.value for k, v in zip(keys, vals)}


def fft_describe(n, batch, dims, dtype, schedule=None) -> dict:
    passes = ctypes.c_int()
    names = ((ctypes.c_char * 32) * 4)()
    split = _i64([0, 0])
    _check(load().fft_describe(_i64(n), int(batch), int(dims), int(dtype), _sched(schedule),
                               ctypes.byref(passes), ctypes.byref(names), split), "fft_describe")
    return {"passes": passes.value,
            "names": [bytes(v.value).decode() for v in names][:passes.value],
            "split": [split[0], split[1]]}


def fft_profile_enable(plan: int, slots: int = 1) -> None:
    """Time the next `slots` execs per launch with HIP events (0: off)."""
    _check(load().fft_profile_enable(plan, int(slots)), "fft_profile_enable")


def fft_profile_sample(plan: int, every: int) -> None:
    """Time one exec in `every` (events recorded on those execs only)."""
    _check(load().fft_profile_sample(plan, int(every)), "fft_profile_sample")


def fft_profile_collect(plan: int) -> None:
    _check(load().fft_profile_collect(plan), "fft_profile_collect")


def fft_profile_read(plan: int, pass_index: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().fft_profile_read(plan, int(pass_index), ctypes.byref(ms), ctypes.byref(n)),
           "fft_profile_read")
    return ms.value, n.value


def fft_twiddle_host(count: int, R: int, M: int, mul: int = 1):
    """Host twiddle table entries W_M^{e(i)} as a complex64 numpy array."""
    import numpy as np
    out = np.empty(2 * int(count), dtype=np.float32)
    _check(load().fft_twiddle_host(int(count), int(R), int(M), int(mul),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
           "fft_twiddle_host")
    return out[0::2] + 1j * out[1::2].astype(np.complex64)


def fft_describe_many(sizes, dtype=FFT_C64, schedule=None):
    """Host-only work queue of a batched plan: (items [n, 4], first_len, first_tiles)."""
    import numpy as np
    lib = load()
    sz = _i64(sizes)
    n = ctypes.c_int64()
    _check(lib.fft_describe_many(sz, len(sizes), int(dtype), _sched(schedule), None, 0,
                                 ctypes.byref(n), None, None), "fft_describe_many")
    items = np.zeros((n.value, 4), dtype=np.int32)
    fl = np.zeros(len(sizes), dtype=np.int32)
    ft = np.zeros(len(sizes), dtype=np.int32)
    p32 = ctypes.POINTER(ctypes.c_int32)
    _check(lib.fft_describe_many(sz, len(sizes), int(dtype), _sched(schedule),
                                 items.ctypes.data_as(p32), n.value, ctypes.byref(n),
                                 fl.ctypes.data_as(p32), ft.ctypes.data_as(p32)), "fft_describe_many")
    return items, fl, ft


def fft_describe_many_launches(sizes, dtype=FFT_C64, schedule=None):
    """Host-only launch offsets into a batched plan's item list (n + 1 entries)."""
    import numpy as np
    lib = load()
    sz = _i64(sizes)
    n = ctypes.c_int64()
    _check(lib.fft_describe_many_launches(sz, len(sizes), int(dtype), _sched(schedule), None, 0,
                                        ctypes.byref(n)), "fft_describe_many_launches")
    q = np.zeros(n.value + 1, dtype=np.int32)
    _check(lib.fft_describe_many_launches(sz, len(sizes), int(dtype), _sched(schedule),
                                        q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n.value + 1,
                                        ctypes.byref(n)), "fft_describe_many_launches")
    return q
