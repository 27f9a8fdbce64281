"""MI355X-native complex FFT (arxiv 1707.07263, "A GPU Based Memory Optimized
Parallel Method For FFT Implementation"), rebuilt for gfx950.

* ``capi``      - the C ABI of include/mi355fft.h (libmi355fft.so) via ctypes.
* ``api``       - torch-facing helpers: fft, ifft, fft2, fft_many, FFTFunction.
* ``workloads`` - seeded synthetic inputs shaped like the paper's workloads.
* ``autotune``  - schedule search over the compiled kernel variants.

The transforms run only in the library's HIP kernels; there is no CPU path.
"""
from . import capi, workloads  # noqa: F401

__all__ = ["capi", "workloads", "fft", "ifft", "fft2", "ifft2", "fft_many", "FFTFunction",
           "fft_autograd", "get_plan", "get_many_plan"]


def __getattr__(name):
    # torch-facing helpers load lazily so that importing the package (for the
    # input generators, say) does not touch the GPU library
    import importlib
    if name in ("api", "autotune"):
        return importlib.import_module(f"{__name__}.{name}")
    if name in ("fft", "ifft", "fft2", "ifft2", "fft_many", "FFTFunction", "fft_autograd",
                "get_plan", "get_many_plan", "clear_cache", "variants"):
        return getattr(importlib.import_module(f"{__name__}.api"), name)
    raise AttributeError(name)
