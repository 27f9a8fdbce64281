// 256-point transforms with the radix-16 stages as matrix-core products
// (the matrix-core experiment beside the butterfly kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfft {

// `batch` transforms of 256 complex64 points, contiguous; w256 holds
// W_256^e, e < 256; conj_in / conj_out give the inverse direction.
hipError_t launch_dft256_mfma(const void* in, void* out, int64_t batch, const float2* w256, float scale,
                              int conj_in, int conj_out, hipStream_t s);

}  // namespace mfft
