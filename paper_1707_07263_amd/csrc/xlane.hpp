// 256-point transforms whose exchange between the two radix-16 stages moves
// values across the lanes of a wavefront instead of through LDS (the
// cross-lane experiment beside the butterfly kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfft {

// `batch` transforms of 256 complex64 points, contiguous; w256 holds
// W_256^e, e < 256; conj_in / conj_out give the inverse direction.
// mode 0: DPP row moves and ds_swizzle; mode 1: ds_bpermute.
hipError_t launch_dft256_xlane(const void* in, void* out, int64_t batch, const float2* w256, float scale,
                               int conj_in, int conj_out, int mode, hipStream_t s);

}  // namespace mfft
