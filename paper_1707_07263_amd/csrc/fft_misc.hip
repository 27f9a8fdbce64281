// Small kernels: copy-scale for length-1 transforms, and FP64 twiddle-table
// generation on the GPU (used for 1-D lengths >= 2^22).
#include "twiddle.hpp"
#include "variants.hpp"

namespace mfft {

hipError_t launch_scale_copy(int dtype, const void* in, void* out, int64_t n, float scale,
                             hipStream_t s) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (n <= 0) return hipSuccess;
  switch (dtype) {
    case DT_C64:
      hipLaunchKernelGGL(k_scale_copy<float2>, dim3(blocks), dim3(256), 0, s,
                         (const float2*)in, (float2*)out, n, scale);
      break;
    case DT_C16F:
      hipLaunchKernelGGL(k_scale_copy<__half2>, dim3(blocks), dim3(256), 0, s,
                         (const __half2*)in, (__half2*)out, n, scale);
      break;
    default:
      hipLaunchKernelGGL(k_scale_copy<c16bf>, dim3(blocks), dim3(256), 0, s,
                         (const c16bf*)in, (c16bf*)out, n, scale);
      break;
  }
  return hipGetLastError();
}

// One thread per table entry: entry i of segment g is W_M^{e(i)} rounded from
// float64 to float32 (see twiddle.hpp for e(i)).
__global__ void __launch_bounds__(256) k_twiddle_fp64(float2* table, const TwSeg* segs, int nseg) {
  const int g = blockIdx.y;
  if (g >= nseg) return;
  const TwSeg sg = segs[g];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < sg.count;
       i += (int64_t)gridDim.x * 256) {
    double c, s;
    twiddle_fp64(seg_exponent(sg, i), sg.M, &c, &s);
    table[sg.off + i] = make_float2((float)c, (float)-s);
  }
}

hipError_t launch_twiddle_fp64(float2* table, const TwSeg* d_segs, int nseg, int64_t max_count,
                               hipStream_t s) {
  unsigned bx = (unsigned)((max_count + 255) / 256);
  if (bx > 4096) bx = 4096;
  if (bx == 0) bx = 1;
  hipLaunchKernelGGL(k_twiddle_fp64, dim3(bx, (unsigned)nseg), dim3(256), 0, s, table, d_segs, nseg);
  return hipGetLastError();
}

}  // namespace mfft
