// Experiment: 256-point transforms (256 = 16 x 16, eq. 5) whose exchange
// between the two radix-16 stages stays inside the wavefront.
//
// Sixteen lanes (one DPP row) hold one signal, sixteen points each.  Stage 1
// is the Stockham step of the butterfly kernels with span 1: lane t holds
// points t + 16q and, after a 16-point DFT in registers, output r of it
// belongs at position 16t + r.  Stage 2 (span 16) needs in lane t the points
// t + 16q of that array, that is register t of lane q: a 16 x 16 transpose
// across the 16 lanes.  The butterfly kernels do it through LDS with a
// workgroup barrier; here it is four rounds of pairwise swaps between lanes
// t and t ^ d (d = 1, 2, 4, 8), each round moving half of a lane's sixteen
// values, with no LDS memory and no barrier.  Then the twiddles W_256^{t r},
// a second 16-point DFT, and the outputs t + 16r are in natural order.
// Kept beside the LDS exchange to compare the two in rocprof.
#include "xlane.hpp"

#include "fft_device.hpp"

namespace mfft {

namespace {

// Value of lane t ^ D for every lane.
//   mode 0: DPP quad permutes (D = 1, 2), ds_swizzle in bit-mask mode (D = 4)
//           and a DPP rotate of the 16-lane row by 8 (D = 8);
//   mode 1: ds_bpermute (a gather through the LDS crossbar, no LDS memory).
template <int D, int MODE>
__device__ __forceinline__ float xor_lane(float x, int lane) {
  if constexpr (MODE == 1) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ D) << 2, __float_as_int(x)));
  } else if constexpr (D == 1) {
    // quad_perm (1, 0, 3, 2)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
  } else if constexpr (D == 2) {
    // quad_perm (2, 3, 0, 1)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
  } else if constexpr (D == 4) {
    // bit-mask swizzle over 32 lanes: and 0x1f, or 0, xor 4
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x1F | (4 << 10)));
  } else {
    static_assert(D == 8, "xor distances 1, 2, 4, 8");
    // row_ror:8 -- within a row of 16 lanes, lane t reads lane (t + 8) mod 16 = t ^ 8
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
  }
}

// One round of the transpose: for each register pair (i, i | D) the lane
// whose bit D is clear keeps v[i] and replaces v[i | D] by its partner's
// v[i]; the partner keeps v[i | D] and replaces v[i] by this lane's v[i | D].
// Each lane sends and receives through the same register.
template <int D, int MODE>
__device__ __forceinline__ void swap_round(float2* v, int t, int lane) {
  const bool hi = (t & D) != 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i & D) continue;
    const int j = i | D;
    // selects on values, not on which register is written: a conditional
    // store to v[hi ? i : j] would index the array at run time
    const float2 vi = v[i], vj = v[j];
    const float2 s = hi ? vi : vj;
    const float2 r = make_float2(xor_lane<D, MODE>(s.x, lane), xor_lane<D, MODE>(s.y, lane));
    v[i] = hi ? r : vi;
    v[j] = hi ? vj : r;
  }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_dft256_xlane(const float2* __restrict__ in, float2* __restrict__ out,
                                                      int64_t batch, const float2* __restrict__ w256,
                                                      float scale, int conj_in, int conj_out) {
  const int lane = threadIdx.x & 63;
  const int t = threadIdx.x & 15;
  const int64_t sig = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  // every lane of a 16-lane group takes part in the swaps: a group past the
  // end of the batch works on the last signal and does not store
  const bool ok = sig < batch;
  const int64_t s0 = ok ? sig : batch - 1;
  const float2* x = in + s0 * 256;
  const uint32_t sin_ = conj_in ? 0x80000000u : 0u;
  const uint32_t sout = conj_out ? 0x80000000u : 0u;

  float2 v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const float2 e = x[t + 16 * q];
    v[q] = make_float2(e.x, __uint_as_float(__float_as_uint(e.y) ^ sin_));
  }
  Dft<16>::run(v);  // output r of this lane belongs at 16 t + r

  swap_round<1, MODE>(v, t, lane);
  swap_round<2, MODE>(v, t, lane);
  swap_round<4, MODE>(v, t, lane);
  swap_round<8, MODE>(v, t, lane);
  // now v[q] holds point t + 16 q of the first stage's output

#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w256[(t * r) & 255]);
  Dft<16>::run(v);  // output r is X[t + 16 r]

  if (ok) {
    float2* y = out + sig * 256;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 o = cscale(v[r], scale);
      y[t + 16 * r] = make_float2(o.x, __uint_as_float(__float_as_uint(o.y) ^ sout));
    }
  }
}

}  // namespace

hipError_t launch_dft256_xlane(const void* in, void* out, int64_t batch, const float2* w256, float scale,
                               int conj_in, int conj_out, int mode, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t blocks = (batch + 15) / 16;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  if (mode == 1)
    hipLaunchKernelGGL(k_dft256_xlane<1>, dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)in,
                       (float2*)out, batch, w256, scale, conj_in, conj_out);
  else
    hipLaunchKernelGGL(k_dft256_xlane<0>, dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)in,
                       (float2*)out, batch, w256, scale, conj_in, conj_out);
  return hipGetLastError();
}

}  // namespace mfft
