// Experiment: the radix-16 sub-DFT as a small dense complex matrix product
// on the matrix cores, for batches of 256-point transforms (256 = 16 x 16,
// two such stages with the W_256 twiddle between them, eq. 5).  Kept beside
// the butterfly kernels to compare the two in rocprof.
//
// One wave transforms one signal.  v_mfma_f32_16x16x4f32 multiplies a 16x4
// block A (lane l holds A[l % 16][l / 16]) by a 4x16 block B (lane l holds
// B[l / 16][l % 16]) into a 16x16 block D (lane l holds D[4 (l / 16) + r][l % 16],
// r = 0..3).  A 16-point DFT of 16 columns X (16 x 16, complex) is
// F16 * X, with F16[i][k] = W_16^{ik}, done as four real products
// (re*re - im*im, re*im + im*re) over four k-steps of 4: 16 instructions.
//   stage 1: X[n1][n2] = x[16 n1 + n2]; lane (g, j) = (l / 16, l % 16) holds
//            X[g + 4r][j], exactly B's rows 4s + g at k-step s = r;
//            result Y1[k1][n2] in D layout, times W_256^{n2 k1};
//   stage 2: the transpose Y1^T through LDS, then F16 * Y1^T gives
//            X[k1 + 16 k2] at D position (k2, k1).
#include "mfma.hpp"

#include "fft_device.hpp"

namespace mfft {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_dft256_mfma(const float2* __restrict__ in, float2* __restrict__ out,
                                                     int64_t batch, const float2* __restrict__ w256,
                                                     float scale, int conj_in, int conj_out) {
  __shared__ float2 lds[4][16 * 17];
  const int wave = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int g = l >> 4, j = l & 15;
  const int64_t b = (int64_t)blockIdx.x * 4 + wave;
  if (b >= batch) return;  // whole waves only: no barrier below spans waves
  const float2* x = in + b * 256;
  float2* y = out + b * 256;
  const uint32_t sin_ = conj_in ? 0x80000000u : 0u;
  const uint32_t sout = conj_out ? 0x80000000u : 0u;

  // A operands: F16[j][4s + g] = W_16^{j (4s + g)} = W_256^{16 j (4s + g) mod 256}
  float fre[4], fim[4], fimn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float2 w = w256[(16 * j * (4 * s + g)) & 255];
    fre[s] = w.x;
    fim[s] = w.y;
    fimn[s] = -w.y;
  }
  // stage 1 inputs: X[g + 4r][j] = x[16 (g + 4r) + j]
  float xr[4], xi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float2 v = x[16 * (g + 4 * r) + j];
    xr[r] = v.x;
    xi[r] = __uint_as_float(__float_as_uint(v.y) ^ sin_);
  }
  v4f cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(fre[s], xr[s], cre, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(fimn[s], xi[s], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(fre[s], xi[s], cim, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(fim[s], xr[s], cim, 0, 0, 0);
  }
  // Y1[k1 = 4g + r][n2 = j] times W_256^{n2 k1}; stored transposed as
  // M[n2][k1] (row n2 padded to 17)
  float2* m = lds[wave];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k1 = 4 * g + r;
    const float2 t = w256[(j * k1) & 255];
    const float2 v = make_float2(cre[r] * t.x - cim[r] * t.y, cre[r] * t.y + cim[r] * t.x);
    m[j * 17 + k1] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  // stage 2 inputs: B[4s + g][j] = Y1^T[n2 = 4s + g][k1 = j]
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float2 v = m[(4 * s + g) * 17 + j];
    xr[s] = v.x;
    xi[s] = v.y;
  }
  cre = (v4f){0.f, 0.f, 0.f, 0.f};
  cim = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(fre[s], xr[s], cre, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(fimn[s], xi[s], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(fre[s], xi[s], cim, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(fim[s], xr[s], cim, 0, 0, 0);
  }
  // D position (k2 = 4g + r, k1 = j) -> X[k1 + 16 k2]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2 v = make_float2(cre[r] * scale, cim[r] * scale);
    v.y = __uint_as_float(__float_as_uint(v.y) ^ sout);
    y[j + 16 * (4 * g + r)] = v;
  }
}

}  // namespace

hipError_t launch_dft256_mfma(const void* in, void* out, int64_t batch, const float2* w256, float scale,
                              int conj_in, int conj_out, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t blocks = (batch + 3) / 4;
  hipLaunchKernelGGL(k_dft256_mfma, dim3((unsigned)blocks), dim3(256), 0, s, (const float2*)in, (float2*)out,
                     batch, w256, scale, conj_in, conj_out);
  return hipGetLastError();
}

}  // namespace mfft
