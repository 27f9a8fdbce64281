// The method the paper improves on (Sec. 2.2, Fig. 2): every butterfly level
// of the transform is its own kernel launch, reading all points from global
// memory and writing them back, so an N-point transform moves the data
// log2(N) times.  Kept as an ablation beside the LDS-resident passes.
//
// Each launch is one radix-2 level in self-sorting (Stockham) order, so no
// bit-reversal pass is needed and the output is in natural order: at level s
// (span Ns = 2^s) butterfly j of a transform combines x[j] and
// x[j + N/2] * W_{2Ns}^{j mod Ns} and writes the pair to positions
// 2j - (j mod Ns) and that plus Ns.  The levels ping-pong between the output
// and a plan-owned buffer; the twiddles W_N^m, m < N/2, come from one table.
#include "levels.hpp"

#include <algorithm>

#include "fft_device.hpp"

namespace mfft {

namespace {

template <typename TS>
__global__ void __launch_bounds__(256) k_level(const TS* __restrict__ in, TS* __restrict__ out,
                                               int lgN, int s, int64_t total, const float2* tw,
                                               float scale, int conj_in, int conj_out) {
  const int64_t half = (int64_t)1 << (lgN - 1);
  const int64_t ns = (int64_t)1 << s;
  const int tw_sh = lgN - 1 - s;  // W_{2Ns}^k = W_N^{k * N / (2 Ns)}
  const uint32_t sin_ = conj_in ? 0x80000000u : 0u;
  const uint32_t sout = conj_out ? 0x80000000u : 0u;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx >> (lgN - 1);
    const int64_t j = idx & (half - 1);
    const int64_t k = j & (ns - 1);
    const TS* x = in + (b << lgN);
    TS* y = out + (b << lgN);
    float2 a = load_c(x + j);
    float2 c = load_c(x + j + half);
    a.y = __uint_as_float(__float_as_uint(a.y) ^ sin_);
    c.y = __uint_as_float(__float_as_uint(c.y) ^ sin_);
    c = cmul(c, tw[k << tw_sh]);
    float2 u = cscale(make_float2(a.x + c.x, a.y + c.y), scale);
    float2 v = cscale(make_float2(a.x - c.x, a.y - c.y), scale);
    u.y = __uint_as_float(__float_as_uint(u.y) ^ sout);
    v.y = __uint_as_float(__float_as_uint(v.y) ^ sout);
    const int64_t d = 2 * j - k;
    store_c(y + d, u);
    store_c(y + d + ns, v);
  }
}

template <typename TS>
hipError_t launch_level(const void* in, void* out, int lgN, int s, int64_t total, const float2* tw,
                        float scale, int conj_in, int conj_out, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_level<TS>, dim3(grid), dim3(256), 0, st, (const TS*)in, (TS*)out, lgN, s,
                     total, tw, scale, conj_in, conj_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_levels(const LevelsArgs& a, hipStream_t st) {
  const int L = a.lgN;
  const int64_t total = a.batch << (L - 1);  // butterflies per level
  const int64_t want = (total + 255) / 256;
  const int grid = (int)std::min<int64_t>(want, (int64_t)a.cus * 16);
  const size_t bytes = (size_t)(a.batch << L) * (size_t)(a.dtype == 0 ? 8 : 4);
  // level k writes `out` when the remaining levels after it are even in
  // number; in place, level 0 must not write the array it reads, so the
  // parity starts on the buffer and a final copy lands the result
  const bool same = a.in == a.out;
  const void* src = a.in;
  void* last = nullptr;
  for (int k = 0; k < L; ++k) {
    void* dst = same ? ((k & 1) ? a.out : a.buf) : (((L - 1 - k) & 1) ? a.buf : a.out);
    const bool first = k == 0, final_level = k == L - 1;
    float scale = a.user_scale ? (final_level ? a.scale : 1.0f) : (a.inverse ? 0.5f : 1.0f);
    const int ci = (a.inverse && first) ? 1 : 0;
    const int co = (a.inverse && final_level) ? 1 : 0;
    hipError_t e;
    switch (a.dtype) {
      case 0: e = launch_level<float2>(src, dst, L, k, total, a.tw, scale, ci, co, grid, st); break;
      case 1: e = launch_level<__half2>(src, dst, L, k, total, a.tw, scale, ci, co, grid, st); break;
      default: e = launch_level<c16bf>(src, dst, L, k, total, a.tw, scale, ci, co, grid, st); break;
    }
    if (e != hipSuccess) return e;
    src = dst;
    last = dst;
  }
  if (last != a.out) return hipMemcpyAsync(a.out, last, bytes, hipMemcpyDeviceToDevice, st);
  return hipSuccess;
}

}  // namespace mfft
