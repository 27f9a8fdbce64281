// Row pass of a 2-D transform fused with the first radix-W step of its
// columns (Sec. 2.3.2: rows, then columns; each column length R split as
// R = W * M by eq. 5).
//
// With row index n = n1 + M*j (n1 < M, j < W) and column frequency
// k = W*k1 + k2 (k2 < W), the column DFT of the row-transformed image Y is
//   X[W k1 + k2] = sum_{n1} W_M^{n1 k1} * ( W_R^{n1 k2} * sum_j W_W^{j k2} Y[n1 + M j] ).
// A tile of this pass holds the W rows n1 + M*j of one image: it transforms
// each row (C points) and then, per column, takes the W-point DFT across the
// tile's rows and the twiddle W_R^{n1 k2}, and writes the result for k2 to
// row W*n1 + k2, so a tile reads W whole rows and writes W consecutive whole
// rows.  The column step goes through LDS: lane c takes column c of every
// row, so each store instruction writes one contiguous run of a row.  (Row
// outputs interleaved across lanes, W per DPP quad, would skip that LDS
// round trip, but then each store writes W separate 128 B pieces; measured
// 86 against 66 us for the 4096-point rows of a 4096^2 image.)
//
// What is left are M-point column transforms over rows W*n1 + k2 (stride W
// rows) for each k2, in place, with output frequency k1 landing on row
// W*k1 + k2: a column pass of M-point lines whose tiles can be W times wider
// than those of an R-point column pass for the same LDS.
#pragma once

#include "fft_device.hpp"

namespace mfft {

// TWP 1: the stage twiddles in LDS; TWP 2: built from two factor tables of
// W_L, which leaves the LDS to a one-round exchange of the four rows
template <int L, int P, int W, int EX, int TWP>
__host__ __device__ constexpr int rowcol_lds_entries() {
  return (EX == 0 ? W * LdsLayout<L>::LS : (W * LdsLayout<L>::LS + 1) / 2) +
         (TWP == 2 ? tw_split_entries(L) : TwLds<L, P>::SIZE);
}

// PassArgs as used here: lines = R rows per image, tiles_per_batch = M =
// R / W (a power of two, tw_shift = log2 M), in_line = out_line = C,
// in_elem = out_elem = 1, in_batch = out_batch = R * C, tw = the row length's
// stage table (TWP 1) or the factor tables of W_L (TWP 2), tw_lo = W_R^e
// for e < R.  Persistent: workgroup g walks tiles g, g + G, ... with the
// next tile's loads in flight.
template <int L, int P, int W, int EX, int TWP, typename TS>
__global__ void __launch_bounds__((W * Sched<L, P>::T), 1) k_rowcol(PassArgs a) {
  using S = Sched<L, P>;
  using LY = LdsLayout<L>;
  constexpr int T = S::T;    // lanes per row
  constexpr int PP = S::PP;  // points per lane
  constexpr int NT = W * T;
  constexpr int CPL = L / NT;  // columns per lane in the column step
  static_assert(W == 2 || W == 4, "radix of the fused column step");
  static_assert(CPL * W == PP && CPL * NT == L, "a lane takes CPL columns of all W rows");
  constexpr int XN = EX == 0 ? W * LY::LS : (W * LY::LS + 1) / 2;
  __shared__ float2 lds[rowcol_lds_entries<L, P, W, EX, TWP>()];
  float2* xch = lds;
  float2* twl = lds + XN;

  int tid = threadIdx.x;
  if constexpr (TWP == 2) {
    for (int i = tid; i < tw_split_entries(L); i += NT) twl[i] = a.tw[i];
  } else {
    TwLds<L, P>::copy(twl, a.tw, tid, NT);
  }
  const int lgM = a.tw_shift;
  const int64_t M = (int64_t)1 << lgM;
  const uint32_t sgn_in = a.conj_in ? 0x80000000u : 0u;
  const uint32_t sgn_out = a.conj_out ? 0x80000000u : 0u;

  using PreT = typename std::conditional<sizeof(TS) == 8, float2, TS>::type;
  PreT vn[PP];
  float2 wn[W];
  auto prefetch = [&](int64_t tl) {
    asm volatile("" : "+v"(tid));
    const int64_t b = tl >> lgM;
    const int64_t n1 = tl & (M - 1);
    const int m = tid / T, t = tid % T;
    const TS* src = reinterpret_cast<const TS*>(a.in) + b * a.in_batch + (n1 + m * M) * a.in_line +
                    (int64_t)t * a.in_elem;
    const int64_t step = (int64_t)T * a.in_elem;
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      if constexpr (sizeof(TS) == 8)
        vn[q] = load_stream(reinterpret_cast<const float2*>(src + q * step));
      else
        vn[q] = src[q * step];
    }
    // W_R^{n1 k2}, k2 < W (n1 k2 < M W = R)
#pragma unroll
    for (int k2 = 1; k2 < W; ++k2) wn[k2] = a.tw_lo[n1 * k2];
  };

  const int64_t G = gridDim.x;
  int64_t tile = tile_of(blockIdx.x, G, a.xcd_remap);
  if (tile < a.total_tiles) prefetch(tile);
  // drained here so that the top of the loop sees the same memory state on
  // its first pass as from its back edge (else its wait covers the stores)
  vm_wait<0>();
  lds_barrier();  // stage twiddles visible
  for (; tile < a.total_tiles; tile += G) {
    asm volatile("" : "+v"(tid));
    float2 v[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      if constexpr (sizeof(TS) == 8)
        v[q] = vn[q];
      else
        v[q] = load_c(&vn[q]);
      v[q].y = __uint_as_float(__float_as_uint(v[q].y) ^ sgn_in);
    }
    float2 w[W];
    w[0] = make_float2(1.f, 0.f);
#pragma unroll
    for (int k2 = 1; k2 < W; ++k2) w[k2] = wn[k2];
    const int64_t b = tile >> lgM;
    const int64_t n1 = tile & (M - 1);
    if (tile + G < a.total_tiles) prefetch(tile + G);

    // the W row transforms (contiguous rows in and out: point-fastest lanes)
    int m = tid / T, t = tid % T;
    run_stages<L, P, W, EX, TWP>(v, xch, m, t, m, t, false, twl);

    // column step: lane tid takes columns c = tid + i*NT of every row j,
    // v[j*CPL + i] <- row j, column c (the exchange buffer is free: the
    // stages end with a barrier after their last LDS read)
    if constexpr (EX == 0) {
#pragma unroll
      for (int q = 0; q < PP; ++q) xch[LY::idx(m, t + q * T)] = v[q];
      lds_barrier();
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int i = 0; i < CPL; ++i) v[j * CPL + i] = xch[LY::idx(j, tid + i * NT)];
    } else {
      float* xf = reinterpret_cast<float*>(xch);
#pragma unroll
      for (int q = 0; q < PP; ++q) xf[LY::idx(m, t + q * T)] = v[q].x;
      lds_barrier();
      // the real parts are dead once written: reuse their registers
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int i = 0; i < CPL; ++i) v[j * CPL + i].x = xf[LY::idx(j, tid + i * NT)];
      lds_barrier();
#pragma unroll
      for (int q = 0; q < PP; ++q) xf[LY::idx(m, t + q * T)] = v[q].y;
      lds_barrier();
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int i = 0; i < CPL; ++i) v[j * CPL + i].y = xf[LY::idx(j, tid + i * NT)];
    }
    TS* dst = reinterpret_cast<TS*>(a.out) + b * a.out_batch + (W * n1) * a.out_line;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      float2 x[W];
#pragma unroll
      for (int j = 0; j < W; ++j) x[j] = v[j * CPL + i];
      Dft<W>::run(x);
      const int64_t c = tid + i * NT;
#pragma unroll
      for (int k2 = 0; k2 < W; ++k2) {
        float2 y = k2 ? cmul(x[k2], w[k2]) : x[k2];
        y = cscale(y, a.scale);
        y.y = __uint_as_float(__float_as_uint(y.y) ^ sgn_out);
        store_c(dst + k2 * a.out_line + c * a.out_elem, y);
      }
    }
    lds_barrier();  // LDS reads of this tile done before the next one writes
  }
}

}  // namespace mfft
