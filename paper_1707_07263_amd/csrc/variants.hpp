// Registry of compiled kernel variants.  Each variant is one instantiation of
// the strip-pass template (sub-transform length L, points per lane P, lines
// per workgroup W, lane mappings, inter-pass twiddle on/off, storage type).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"
#include "rowcol.hpp"

namespace mfft {

// ROLE_ROWCOL: 2-D row pass fused with a radix-W column step (k_rowcol)
enum Role { ROLE_ROW = 0, ROLE_SPLIT_A = 1, ROLE_COL = 2, ROLE_COL_TW = 3, ROLE_ROWCOL = 4 };
enum Dtype { DT_C64 = 0, DT_C16F = 1, DT_C16BF = 2 };

// start/stop: events (or null) that take the kernel's own start and end
// times, from its dispatch packet rather than from queue markers around it
using LaunchFn = hipError_t (*)(const PassArgs&, hipStream_t, hipEvent_t start, hipEvent_t stop);

struct Variant {
  const char* name;
  int L, P, W, threads, role, dtype;
  int lds_bytes;
  int tw_entries;  // stage-table entries for this (L, P)
  int ex;          // LDS exchange: 0 = (re, im) pairs, 1 = real then imaginary
  int tw_split = 0;  // stage twiddles from the two factor tables of W_L (k_rowcol TWP 2)
  int persistent;  // k_pipe (grid = resident workgroups, tiles walked in a loop) with
                   // 1 or 2 tiles' loads in flight; 0: k_strip
  LaunchFn launch;
  int (*blocks_per_cu)();  // persistent variants: resident workgroups per CU
};

template <int L, int P, int W, int LOADM, int STOREM, bool TWID, int EX, typename TS>
hipError_t launch_strip(const PassArgs& a, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  constexpr int NT = W * Sched<L, P>::T;
  hipExtLaunchKernelGGL((k_strip<L, P, W, LOADM, STOREM, TWID, EX, TS>), dim3((unsigned)a.total_tiles),
                        dim3(NT), 0, s, start, stop, 0, a);
  return hipGetLastError();
}

template <int L, int P, int W, int LOADM, int STOREM, bool TWID, int EX, typename TS, int DEPTH>
hipError_t launch_pipe(const PassArgs& a, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  constexpr int NT = W * Sched<L, P>::T;
  const unsigned grid = (unsigned)(a.grid > 0 ? a.grid : a.total_tiles);
  hipExtLaunchKernelGGL((k_pipe<L, P, W, LOADM, STOREM, TWID, EX, TS, DEPTH>), dim3(grid), dim3(NT), 0, s,
                        start, stop, 0, a);
  return hipGetLastError();
}

template <int L, int P, int W, int LOADM, int STOREM, bool TWID, int EX, typename TS, int DEPTH>
int blocks_pipe() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pipe<L, P, W, LOADM, STOREM, TWID, EX, TS, DEPTH>,
                                                   W * Sched<L, P>::T, 0) != hipSuccess)
    return 0;
  return n;
}

template <typename TS> struct DtOf;
template <> struct DtOf<float2> { static constexpr int v = DT_C64; };
template <> struct DtOf<__half2> { static constexpr int v = DT_C16F; };
template <> struct DtOf<c16bf> { static constexpr int v = DT_C16BF; };

template <int ROLE, int L, int P, int W, int EX, typename TS, int PERSIST = 0>
Variant make_variant(const char* name) {
  constexpr int LOADM = ROLE == ROLE_ROW ? 0 : 1;
  constexpr int STOREM = (ROLE == ROLE_COL || ROLE == ROLE_COL_TW) ? 1 : 0;
  constexpr bool TWID = ROLE == ROLE_SPLIT_A || ROLE == ROLE_COL_TW;
  Variant v;
  v.name = name;
  v.L = L;
  v.P = Sched<L, P>::PP;
  v.W = W;
  v.threads = W * Sched<L, P>::T;
  v.role = ROLE;
  v.dtype = DtOf<TS>::v;
  v.tw_entries = Sched<L, P>::TW;
  v.ex = EX;
  v.persistent = PERSIST;
  if constexpr (PERSIST) {
    // PERSIST = tiles in flight while one is computed (1 or 2)
    v.lds_bytes = pipe_lds_entries<L, P, W, EX, TWID>() * 8;
    v.launch = &launch_pipe<L, P, W, LOADM, STOREM, TWID, EX, TS, PERSIST>;
    v.blocks_per_cu = &blocks_pipe<L, P, W, LOADM, STOREM, TWID, EX, TS, PERSIST>;
  } else {
    v.lds_bytes = W * LdsLayout<L>::LS * (EX == 0 ? 8 : 4);
    v.launch = &launch_strip<L, P, W, LOADM, STOREM, TWID, EX, TS>;
    v.blocks_per_cu = nullptr;
  }
  return v;
}

template <int L, int P, int W, int EX, int TWP, typename TS>
hipError_t launch_rowcol(const PassArgs& a, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  constexpr int NT = W * Sched<L, P>::T;
  const unsigned grid = (unsigned)(a.grid > 0 ? a.grid : a.total_tiles);
  hipExtLaunchKernelGGL((k_rowcol<L, P, W, EX, TWP, TS>), dim3(grid), dim3(NT), 0, s, start, stop, 0, a);
  return hipGetLastError();
}

template <int L, int P, int W, int EX, int TWP, typename TS>
int blocks_rowcol() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rowcol<L, P, W, EX, TWP, TS>, W * Sched<L, P>::T, 0) !=
      hipSuccess)
    return 0;
  return n;
}

// A fused row pass: L = row length, W = rows per tile = radix of its
// column step, persistent.
template <int L, int P, int W, int EX, int TWP, typename TS>
Variant make_rowcol_variant(const char* name) {
  Variant v;
  v.name = name;
  v.L = L;
  v.P = Sched<L, P>::PP;
  v.W = W;
  v.threads = W * Sched<L, P>::T;
  v.role = ROLE_ROWCOL;
  v.dtype = DtOf<TS>::v;
  v.tw_entries = Sched<L, P>::TW;
  v.ex = EX;
  v.tw_split = TWP == 2;
  v.persistent = 1;
  v.lds_bytes = rowcol_lds_entries<L, P, W, EX, TWP>() * 8;
  v.launch = &launch_rowcol<L, P, W, EX, TWP, TS>;
  v.blocks_per_cu = &blocks_rowcol<L, P, W, EX, TWP, TS>;
  return v;
}

// Each instantiation file appends its variants.
void add_variants_c64_row(void (*add)(const Variant&));
void add_variants_c64_a(void (*add)(const Variant&));
void add_variants_c64_col(void (*add)(const Variant&));
void add_variants_c64_col2(void (*add)(const Variant&));
void add_variants_c64_pipe(void (*add)(const Variant&));
void add_variants_c16(void (*add)(const Variant&));
void add_variants_c64_rowcol(void (*add)(const Variant&));

// trivial length-1 / copy-scale kernel
hipError_t launch_scale_copy(int dtype, const void* in, void* out, int64_t n, float scale,
                             hipStream_t s);

}  // namespace mfft
