// Twiddle-table description and the float64 evaluation of W_M^e shared by the
// host generator and the GPU generator, so both produce the same table.
//
// Sec. 2.3.1 precomputes sin and cos "by a certain angle" into a look-up
// table.  Here every table entry is W_M^e = exp(-2*pi*i*e/M) evaluated in
// float64 and rounded to float32.  The angle is reduced exactly with integer
// arithmetic first (eq. 3 periodicity, then quadrant and octant symmetry), so
// sin/cos only ever see an argument in [0, pi/4] and each entry is the float32
// nearest the true value except in vanishingly rare near-tie cases.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mfft {

// Segment of a table: entries table[off + i], i < count, hold W_M^{e(i)} with
//   e(i) = (i / R) * (i % R) * mul   if R > 0  (2-D table: row i / R, column i % R)
//   e(i) = i * mul                   if R == 0 (linear table)
struct TwSeg {
  int64_t off, count, R, M, mul;
};

__host__ __device__ inline int64_t seg_exponent(const TwSeg& s, int64_t i) {
  return s.R > 0 ? (i / s.R) * (i % s.R) * s.mul : i * s.mul;
}

// cos and sin of 2*pi*e/M in float64 (M a power of two, any integer e).
__host__ __device__ inline void twiddle_fp64(int64_t e, int64_t M, double* c_out, double* s_out) {
  const double half_pi = 1.57079632679489661923132169163975144;
  int64_t r = e % M;
  if (r < 0) r += M;
  // 2*pi*r/M = q*(pi/2) + (pi/2)*(rem/M), with rem = 4r - qM in [0, M)
  const int64_t q = (4 * r) / M;
  const int64_t rem = 4 * r - q * M;
  double cs, sn;
  if (2 * rem <= M) {
    const double a = half_pi * ((double)rem / (double)M);  // in [0, pi/4]
    cs = cos(a);
    sn = sin(a);
  } else {
    const double b = half_pi * ((double)(M - rem) / (double)M);  // in (0, pi/4)
    cs = sin(b);
    sn = cos(b);
  }
  switch (q & 3) {
    case 0: *c_out = cs; *s_out = sn; break;
    case 1: *c_out = -sn; *s_out = cs; break;
    case 2: *c_out = -cs; *s_out = -sn; break;
    default: *c_out = sn; *s_out = -cs; break;
  }
}

hipError_t launch_twiddle_fp64(float2* table, const TwSeg* d_segs, int nseg, int64_t max_count,
                               hipStream_t s);

}  // namespace mfft
