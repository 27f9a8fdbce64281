// Device side of the MI355X FFT: complex helpers, in-register DFT codelets,
// the LDS-exchange Stockham engine and the strip-pass kernel template.
//
// The engine runs all butterfly stages of an L-point sub-transform inside one
// workgroup: each lane keeps P points in registers, runs radix-R butterflies
// there, and stages exchange data through LDS (the "all the butterflies in
// shared memory" idea of Sec. 2.3.2).  Stage twiddles W_{Ns*R}^{k*r} are read
// from a per-(L, P) table built once per plan (the sin/cos look-up table of
// Sec. 2.3.1); the reducibility of eq. 5 is what lets one table of an
// L-point transform serve every radix inside it.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <type_traits>
#include <stdint.h>

namespace mfft {

// ---------------------------------------------------------------------------
// complex helpers (float2 = (re, im))
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// a * (-i)
__device__ __forceinline__ float2 mul_negi(float2 a) { return make_float2(a.y, -a.x); }

// x * W_64^e with W_64 = exp(-2*pi*i/64), e a compile-time constant after
// unrolling (0 <= e < 64).  Exact forms for multiples of pi/4; otherwise the
// cosine comes from a quarter-wave table of cos(2*pi*k/64), k = 0..16.
__device__ __forceinline__ float2 mul_w64(float2 x, int e) {
  constexpr float Q[17] = {
      1.0f,                        0.995184726672196886244837f, 0.980785280403230449126182f,
      0.956940335732208864935798f, 0.923879532511286756128183f, 0.881921264348355029712757f,
      0.831469612302545237078788f, 0.773010453362736960810907f, 0.707106781186547524400844f,
      0.634393284163645498215172f, 0.555570233019602224742831f, 0.471396736825997648556388f,
      0.382683432365089771728460f, 0.290284677254462367636192f, 0.195090322016128267848285f,
      0.098017140329560601994196f, 0.0f};
  constexpr float R2 = 0.707106781186547524400844f;
  e &= 63;
  if (e == 0) return x;
  if (e == 16) return make_float2(x.y, -x.x);
  if (e == 32) return make_float2(-x.x, -x.y);
  if (e == 48) return make_float2(-x.y, x.x);
  if (e == 8) return make_float2((x.x + x.y) * R2, (x.y - x.x) * R2);
  if (e == 24) return make_float2((x.y - x.x) * R2, -(x.x + x.y) * R2);
  if (e == 40) return make_float2(-(x.x + x.y) * R2, (x.x - x.y) * R2);
  if (e == 56) return make_float2((x.x - x.y) * R2, (x.x + x.y) * R2);
  float c, s;  // W = (c, -s) with c = cos(2 pi e/64), s = sin(2 pi e/64)
  if (e < 16) { c = Q[e]; s = Q[16 - e]; }
  else if (e < 32) { c = -Q[32 - e]; s = Q[e - 16]; }
  else if (e < 48) { c = -Q[e - 32]; s = -Q[48 - e]; }
  else { c = Q[64 - e]; s = -Q[e - 48]; }
  return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
}

// ---------------------------------------------------------------------------
// forward DFT codelets in registers, natural order in and out:
//   A[k] = sum_r a[r] W_R^{rk}
// R = 2, 4 directly; larger R as an in-register four-step R = R1*R2 with
// compile-time twiddles W_R^{n2*k1}.
// ---------------------------------------------------------------------------
template <int R> struct Dft;

template <> struct Dft<1> {
  __device__ __forceinline__ static void run(float2*) {}
};
template <> struct Dft<2> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 t = csub(a[0], a[1]);
    a[0] = cadd(a[0], a[1]);
    a[1] = t;
  }
};
template <> struct Dft<4> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    float2 t2 = cadd(a[1], a[3]), t3 = mul_negi(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

// R = R1 * R2: n = R2*n1 + n2, k = k1 + R1*k2.
template <int R1, int R2> struct DftSplit {
  static constexpr int R = R1 * R2;
  __device__ __forceinline__ static void run(float2* a) {
    float2 y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 s[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) s[n1] = a[R2 * n1 + n2];
      Dft<R1>::run(s);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[k1 * R2 + n2] = mul_w64(s[k1], (n2 * k1 * (64 / R)) & 63);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      Dft<R2>::run(&y[k1 * R2]);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = y[k1 * R2 + k2];
    }
  }
};
template <> struct Dft<8> {
  __device__ __forceinline__ static void run(float2* a) { DftSplit<2, 4>::run(a); }
};
template <> struct Dft<16> {
  __device__ __forceinline__ static void run(float2* a) { DftSplit<4, 4>::run(a); }
};
template <> struct Dft<32> {
  __device__ __forceinline__ static void run(float2* a) { DftSplit<4, 8>::run(a); }
};

// ---------------------------------------------------------------------------
// compile-time schedule of an L-point sub-transform with P points per lane
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

template <int L, int P> struct Sched {
  static_assert(L >= 2 && (L & (L - 1)) == 0, "L must be a power of two >= 2");
  static constexpr int PP = P < L ? P : L;          // points per lane
  static constexpr int T = L / PP;                  // lanes per line
  static constexpr int LP = ilog2(PP);
  static constexpr int S = (ilog2(L) + LP - 1) / LP;  // stages
  static constexpr int FIRST = L >> ((S - 1) * LP);   // radix of stage 0
  __host__ __device__ static constexpr int radix(int s) { return s == 0 ? FIRST : PP; }
  __host__ __device__ static constexpr int ns(int s) { return s == 0 ? 1 : FIRST << ((s - 1) * LP); }
  // stage s >= 1 reads W_{ns*R}^{k*r} at tw[off(s) + k*R + r]
  __host__ __device__ static constexpr int off(int s) {
    return s <= 1 ? 0 : off(s - 1) + ns(s - 1) * radix(s - 1);
  }
  static constexpr int TW = off(S);  // table entries
};

// LDS index of point e of line m: one pad slot per 32 points, and a line
// stride of 2 modulo 32 slots, so that lanes striding across lines and lanes
// stepping 32 points inside a line fall on different banks (measured against
// one pad per 16 points with an odd stride: the 2-D image 142.3 -> 137.1 us,
// the other workloads unchanged or slightly faster).
template <int L> struct LdsLayout {
  static constexpr int LS = L + (L >> 5) + 2;
  __device__ __forceinline__ static int idx(int m, int e) { return m * LS + e + (e >> 5); }
};

// ---------------------------------------------------------------------------
// element storage types
// ---------------------------------------------------------------------------
struct c16bf { uint16_t x, y; };

__device__ __forceinline__ float2 load_c(const float2* p) { return *p; }
__device__ __forceinline__ float2 load_c(const __half2* p) { return __half22float2(*p); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float2 load_c(const c16bf* p) {
  c16bf v = *p;
  return make_float2(bf16_to_f32(v.x), bf16_to_f32(v.y));
}
// A complex64 point of a strided (column) pass, which reads every point
// once: loaded with the nontemporal hint, so that the caches favour the
// pass's output, which the next pass reads, over its input (measured on the
// two-pass 2^20 split: both passes of both directions got faster).  Only
// where a strip's row segment covers whole 128 B lines (16 or more columns):
// narrower strips share each line with the neighbouring strip, which then
// finds it evicted and fetches it again (the 8-column 2-D column pass got
// a third slower).
template <int LOADM, int W, typename TS>
__host__ __device__ constexpr bool kStreamLoads() {
  return LOADM == 1 && sizeof(TS) == 8 && W * sizeof(TS) >= 128;
}
__device__ __forceinline__ float2 load_stream(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v r = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(r.x, r.y);
}
__device__ __forceinline__ void store_c(float2* p, float2 v) { *p = v; }
// Two float32 values -> a packed float16 pair (lo in the low half), round
// to nearest, ties to even (the default rounding mode): one vector
// instruction on gfx950, where converting each half and packing takes three.
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi) {
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  f16x2 r;
  r.x = (_Float16)lo;
  r.y = (_Float16)hi;
  return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ void store_c(__half2* p, float2 v) {
  *reinterpret_cast<uint32_t*>(p) = pack_f16x2(v.x, v.y);
}
// Two float32 values -> a packed bfloat16 pair (lo in the low half), round
// to nearest, ties to even; NaN stays NaN.  gfx950 converts the pair in one
// vector instruction (the conversion written out with integer operations
// took about a dozen per pair).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  bf16x2 r;
  r.x = (__bf16)lo;
  r.y = (__bf16)hi;
  return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ void store_c(c16bf* p, float2 v) {
  *reinterpret_cast<uint32_t*>(p) = pack_bf16x2(v.x, v.y);
}

// ---------------------------------------------------------------------------
// pass arguments (one kernel launch)
// ---------------------------------------------------------------------------
struct PassArgs {
  const void* in;
  void* out;
  int64_t in_batch, out_batch;  // element stride between batches
  int64_t in_line, out_line;    // element stride between adjacent lines
  int64_t in_elem, out_elem;    // element stride between points of a line
  int64_t total_tiles;          // tiles_per_batch * batch
  int32_t tiles_per_batch;      // ceil(lines / W)
  int32_t lines;                // lines per batch
  const float2* tw;             // stage table of this (L, P)
  const float2* tw_lo;          // inter-pass: W_N^{j & mask}
  const float2* tw_hi;          // inter-pass: W_N^{(j >> shift) << shift}
  const float2* tw_step;        // inter-pass: W_N^{line*q*T}, [lines][P]
  int32_t tw_shift, tw_mask;
  float scale;                  // applied to every output value
  int32_t conj_in, conj_out;    // inverse direction: conj on first load / last store
  int32_t xcd_remap;            // 1: consecutive tiles on one XCD
  int32_t grid;                 // persistent kernels: workgroups launched (host sets)
  int32_t tw_line_shift;        // inter-pass twiddle uses line >> shift as its row index
  // row pass of the three-pass 2-D plan: tile t of a batch reads rows
  // line_map[t*W + m] and writes each row r to its transpose in an S x S
  // grid of rows, S = 2^tr_shift (pairs (r, r^T) share a tile, so the
  // permutation happens in place)
  const int32_t* line_map;
  int32_t tr_shift;
  // row pass of the blocked 2-D plan: outputs go to column blocks of
  // 2^blk_lg columns, block j of an image holding columns j*2^blk_lg ..
  // (j+1)*2^blk_lg - 1 of its 2^blk_rows_lg rows, row after row (0: natural
  // order)
  int32_t blk_lg, blk_rows_lg;
};

// Where point t + q*T of row `line` goes in the blocked layout: the lane's
// first element, and the step between its points (T a multiple of the block
// width, so a lane stays in one column of a block as q runs).
__device__ __forceinline__ int64_t blk_base(const PassArgs& a, int64_t line, int t) {
  const int64_t img = line >> a.blk_rows_lg;
  const int64_t r = line & ((1 << a.blk_rows_lg) - 1);
  return img * (a.out_line << a.blk_rows_lg) + ((int64_t)(t >> a.blk_lg) << (a.blk_rows_lg + a.blk_lg)) +
         (r << a.blk_lg) + (t & ((1 << a.blk_lg) - 1));
}

__device__ __forceinline__ int row_transpose(int r, int sh) {
  return ((r & ((1 << sh) - 1)) << sh) | (r >> sh);
}

// Map a workgroup id to a tile so that tiles t, t+1, ... run on the same XCD
// (workgroups are dealt round-robin to the 8 XCDs, each with its own L2).
__device__ __forceinline__ int64_t tile_of(int64_t b, int64_t n, int remap) {
  if (!remap || (n & 7)) return b;
  return (b & 7) * (n >> 3) + (b >> 3);
}

// Wait until at most N vector memory operations of this wave are
// outstanding.
template <int N>
__device__ __forceinline__ void vm_wait() {
  // s_waitcnt: vmcnt in bits [3:0] and [15:14], expcnt [6:4] = 7 and
  // lgkmcnt [11:8] = 15 left at their maxima (not waited for)
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier that orders LDS accesses only (fences scoped to the
// "local" address space): global loads issued before it stay in flight, which
// is what lets the persistent kernel prefetch the next tile across the
// exchanges of the current one.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Entries of the two factor tables of W_L (TWP 2): 2^LA + 2^(log2 L - LA).
__host__ __device__ constexpr int tw_split_entries(int L) {
  return (1 << ((ilog2(L) + 1) / 2)) + (1 << (ilog2(L) - (ilog2(L) + 1) / 2));
}

// Stage twiddles staged in LDS: the same entries as the global table, with
// each k-row of R factors padded to R + 1.  Lanes k of a wave read row k
// together; with an odd row stride those rows start on different banks (a
// stride of R + 2 put rows k and k + 16 on the same banks: the first pass of
// the 2^20 split stalled twice as many cycles on bank conflicts and ran
// about 1 us slower per launch).
template <int L, int P> struct TwLds {
  using S = Sched<L, P>;
  __host__ __device__ static constexpr int rp(int s) { return S::radix(s) >= 4 ? S::radix(s) + 1 : S::radix(s); }
  __host__ __device__ static constexpr int off(int s) {
    return s <= 1 ? 0 : off(s - 1) + S::ns(s - 1) * rp(s - 1);
  }
  static constexpr int SIZE = off(S::S) > 0 ? off(S::S) : 1;
  // cooperative copy from the global table (entries tw[S::off(s) + k*R + r])
  __device__ __forceinline__ static void copy(float2* dst, const float2* __restrict__ src, int tid, int nt) {
    for (int i = tid; i < S::TW; i += nt) {
      int s = 1;
#pragma unroll
      for (int q = 2; q < S::S; ++q)
        if (i >= S::off(q)) s = q;
      const int R = S::radix(s);
      const int loc = i - S::off(s);
      const int k = loc / R, r = loc % R;
      dst[off(s) + k * rp(s) + r] = src[i];
    }
  }
};

// ---------------------------------------------------------------------------
// LDS exchange between two stages.  Lane (m, t) holds the previous stage's
// outputs in v[b + r*NB] destined for positions o0[b] + r*NS of line m; after
// the exchange lane (m2, t2) holds points t2 + q*T of line m2 in v[q].
// EX = 0 moves (re, im) pairs in one round through a float2 array; EX = 1
// moves the real parts, then the imaginary parts, through a float array of
// half the size (twice the barriers, half the LDS, so twice the workgroups
// fit on a CU).
// ---------------------------------------------------------------------------
template <int L, int PP, int EX, int R, int NS>
__device__ __forceinline__ void exchange(float2* v, void* ldsv, int m, int m2, int t2, const int* o0) {
  using LY = LdsLayout<L>;
  constexpr int T = L / PP;
  constexpr int NB = PP / R;
  if constexpr (EX == 0) {
    float2* lds = reinterpret_cast<float2*>(ldsv);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[LY::idx(m, o0[b] + r * NS)] = v[b + r * NB];
    lds_barrier();
#pragma unroll
    for (int q = 0; q < PP; ++q) v[q] = lds[LY::idx(m2, t2 + q * T)];
    lds_barrier();
  } else {
    float* lds = reinterpret_cast<float*>(ldsv);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[LY::idx(m, o0[b] + r * NS)] = v[b + r * NB].x;
    lds_barrier();
    // the real parts are dead once written: reuse their registers
#pragma unroll
    for (int q = 0; q < PP; ++q) v[q].x = lds[LY::idx(m2, t2 + q * T)];
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[LY::idx(m, o0[b] + r * NS)] = v[b + r * NB].y;
    lds_barrier();
#pragma unroll
    for (int q = 0; q < PP; ++q) v[q].y = lds[LY::idx(m2, t2 + q * T)];
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// The engine: all stages of W independent L-point transforms held by one
// workgroup, P points per lane.  On entry lane (m, t) holds points t + q*T of
// line m in v[q]; on exit lane (m_st, t_st) holds outputs t_st + q*T of line
// m_st (natural order).  Stage s (radix R, span NS) is a Stockham
// (self-sorting) decimation-in-time step: butterfly j takes points
// j + r*L/R, multiplies them by W_{NS*R}^{(j mod NS)*r}, runs an R-point DFT
// and writes output r to (j div NS)*NS*R + (j mod NS) + r*NS.  The lane
// mapping switches from (m, t) to (m_st, t_st) at the first LDS exchange.
// Stages are unrolled by compile-time recursion so that every radix, span
// and register index is a constant.
// ---------------------------------------------------------------------------
template <int L, int P, int EX, int s, int TWP = 0>
struct Stage {
  using S = Sched<L, P>;
  static constexpr int T = S::T;
  static constexpr int PP = S::PP;
  static constexpr int R = S::radix(s);
  static constexpr int NS = S::ns(s);
  static constexpr int NB = PP / R;
  __device__ __forceinline__ static void run(float2* v, void* lds, int& m, int& t, int m_st,
                                             int t_st, const float2* __restrict__ twt) {
    int o0[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * T;
      const int k = j & (NS - 1);
      o0[b] = (j / NS) * NS * R + k;
      float2 x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[b + r * NB];
      if constexpr (s > 0 && TWP == 2) {
        // TWP 2: W_{NS*R}^{k r} = W_L^e, e = k r L/(NS R), from two factor
        // tables in LDS, twt[i] = W_L^i (i < 2^LA) and
        // twt[2^LA + i] = W_L^{i 2^LA}: a few hundred bytes instead of the
        // stage table
        constexpr int LG = ilog2(L), LA = (LG + 1) / 2, SC = L / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int e = k * r * SC;
          x[r] = cmul(x[r], cmul(twt[e & ((1 << LA) - 1)], twt[(1 << LA) + (e >> LA)]));
        }
      } else if constexpr (s > 0) {
        // TWP 0: global table; TWP 1: LDS copy with padded rows
        const float2* tw = TWP == 0 ? twt + S::off(s) + k * R
                                    : twt + TwLds<L, P>::off(s) + k * TwLds<L, P>::rp(s);
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[r]);
      }
      Dft<R>::run(x);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * NB] = x[r];
    }
    if constexpr (s < S::S - 1) {
      exchange<L, PP, EX, R, NS>(v, lds, m, m_st, t_st, o0);
      m = m_st;
      t = t_st;
      Stage<L, P, EX, s + 1, TWP>::run(v, lds, m, t, m_st, t_st, twt);
    }
  }
};

template <int L, int P, int W, int EX, int TWP = 0>
__device__ __forceinline__ void run_stages(float2* v, void* lds, int& m, int& t,
                                           int m_st, int t_st, bool remap,
                                           const float2* __restrict__ twt) {
  using S = Sched<L, P>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  Stage<L, P, EX, 0, TWP>::run(v, lds, m, t, m_st, t_st, twt);
  if constexpr (S::S == 1) {
    if (remap) {
      // one-stage transform whose load and store mappings differ: transpose
      // through LDS (`remap` is uniform across the workgroup)
      int o0[PP];
#pragma unroll
      for (int q = 0; q < PP; ++q) o0[q] = t + q * T;
      exchange<L, PP, EX, 1, 1>(v, lds, m, m_st, t_st, o0);
      m = m_st;
      t = t_st;
    }
  }
}

// ---------------------------------------------------------------------------
// The strip pass.  A workgroup transforms W lines ("a strip") of L points.
// Lane mapping: LOADM/STOREM = 1 puts the line index m fastest across lanes
// (W adjacent lines of a strided view -> W-wide contiguous segments), 0 puts
// the point index fastest (contiguous lines).  With TWID the outputs are
// multiplied by W_N^{line*k} (the inter-pass twiddle of the N1 x N2 split).
// ---------------------------------------------------------------------------
// Waves per SIMD the kernel must allow so that every workgroup its LDS
// footprint lets onto a CU can be resident (4 SIMDs per CU, at most 8 waves
// per SIMD, 160 KB of LDS per CU); passed to the register allocator, capped
// at 4 waves (128 VGPRs) so that no variant is squeezed into spilling.
// Only row passes (contiguous lines in and out) take a line map; for the
// other lane mappings the persistent pass knows it is absent at compile
// time, so its loop carries no load whose result the next tile's addresses
// would wait for.
template <int LOADM, int STOREM>
__host__ __device__ constexpr bool kLineMap() {
  return LOADM == 0 && STOREM == 0;
}

template <int L, int P, int W, int EX>
__host__ __device__ constexpr int strip_min_waves() {
  constexpr int nt = W * Sched<L, P>::T;
  constexpr int lds = W * LdsLayout<L>::LS * (EX == 0 ? 8 : 4);
  constexpr int per_cu_lds = 163840 / (lds > 0 ? lds : 1);
  constexpr int waves_wg = (nt + 63) / 64;
  constexpr int per_cu = per_cu_lds < 32 / waves_wg ? per_cu_lds : 32 / waves_wg;
  constexpr int w = (per_cu * waves_wg + 3) / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

template <int L, int P, int W, int LOADM, int STOREM, bool TWID, int EX, typename TS>
__global__ void __launch_bounds__((W * Sched<L, P>::T), (strip_min_waves<L, P, W, EX>()))
k_strip(PassArgs a) {
  using S = Sched<L, P>;
  using LY = LdsLayout<L>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  __shared__ float2 lds[EX == 0 ? W * LY::LS : (W * LY::LS + 1) / 2];

  const int tid = threadIdx.x;
  const int64_t tile = tile_of(blockIdx.x, a.total_tiles, a.xcd_remap);
  const int64_t bat = tile / a.tiles_per_batch;
  const int line0 = (int)(tile - bat * a.tiles_per_batch) * W;

  int m = LOADM ? tid % W : tid / T;
  int t = LOADM ? tid / W : tid % T;
  const int m_st = STOREM ? tid % W : tid / T;
  const int t_st = STOREM ? tid / W : tid % T;

  const int tile_in_batch = (int)(tile - bat * a.tiles_per_batch);
  float2 v[PP];
  {
    // lines past the end of a partial strip load a valid line and are not stored
    const int ln = a.line_map ? a.line_map[tile_in_batch * W + m] : min(line0 + m, a.lines - 1);
    const TS* src = reinterpret_cast<const TS*>(a.in) + bat * a.in_batch +
                    (int64_t)ln * a.in_line + (int64_t)t * a.in_elem;
    const int64_t step = (int64_t)T * a.in_elem;
    const uint32_t sgn = a.conj_in ? 0x80000000u : 0u;
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      if constexpr (kStreamLoads<LOADM, W, TS>())
        v[q] = load_stream(reinterpret_cast<const float2*>(src + q * step));
      else
        v[q] = load_c(src + q * step);
      v[q].y = __uint_as_float(__float_as_uint(v[q].y) ^ sgn);
    }
  }

  run_stages<L, P, W, EX>(v, lds, m, t, m_st, t_st, LOADM != STOREM, a.tw);

  // epilogue: inter-pass twiddle, scale, conjugate, store
  {
    const int line = a.line_map ? row_transpose(a.line_map[tile_in_batch * W + m], a.tr_shift)
                                : line0 + m;
    const bool ok = a.line_map ? true : line < a.lines;
    TS* dst = reinterpret_cast<TS*>(a.out) + bat * a.out_batch + (int64_t)line * a.out_line +
              (int64_t)t * a.out_elem;
    int64_t step = (int64_t)T * a.out_elem;
    if (!TWID && STOREM == 0 && a.blk_lg) {
      dst = reinterpret_cast<TS*>(a.out) + blk_base(a, line, t);
      step = (int64_t)T << a.blk_rows_lg;
    }
    // inter-pass twiddle W_N^{row*(t + q*T)} = W_N^{row*t} * W_N^{row*q*T}
    // (row = line >> tw_line_shift): one base per lane, and a step row
    // shared by the lanes of a line
    float2 tw_base = make_float2(1.f, 0.f);
    const float2* tw_row = a.tw_step;
    if (TWID && ok) {
      const uint32_t row = (uint32_t)line >> a.tw_line_shift;
      const uint32_t jb = row * (uint32_t)t;
      tw_base = cmul(a.tw_hi[jb >> a.tw_shift], a.tw_lo[jb & (uint32_t)a.tw_mask]);
      tw_row = a.tw_step + (int64_t)row * PP;
    }
    const uint32_t sgn = a.conj_out ? 0x80000000u : 0u;
    if (ok) {
#pragma unroll
      for (int q = 0; q < PP; ++q) {
        float2 y = v[q];
        if (TWID) y = cmul(y, cmul(tw_base, tw_row[q]));
        y = cscale(y, a.scale);
        y.y = __uint_as_float(__float_as_uint(y.y) ^ sgn);
        store_c(dst + q * step, y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined strip pass.  One workgroup per CU walks the
// tiles tile = blockIdx.x, + gridDim.x, ...; while it computes and stores one
// tile, the loads of its next DEPTH tiles (data, and for the split's first
// pass the twiddle inputs) are already in flight, so memory transfer
// overlaps the butterflies instead of alternating with them.  With DEPTH 2
// the loads of two tiles are in flight at every point of the walk, which
// keeps the memory system busy through a tile's compute and stores as well
// (the first pass has only a few tiles per CU, so the ramp at the start and
// the drain at the end weigh).  Everything read between issuing a prefetch
// and consuming it comes from LDS (the stage twiddles are copied there
// once), since waiting on any later global load would also wait for the
// prefetch.  Same lane mappings, stages and outputs as k_strip.
// ---------------------------------------------------------------------------
template <int L, int P, int W, int EX, bool TWID>
__host__ __device__ constexpr int pipe_lds_entries() {
  return (EX == 0 ? W * LdsLayout<L>::LS : (W * LdsLayout<L>::LS + 1) / 2) + TwLds<L, P>::SIZE +
         (TWID ? W * (Sched<L, P>::PP + 2) : 0);
}

template <int L, int P, int W, int LOADM, int STOREM, bool TWID, int EX, typename TS, int DEPTH>
__global__ void __launch_bounds__((W * Sched<L, P>::T), 1)
k_pipe(PassArgs a) {
  static_assert(DEPTH == 1 || DEPTH == 2, "one or two tiles in flight");
  using S = Sched<L, P>;
  using LY = LdsLayout<L>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  constexpr int NT = W * T;
  constexpr int XN = EX == 0 ? W * LY::LS : (W * LY::LS + 1) / 2;
  __shared__ float2 lds[pipe_lds_entries<L, P, W, EX, TWID>()];
  float2* xch = lds;
  float2* twl = lds + XN;
  float2* rowl = lds + XN + TwLds<L, P>::SIZE;

  int tid = threadIdx.x;
  int m_ld, t_ld, m_st, t_st;
  // lane indices, recomputed from an opaque copy of the lane id once per
  // tile: values derived from them are then cheap to rebuild in the loop
  // and are not held in registers across it
  auto lanes = [&]() {
    asm volatile("" : "+v"(tid));
    m_ld = LOADM ? tid % W : tid / T;
    t_ld = LOADM ? tid / W : tid % T;
    m_st = STOREM ? tid % W : tid / T;
    t_st = STOREM ? tid / W : tid % T;
  };
  lanes();
  const uint32_t sgn_in = a.conj_in ? 0x80000000u : 0u;
  const uint32_t sgn_out = a.conj_out ? 0x80000000u : 0u;

  TwLds<L, P>::copy(twl, a.tw, tid, NT);

  // registers of a prefetched tile; 16-bit pairs stay in their storage type
  // (one register each) until they are converted when the tile is consumed.
  // A tile's W*PP step-row entries are held KR per lane.
  using PreT = typename std::conditional<sizeof(TS) == 8, float2, TS>::type;
  constexpr int KR = TWID ? (W * PP + NT - 1) / NT : 1;
  struct Pre {
    PreT v[PP];
    float2 row[KR];
    float2 lo, hi;
  };
  auto prefetch = [&](Pre& n, int64_t tl) {
    const int64_t bat = tl / a.tiles_per_batch;
    const int line0 = (int)(tl - bat * a.tiles_per_batch) * W;
    const int tib = (int)(tl - bat * a.tiles_per_batch);
    const int ln = (kLineMap<LOADM, STOREM>() && a.line_map) ? a.line_map[tib * W + m_ld]
                                                              : min(line0 + m_ld, a.lines - 1);
    const TS* src = reinterpret_cast<const TS*>(a.in) + bat * a.in_batch +
                    (int64_t)ln * a.in_line + (int64_t)t_ld * a.in_elem;
    const int64_t step = (int64_t)T * a.in_elem;
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      if constexpr (kStreamLoads<LOADM, W, TS>())
        n.v[q] = load_stream(reinterpret_cast<const float2*>(src + q * step));
      else if constexpr (sizeof(TS) == 8)
        n.v[q] = load_c(src + q * step);
      else
        n.v[q] = src[q * step];
    }
    if (TWID) {
      // this tile's step rows W_N^{row*q*T} and the lane's base W_N^{row*t},
      // row = line >> tw_line_shift
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        const int e = tid + j * NT;
        if (W * PP == KR * NT || e < W * PP)
          n.row[j] = a.tw_step[(int64_t)((uint32_t)min(line0 + e / PP, a.lines - 1) >> a.tw_line_shift) * PP +
                               (e % PP)];
      }
      const uint32_t jb = ((uint32_t)min(line0 + m_st, a.lines - 1) >> a.tw_line_shift) * (uint32_t)t_st;
      n.lo = a.tw_lo[jb & (uint32_t)a.tw_mask];
      n.hi = a.tw_hi[jb >> a.tw_shift];
    }
  };

  // one tile: consume the registers prefetched for it, refill them with the
  // tile `ahead` (if any), then butterflies, twiddle and stores
  auto body = [&](Pre& n, int64_t tile, int64_t ahead) {
    lanes();
    float2 v[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      if constexpr (sizeof(TS) == 8)
        v[q] = n.v[q];
      else
        v[q] = load_c(&n.v[q]);
      v[q].y = __uint_as_float(__float_as_uint(v[q].y) ^ sgn_in);
    }
    float2 tw_base = make_float2(1.f, 0.f);
    if (TWID) {
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        const int e = tid + j * NT;
        // rows of PP + 2 entries: the lines of a wave read their step rows
        // on different banks
        if (W * PP == KR * NT || e < W * PP) rowl[(e / PP) * (PP + 2) + e % PP] = n.row[j];
      }
      tw_base = cmul(n.hi, n.lo);
    }
    const int64_t bat = tile / a.tiles_per_batch;
    const int line0 = (int)(tile - bat * a.tiles_per_batch) * W;
    if (ahead < a.total_tiles) prefetch(n, ahead);

    int m = m_ld, t = t_ld;
    run_stages<L, P, W, EX, 1>(v, xch, m, t, m_st, t_st, LOADM != STOREM, twl);
    if (TWID) lds_barrier();  // step rows visible (also when no exchange ran)

    const int tib = (int)(tile - bat * a.tiles_per_batch);
    const bool lmap = kLineMap<LOADM, STOREM>() && a.line_map;
    const int line = lmap ? row_transpose(a.line_map[tib * W + m], a.tr_shift) : line0 + m;
    // rows past the end of a partial strip loaded a copy of the last line and
    // computed exactly its result (same data, same twiddles, same order of
    // operations): they store it over the last line, the same bits.  Every
    // lane stores, so the number of memory operations after the prefetch is
    // the same on every path and the next tile waits for its own prefetch
    // only, not for these stores.
    const int line_st = lmap ? line : min(line, a.lines - 1);
    TS* dst = reinterpret_cast<TS*>(a.out) + bat * a.out_batch + (int64_t)line_st * a.out_line +
              (int64_t)t * a.out_elem;
    int64_t step = (int64_t)T * a.out_elem;
    if (!TWID && STOREM == 0 && a.blk_lg) {
      dst = reinterpret_cast<TS*>(a.out) + blk_base(a, line_st, t);
      step = (int64_t)T << a.blk_rows_lg;
    }
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      float2 y = v[q];
      if (TWID) y = cmul(y, cmul(tw_base, rowl[m * (PP + 2) + q]));
      y = cscale(y, a.scale);
      y.y = __uint_as_float(__float_as_uint(y.y) ^ sgn_out);
      store_c(dst + q * step, y);
    }
    lds_barrier();  // LDS reads of this tile done before the next one overwrites
  };

  // with the XCD remap, the workgroups of one XCD start on consecutive
  // tiles, so that neighbouring strips, which share cache lines when a row
  // segment is narrower than a line, are in flight on one L2 together
  const int64_t G = gridDim.x;
  int64_t tile = tile_of(blockIdx.x, G, a.xcd_remap);
  // The prologue's prefetch is drained before the walk starts, so that the
  // top of the loop sees the same memory state from the prologue as from
  // its back edge (the previous tile's stores in flight, its prefetch
  // done); otherwise the compiler's wait at the top, which must hold for
  // both paths, waits for those stores as well.
  if constexpr (DEPTH == 1) {
    Pre pa;
    if (tile < a.total_tiles) prefetch(pa, tile);
    vm_wait<0>();
    lds_barrier();  // stage twiddles visible
    for (; tile < a.total_tiles; tile += G) body(pa, tile, tile + G);
  } else {
    // two register sets alternate: the walk is unrolled by two so that each
    // set keeps fixed registers
    Pre pa, pb;
    if (tile < a.total_tiles) prefetch(pa, tile);
    if (tile + G < a.total_tiles) prefetch(pb, tile + G);
    vm_wait<0>();
    lds_barrier();  // stage twiddles visible
    for (; tile < a.total_tiles; tile += 2 * G) {
      body(pa, tile, tile + 2 * G);
      if (tile + G < a.total_tiles) body(pb, tile + G, tile + 3 * G);
    }
  }
}

// Length-1 transforms and other trivial cases: out = scale * in (conj is a
// no-op pair for length 1).
template <typename TS>
__global__ void __launch_bounds__(256) k_scale_copy(const TS* in, TS* out, int64_t n, float scale) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) store_c(out + i, cscale(load_c(in + i), scale));
}

}  // namespace mfft
