// Persistent kernel for many transforms of uneven power-of-two lengths.
#include "fft_device.hpp"
#include "many.hpp"
#include "variants.hpp"

namespace mfft {

// LDS needed by a tile of length 2^lg: W = NT/T lines of the padded
// layout's line stride (LdsLayout<L>::LS).
template <int P, int NT>
__host__ __device__ constexpr int many_lds_len(int lg) {
  return lg == 0 ? NT
                 : (NT / ((1 << lg) / ((P < (1 << lg)) ? P : (1 << lg)))) *
                       ((1 << lg) + ((1 << lg) >> 5) + 2);
}
template <int P, int NT, int MAXLG = kManyMaxLg>
__host__ __device__ constexpr int many_lds_max(int lg = 0) {
  return lg > MAXLG ? 0
                    : (many_lds_len<P, NT>(lg) > many_lds_max<P, NT, MAXLG>(lg + 1)
                           ? many_lds_len<P, NT>(lg)
                           : many_lds_max<P, NT, MAXLG>(lg + 1));
}

// One tile of length L (lines of L points, W = NT/T of them).
template <int L, int P, int NT, typename TS>
__device__ __forceinline__ void many_tile(const ManyArgs& a, const ManyItem& d, float2* lds, int tid) {
  using S = Sched<L, P>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  constexpr int W = NT / T;
  static_assert(W >= 1 && W * T == NT, "tile must fill the workgroup");
  const bool mfast_in = d.kind != MANY_SINGLE;
  const bool mfast_out = d.kind == MANY_B;
  int m = mfast_in ? tid % W : tid / T;
  int t = mfast_in ? tid / W : tid % T;
  const int m_st = mfast_out ? tid % W : tid / T;
  const int t_st = mfast_out ? tid / W : tid % T;

  const TS* src = reinterpret_cast<const TS*>(a.in);
  TS* dst = reinterpret_cast<TS*>(a.out);
  // the first pass of a split reads `in`; the second reads the intermediate in `out`
  if (d.kind == MANY_B) src = dst;

  // line addressing of the load
  int64_t ibase = 0, ielem = 1;
  bool ok = true;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    ibase = a.order_off[ok ? d.a + m : d.a];
  } else {
    const ManyXform x = a.xf[d.a];
    const int64_t N1 = (int64_t)1 << x.lg1, N2 = (int64_t)1 << (x.lg - x.lg1);
    const int64_t line = (int64_t)d.b * W + m;
    if (d.kind == MANY_A) {
      ok = line < N2;
      ibase = x.off + line;  // column n2 of x viewed as [N1][N2]
      ielem = N2;
    } else {
      ok = line < N1;
      ibase = x.off + line;  // column k1 of T viewed as [N2][N1]
      ielem = N1;
    }
  }
  const bool first = d.kind != MANY_B;
  const bool last = d.kind != MANY_A;
  float2 v[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    v[q] = ok ? load_c(src + ibase + (int64_t)(t + q * T) * ielem) : make_float2(0.f, 0.f);
    if (first && a.inverse) v[q].y = -v[q].y;
  }

  run_stages<L, P, W, 0>(v, lds, m, t, m_st, t_st, mfast_in != mfast_out, a.tw + a.stage_off[ilog2(L)]);

  // line addressing of the store (lane mapping may have changed)
  int64_t obase = 0, oelem = 1;
  float scale = 1.f;
  int64_t twl = 0;
  int lg1 = 0;
  uint32_t line_st = 0;
  ok = true;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    obase = a.order_off[ok ? d.a + m : d.a];
    scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)L : 1.f);
  } else {
    const ManyXform x = a.xf[d.a];
    const int64_t N1 = (int64_t)1 << x.lg1, N2 = (int64_t)1 << (x.lg - x.lg1);
    const int64_t line = (int64_t)d.b * W + m;
    line_st = (uint32_t)line;
    if (d.kind == MANY_A) {
      ok = line < N2;
      obase = x.off + line * N1;  // T[n2*N1 + k1]
      oelem = 1;
      twl = x.tw_lo;
      lg1 = x.lg1;
      // the default inverse scale 1/N is split as 1/N1 here and 1/N2 in the
      // second pass (exact, and keeps 16-bit intermediates in range)
      scale = (a.inverse && !a.use_scale) ? 1.f / (float)N1 : 1.f;
    } else {
      ok = line < N1;
      obase = x.off + line;  // X[k1 + N1*k2]
      oelem = N1;
      scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)N2 : 1.f);
    }
  }
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int e = t + q * T;
    float2 y = v[q];
    if (d.kind == MANY_A) {
      const uint32_t jj = line_st * (uint32_t)e;
      const float2* lo = a.tw + twl;
      const float2* hi = lo + ((int64_t)1 << lg1);
      y = cmul(y, cmul(hi[jj >> lg1], lo[jj & ((1u << lg1) - 1u)]));
    }
    y = cscale(y, scale);
    if (last && a.inverse) y.y = -y.y;
    if (ok) store_c(dst + obase + (int64_t)e * oelem, y);
  }
}

// Length-1 lines: NT transforms of one point each.
template <int NT, typename TS>
__device__ __forceinline__ void many_tile1(const ManyArgs& a, const ManyItem& d, int tid) {
  if (tid < d.b) {
    const int xid = a.order[d.a + tid];
    const int64_t off = a.xf[xid].off;
    float2 y = load_c(reinterpret_cast<const TS*>(a.in) + off);
    y = cscale(y, a.use_scale ? a.scale : 1.f);
    store_c(reinterpret_cast<TS*>(a.out) + off, y);
  }
}

template <typename TS, int P, int NT>
__global__ void __launch_bounds__(NT) k_many(ManyArgs a) {
  __shared__ float2 lds[many_lds_max<P, NT>()];
  __shared__ int s_item, s_last;
  const int tid = threadIdx.x;
  int* queue = a.ws;
  int* exits = a.ws + 1;
  int* watchdog = a.watchdog;
  int* done = a.ws + kManyWsHeader;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= a.n_items) break;  // uniform across the workgroup
    const ManyItem d = a.items[it];
    if (d.kind == MANY_B) {
      // Wait until every first-pass tile of this transform has released its
      // results.  The queue lists all of them before any second-pass tile of
      // the same transform, so they are held by running workgroups that wait
      // on nothing.  Polls are relaxed loads (no cache invalidation per
      // poll); one acquire follows the last poll.  The wait is bounded in
      // wall-clock time (100 MHz counter) and flags the watchdog word if the
      // bound is hit, so the kernel always finishes.
      if (tid == 0) {
        const int need = a.xf[d.a].nA;
        if (__hip_atomic_load(&done[d.a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          while (__hip_atomic_load(&done[d.a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            __builtin_amdgcn_s_sleep(8);
            if (__builtin_amdgcn_s_memrealtime() - t0 > (uint64_t)a.wait_ticks) {
              atomicOr(watchdog, 1);
              break;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
    switch (d.lg) {
      case 0: many_tile1<NT, TS>(a, d, tid); break;
      case 1: many_tile<2, P, NT, TS>(a, d, lds, tid); break;
      case 2: many_tile<4, P, NT, TS>(a, d, lds, tid); break;
      case 3: many_tile<8, P, NT, TS>(a, d, lds, tid); break;
      case 4: many_tile<16, P, NT, TS>(a, d, lds, tid); break;
      case 5: many_tile<32, P, NT, TS>(a, d, lds, tid); break;
      case 6: many_tile<64, P, NT, TS>(a, d, lds, tid); break;
      case 7: many_tile<128, P, NT, TS>(a, d, lds, tid); break;
      case 8: many_tile<256, P, NT, TS>(a, d, lds, tid); break;
      case 9: many_tile<512, P, NT, TS>(a, d, lds, tid); break;
      case 10: if constexpr (NT * P >= 1024) many_tile<1024, P, NT, TS>(a, d, lds, tid); break;
      case 11: if constexpr (NT * P >= 2048) many_tile<2048, P, NT, TS>(a, d, lds, tid); break;
      case 12: if constexpr (NT * P >= 4096) many_tile<4096, P, NT, TS>(a, d, lds, tid); break;
      default: break;
    }
    // the barrier orders every wave's stores of this tile before thread 0's
    // agent-scope release, which makes them visible to the other XCDs
    __syncthreads();
    if (d.kind == MANY_A && tid == 0)
      __hip_atomic_fetch_add(&done[d.a], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // The last workgroup out resets the queue state for the next launch.
  if (tid == 0) {
    const int fin = __hip_atomic_fetch_add(exits, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = fin == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    for (int i = tid; i < a.n_xforms; i += NT) done[i] = 0;
    if (tid == 0) {
      *queue = 0;
      *exits = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Software-pipelined variant: one workgroup per CU.  While a workgroup runs
// the butterflies of one item, the loads of its next item are in flight.
// Everything it reads between issuing those loads and consuming them comes
// from LDS: the stage twiddles of every tile length the plan uses are copied
// there at launch (vector-memory counters retire in order, so waiting on any
// later global load would also wait on the prefetch).
// ---------------------------------------------------------------------------

// LDS offset of the stage twiddles of a 2^LG tile (LG >= 1).
template <int P, int LG>
struct ManyTwOff {
  static constexpr int value = ManyTwOff<P, LG - 1>::value + TwLds<(1 << (LG - 1)), P>::SIZE;
};
template <int P>
struct ManyTwOff<P, 1> {
  static constexpr int value = 0;
};
template <int P, int MAXLG = kManyMaxLg>
constexpr int many_tw_total() { return ManyTwOff<P, MAXLG + 1>::value; }

template <int P, int LG>
void many_tw_map_lg(const int64_t* stage_off, int32_t tw_used, std::vector<int32_t>& map, int& len) {
  if constexpr (LG <= kManyMaxLg) {
    if ((tw_used >> LG) & 1) {
      using S = Sched<(1 << LG), P>;
      using TL = TwLds<(1 << LG), P>;
      const int base = ManyTwOff<P, LG>::value;
      for (int s = 1; s < S::S; ++s)
        for (int k = 0; k < S::ns(s); ++k)
          for (int r = 0; r < S::radix(s); ++r)
            map[base + TL::off(s) + k * TL::rp(s) + r] = (int32_t)(stage_off[LG] + S::off(s) + k * S::radix(s) + r);
      len = base + TL::SIZE;
    }
    many_tw_map_lg<P, LG + 1>(stage_off, tw_used, map, len);
  }
}

template <int P, int LG = 1>
int many_tw_prefix_of(int max_lg) {
  if constexpr (LG > kManyMaxLg) {
    return ManyTwOff<P, kManyMaxLg + 1>::value;
  } else {
    return max_lg < LG ? ManyTwOff<P, LG>::value : many_tw_prefix_of<P, LG + 1>(max_lg);
  }
}

int many_tw_image_prefix(int P, int max_lg) {
  if (P != 16) return 0;
  return many_tw_prefix_of<16>(max_lg);
}

int many_tw_image_map(const int64_t* stage_off, int32_t tw_used, int P, int max_lg,
                      std::vector<int32_t>* map) {
  if (P != 16) return 0;
  map->assign(max_lg >= 12 ? many_tw_total<16, 12>() : many_tw_total<16, 11>(), -1);
  int len = 0;
  many_tw_map_lg<16, 1>(stage_off, tw_used, *map, len);
  return len;
}

__global__ void k_gather_f2(float2* dst, const float2* src, const int32_t* map, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = map[i] >= 0 ? src[map[i]] : make_float2(0.f, 0.f);
}

hipError_t launch_gather_f2(float2* dst, const float2* src, const int32_t* map, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_f2, dim3((n + 255) / 256), dim3(256), 0, s, dst, src, map, n);
  return hipGetLastError();
}

// What the pipelined kernel loads ahead for one item: its points, the
// element offset of each lane's line (one-pass items), and for a split's
// first pass the inter-pass twiddle inputs: the lane's base W_N^{line*t}
// (lo/hi factors) and the tile's step rows W_N^{line*q*T} (W*PP entries,
// up to two per lane).
template <int P>
struct ManyPre {
  float2 v[P];
  float2 rown[2];
  float2 lon, hin;
  int64_t base;
};

template <int P, int NT>
__host__ __device__ constexpr bool many_step_rows(int lg) {
  // W*PP <= 2*NT, with PP = min(P, L), T = L/PP, W = NT/T
  return ((int64_t)NT << (2 * (lg < ilog2(P) ? lg : ilog2(P)))) >> lg <= 2 * NT;
}

// Issue the loads of item d (length 2^lg >= 2): the same lines and lane
// mapping as the compute step below uses, with runtime sizes.
template <int P, int NT, typename TS>
__device__ __forceinline__ void many_prefetch(const ManyArgs& a, const ManyItem& d, const ManyXform& x,
                                              ManyPre<P>& pre, int tid) {
  const int lg = d.lg;
  const int lpp = lg < ilog2(P) ? lg : ilog2(P);
  const int PP = 1 << lpp;
  const int lt = lg - lpp;                    // log2 T
  const int lw = ilog2(NT) - lt;              // log2 W
  const bool mfast = d.kind != MANY_SINGLE;
  const int m = mfast ? (tid & ((1 << lw) - 1)) : (tid >> lt);
  const int t = mfast ? (tid >> lw) : (tid & ((1 << lt) - 1));
  const TS* src = reinterpret_cast<const TS*>(d.kind == MANY_B ? a.out : a.in);
  int64_t ibase = 0, ielem = 1;
  bool ok = true;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    ibase = a.order_off[ok ? d.a + m : d.a];
    pre.base = ibase;
  } else {
    const int64_t line = ((int64_t)d.b << lw) + m;
    const int64_t n1 = (int64_t)1 << x.lg1, n2 = (int64_t)1 << (x.lg - x.lg1);
    ok = line < (d.kind == MANY_A ? n2 : n1);
    ibase = x.off + line;
    ielem = d.kind == MANY_A ? n2 : n1;
    if (d.kind == MANY_A && many_step_rows<P, NT>(lg)) {
      const int64_t line0 = (int64_t)d.b << lw;
      const int wpp = 1 << (lw + lpp);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int i = tid + k * NT;
        if (i < wpp) {
          const int64_t ln = line0 + (i >> lpp) < n2 ? line0 + (i >> lpp) : n2 - 1;
          pre.rown[k] = a.tw[x.tw_step + (ln << lpp) + (i & (PP - 1))];
        }
      }
      // the store mapping is point-fastest: line m_st = tid / T, point t_st = tid % T
      const int64_t lst = line0 + (tid >> lt);
      const uint32_t jb = (uint32_t)(lst < n2 ? lst : n2 - 1) * (uint32_t)(tid & ((1 << lt) - 1));
      pre.lon = a.tw[x.tw_lo + (jb & (uint32_t)(n1 - 1))];
      pre.hin = a.tw[x.tw_lo + n1 + (jb >> x.lg1)];
    }
  }
  const int64_t step = ielem << lt;
  const TS* p0 = src + ibase + (int64_t)t * ielem;
#pragma unroll
  for (int q = 0; q < P; ++q)
    if (q < PP) pre.v[q] = ok ? load_c(p0 + q * step) : make_float2(0.f, 0.f);
}

// Butterflies and store of one item whose points are in v.  `base` is the
// element offset of the lane's line for one-pass items; for a split's first
// pass with step rows, `tw_base` is the lane's W_N^{line*t} and rowl holds
// the tile's W_N^{line*q*T}.  `between` runs after the butterflies and
// before the stores (workgroup-uniform).
template <int L, int P, int NT, typename TS, typename F>
__device__ __forceinline__ void many_body(const ManyArgs& a, const ManyItem& d, float2* v, float2* xch,
                                          const float2* twl, const float2* rowl, float2 tw_base,
                                          int64_t base, int tid, F&& between) {
  using S = Sched<L, P>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  constexpr int W = NT / T;
  constexpr bool kRows = many_step_rows<P, NT>(ilog2(L));
  static_assert(W >= 1 && W * T == NT, "tile must fill the workgroup");
  const bool mfast_in = d.kind != MANY_SINGLE;
  const bool mfast_out = d.kind == MANY_B;
  int m = mfast_in ? tid % W : tid / T;
  int t = mfast_in ? tid / W : tid % T;
  const int m_st = mfast_out ? tid % W : tid / T;
  const int t_st = mfast_out ? tid / W : tid % T;
  const bool first = d.kind != MANY_B;
  const bool last = d.kind != MANY_A;
  const uint32_t sgn_in = (first && a.inverse) ? 0x80000000u : 0u;
#pragma unroll
  for (int q = 0; q < PP; ++q) v[q].y = __uint_as_float(__float_as_uint(v[q].y) ^ sgn_in);

  run_stages<L, P, W, 0, 1>(v, xch, m, t, m_st, t_st, mfast_in != mfast_out, twl);
  between();

  TS* dst = reinterpret_cast<TS*>(a.out);
  int64_t obase = 0, oelem = 1;
  float scale = 1.f;
  int64_t twl_off = 0;
  int lg1 = 0;
  uint32_t line_st = 0;
  bool ok = true;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    obase = base;
    scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)L : 1.f);
  } else {
    const ManyXform x = a.xf[d.a];
    const int64_t N1 = (int64_t)1 << x.lg1, N2 = (int64_t)1 << (x.lg - x.lg1);
    const int64_t line = (int64_t)d.b * W + m;
    line_st = (uint32_t)line;
    if (d.kind == MANY_A) {
      ok = line < N2;
      obase = x.off + line * N1;  // T[n2*N1 + k1]
      twl_off = x.tw_lo;
      lg1 = x.lg1;
      scale = (a.inverse && !a.use_scale) ? 1.f / (float)N1 : 1.f;
    } else {
      ok = line < N1;
      obase = x.off + line;  // X[k1 + N1*k2]
      oelem = N1;
      scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)N2 : 1.f);
    }
  }
  const uint32_t sgn_out = (last && a.inverse) ? 0x80000000u : 0u;
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int e = t + q * T;
    float2 y = v[q];
    if (d.kind == MANY_A) {
      if constexpr (kRows) {
        y = cmul(y, cmul(tw_base, rowl[m * PP + q]));
      } else {
        const uint32_t jj = line_st * (uint32_t)e;
        const float2* lo = a.tw + twl_off;
        const float2* hi = lo + ((int64_t)1 << lg1);
        y = cmul(y, cmul(hi[jj >> lg1], lo[jj & ((1u << lg1) - 1u)]));
      }
    }
    y = cscale(y, scale);
    y.y = __uint_as_float(__float_as_uint(y.y) ^ sgn_out);
    if (ok) store_c(dst + obase + (int64_t)e * oelem, y);
  }
}

// Items are taken in queue order, workgroup g taking items g, g + G, g + 2G
// (G resident workgroups): the tiles are of equal size, and the index and
// descriptors of the next item are known without a round trip to a shared
// counter (measured: a shared counter read two items ahead was slower).
// Forward progress: a workgroup runs its items in order, waits only for a
// second-pass item's first pass (earlier in the queue) and releases its own
// finished first-pass tiles before any wait, so the unfinished item of
// lowest index always has its dependencies released and is being run.
template <typename TS, int P, int NT, int MAXLG>
__global__ void __launch_bounds__(NT, 1) k_many_pipe(ManyArgs a) {
  static_assert(NT * P >= (1 << MAXLG), "every tile length runs the barriers of `between`");
  constexpr int XN = many_lds_max<P, NT, MAXLG>();
  constexpr int TWN = many_tw_total<P, MAXLG>();
  __shared__ float2 lds[XN + TWN + 2 * NT];
  __shared__ int s_ready, s_last;
  float2* xch = lds;
  float2* twl = lds + XN;
  float2* rowl = lds + XN + TWN;
  const int tid = threadIdx.x;
  int* exits = a.ws + 1;
  int* watchdog = a.watchdog;
  int* done = a.ws + kManyWsHeader;

  // Thread 0: bounded wait for transform x's first pass (same protocol as
  // k_many: relaxed polls, one acquire, watchdog flag on expiry).
  auto wait_released = [&](int x) {
    const int need = a.xf[x].nA;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(&done[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      __builtin_amdgcn_s_sleep(8);
      if (__builtin_amdgcn_s_memrealtime() - t0 > (uint64_t)a.wait_ticks) {
        atomicOr(watchdog, 1);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  };
  // Thread 0: whether item `it` can be loaded now (a second-pass item whose
  // first pass has released; acquire if so), 1 for other items.
  auto check = [&](int it) -> int {
    if (it >= a.n_items) return 1;
    const ManyItem di = a.items[it];
    if (di.kind != MANY_B) return 1;
    if (__hip_atomic_load(&done[di.a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < a.xf[di.a].nA) return 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return 1;
  };

  // stage twiddles: one contiguous copy of the plan's LDS image (all loads
  // issued before the first store)
  {
    constexpr int K = (TWN + NT - 1) / NT;
    float2 tmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (tid + k * NT < a.tw_img_len) tmp[k] = a.tw_img[tid + k * NT];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (tid + k * NT < a.tw_img_len) twl[tid + k * NT] = tmp[k];
  }

  const int G = (int)gridDim.x;
  int cur = (int)blockIdx.x;
  ManyItem d{};
  ManyPre<P> pre;
  pre.base = 0;
  if (cur < a.n_items) {
    d = a.items[cur];
    if (d.kind == MANY_B && tid == 0) wait_released(d.a);
  }
  __syncthreads();  // stage twiddles visible; thread 0's acquire before the loads
  if (cur < a.n_items && d.lg >= 1)
    many_prefetch<P, NT, TS>(a, d, d.kind != MANY_SINGLE ? a.xf[d.a] : ManyXform{}, pre, tid);
  int nxt = cur + G;
  if (tid == 0) s_ready = check(nxt);
  __syncthreads();
  int ready = s_ready;
  // descriptors of the next item, read one item ahead
  ManyItem dn{};
  ManyXform xn{};
  if (nxt < a.n_items) {
    dn = a.items[nxt];
    if (dn.kind != MANY_SINGLE) xn = a.xf[dn.a];
  }
  // An A tile's release waits for its stores; it is deferred to the next
  // item's barrier after the butterflies, by which time they have drained.
  int pending = -1;

  while (cur < a.n_items) {
    float2 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = pre.v[q];
    const int64_t base = pre.base;
    float2 tw_base = make_float2(1.f, 0.f);
    if (d.kind == MANY_A && d.lg >= 1 && many_step_rows<P, NT>(d.lg)) {
      lds_barrier();  // the previous tile's reads of the step rows are done
      const int lpp = d.lg < ilog2(P) ? d.lg : ilog2(P);
      const int wpp = (NT << (2 * lpp)) >> d.lg;  // W * PP <= 2 * NT
      rowl[tid] = pre.rown[0];
      if (tid + NT < wpp) rowl[tid + NT] = pre.rown[1];
      tw_base = cmul(pre.hin, pre.lon);
    }
    const bool has_next = nxt < a.n_items;
    if (has_next && !ready) {
      // checked two items ahead and not ready then: look again now, so that
      // its loads can still overlap this item's butterflies
      lds_barrier();  // every lane has read s_ready
      if (tid == 0) s_ready = check(nxt);
      __syncthreads();  // thread 0's acquire precedes every lane's loads
      ready = s_ready;
    }
    if (has_next && ready && dn.lg >= 1) many_prefetch<P, NT, TS>(a, dn, xn, pre, tid);
    const int nxt2 = nxt + G;
    ManyItem dn2{};
    ManyXform xn2{};
    if (nxt2 < a.n_items) {
      dn2 = a.items[nxt2];
      if (dn2.kind != MANY_SINGLE) xn2 = a.xf[dn2.a];
    }
    int ready2 = 1;
    // after the butterflies: release the previous A tile, look at the item
    // after next (thread 0 waits for its wave's memory operations first, this
    // prefetch included, which is the time the butterflies hide)
    auto between = [&]() {
      // the release needs every wave's stores of the previous tile ordered
      // before it (one barrier); the answer of a readiness check needs a
      // second one.  An item two ahead that is not a second-pass item is
      // ready: then no answer is broadcast (the condition is the same for
      // every lane)
      const bool look = has_next && nxt2 < a.n_items && dn2.kind == MANY_B;
      if (pending < 0 && !look) return;
      __syncthreads();
      if (tid == 0) {
        if (pending >= 0)
          __hip_atomic_fetch_add(&done[pending], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (look) s_ready = check(nxt2);
      }
      pending = -1;
      if (look) {
        __syncthreads();  // thread 0's acquire precedes every lane's later loads
        ready2 = s_ready;
      }
    };

    switch (d.lg) {
      case 0: between(); many_tile1<NT, TS>(a, d, tid); break;
      case 1: many_body<2, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 1>::value, rowl, tw_base, base, tid, between); break;
      case 2: many_body<4, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 2>::value, rowl, tw_base, base, tid, between); break;
      case 3: many_body<8, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 3>::value, rowl, tw_base, base, tid, between); break;
      case 4: many_body<16, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 4>::value, rowl, tw_base, base, tid, between); break;
      case 5: many_body<32, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 5>::value, rowl, tw_base, base, tid, between); break;
      case 6: many_body<64, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 6>::value, rowl, tw_base, base, tid, between); break;
      case 7: many_body<128, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 7>::value, rowl, tw_base, base, tid, between); break;
      case 8: many_body<256, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 8>::value, rowl, tw_base, base, tid, between); break;
      case 9: many_body<512, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 9>::value, rowl, tw_base, base, tid, between); break;
      case 10:
        if constexpr (MAXLG >= 10)
          many_body<1024, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 10>::value, rowl, tw_base, base, tid, between);
        else
          between();
        break;
      case 11:
        if constexpr (MAXLG >= 11)
          many_body<2048, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 11>::value, rowl, tw_base, base, tid, between);
        else
          between();
        break;
      case 12:
        if constexpr (MAXLG >= 12)
          many_body<4096, P, NT, TS>(a, d, v, xch, twl + ManyTwOff<P, 12>::value, rowl, tw_base, base, tid, between);
        else
          between();
        break;
      default: between(); break;
    }
    if (d.kind == MANY_A) pending = d.a;
    if (has_next && !ready) {
      // its first pass was still running at the check: release ours (it may
      // be one of them), wait, then load
      __syncthreads();
      if (tid == 0) {
        if (pending >= 0)
          __hip_atomic_fetch_add(&done[pending], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        wait_released(dn.a);
      }
      pending = -1;
      __syncthreads();
      if (dn.lg >= 1) many_prefetch<P, NT, TS>(a, dn, xn, pre, tid);
    }
    cur = nxt;
    d = dn;
    nxt = nxt2;
    dn = dn2;
    xn = xn2;
    ready = ready2;
  }
  if (pending >= 0) {
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&done[pending], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // The last workgroup out resets the queue state for the next launch.
  if (tid == 0) {
    const int fin = __hip_atomic_fetch_add(exits, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = fin == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    for (int i = tid; i < a.n_xforms; i += NT) done[i] = 0;
    if (tid == 0) {
      a.ws[0] = 0;
      *exits = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Two-launch pipelined kernel.  The passes of the split transforms are
// synchronised the way the paper synchronises its passes: by a kernel
// boundary (Sec. 2.3.3).  An exec queues two launches of the same persistent
// kernel: the first runs every first-pass tile and every one-pass tile, the
// second every second-pass tile.  Inside a launch no workgroup ever waits for
// another, so there are no counters, no device-wide fences and no bounded
// waits; items are claimed from the launch's atomic queue head, two ahead,
// so only running workgroups hold items and the tiles spread evenly however
// many workgroups are resident.  (Completion counters inside one launch need
// a device-scope release per first-pass tile, and each costs an L2
// write-back and a full memory wait on that CU: measured at about 10 us per
// release in a streaming kernel of this shape, which is what held the
// single-launch kernel above to a third of peak.)
// ---------------------------------------------------------------------------


// The per-lane loads of an item, issued ahead of its butterflies.
template <int P>
struct XPre {
  float2 v[P];
  float2 rown[2];
  float2 lon, hin;
};

// Issue the loads of item d (lg >= 1): data and, for a first pass, the
// inter-pass twiddle inputs.  `base` is the lane's line offset for one-pass
// items (loaded earlier).
template <int P, int NT, typename TS>
__device__ __forceinline__ void xprefetch(const ManyArgs& a, const ManyItemX& d, int64_t base, XPre<P>& pre,
                                          int tid) {
  const int lg = d.lg;
  const int lpp = lg < ilog2(P) ? lg : ilog2(P);
  const int lt = lg - lpp;            // log2 T
  const int lw = ilog2(NT) - lt;      // log2 W
  const int PP = 1 << lpp;
  const bool mfast = d.kind != MANY_SINGLE;
  const int m = mfast ? (tid & ((1 << lw) - 1)) : (tid >> lt);
  const int t = mfast ? (tid >> lw) : (tid & ((1 << lt) - 1));
  const TS* src = reinterpret_cast<const TS*>(d.kind == MANY_B ? a.out : a.in);
  // Every lane issues every load: lanes past the last line of a partial tile
  // read a valid line (the first of a one-pass tile, the last of a strip)
  // and are not stored.
  int64_t ibase, ielem = 1;
  if (d.kind == MANY_SINGLE) {
    ibase = base;
  } else {
    const int64_t n1 = (int64_t)1 << d.lg1, n2 = (int64_t)1 << (d.lgN - d.lg1);
    const int64_t nl = d.kind == MANY_A ? n2 : n1;
    const int64_t line = min(((int64_t)d.b << lw) + m, nl - 1);
    ibase = d.off + line;
    ielem = nl;
    if (d.kind == MANY_A && many_step_rows<P, NT>(lg)) {
      const int64_t line0 = (int64_t)d.b << lw;
      const int wpp = 1 << (lw + lpp);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int i = tid + k * NT;
        if (i < wpp) {
          const int64_t ln = line0 + (i >> lpp) < n2 ? line0 + (i >> lpp) : n2 - 1;
          pre.rown[k] = a.tw[d.tw_step + (ln << lpp) + (i & (PP - 1))];
        }
      }
      // the store mapping is point-fastest: line tid / T, point tid % T
      const int64_t lst = line0 + (tid >> lt);
      const uint32_t jb = (uint32_t)(lst < n2 ? lst : n2 - 1) * (uint32_t)(tid & ((1 << lt) - 1));
      pre.lon = a.tw[d.tw_lo + (jb & (uint32_t)(n1 - 1))];
      pre.hin = a.tw[d.tw_lo + n1 + (jb >> d.lg1)];
    }
  }
  const int64_t step = ielem << lt;
  const TS* p0 = src + ibase + (int64_t)t * ielem;
#pragma unroll
  for (int q = 0; q < P; ++q)
    if (q < PP) pre.v[q] = load_c(p0 + q * step);
}

// Stores with the nontemporal hint (streamed: the caches need not keep them).
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  f2v r;
  r.x = v.x;
  r.y = v.y;
  __builtin_nontemporal_store(r, reinterpret_cast<f2v*>(p));
}
__device__ __forceinline__ void store_nt(__half2* p, float2 v) {
  __builtin_nontemporal_store(pack_f16x2(v.x, v.y), reinterpret_cast<uint32_t*>(p));
}
__device__ __forceinline__ void store_nt(c16bf* p, float2 v) {
  const uint32_t w = pack_bf16x2(v.x, v.y);
  __builtin_nontemporal_store(w, reinterpret_cast<uint32_t*>(p));
}

// Butterflies and epilogue of one item (its points in v, outputs left in v
// in the store mapping, times the inter-pass twiddle and the scale,
// conjugated back for the inverse).
template <int L, int P, int NT>
__device__ __forceinline__ void xcompute(const ManyArgs& a, const ManyItemX& d, float2* v, float2* xch,
                                         const float2* twl, const float2* rowl, float2 tw_base, int tid) {
  using S = Sched<L, P>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  constexpr int W = NT / T;
  constexpr bool kRows = many_step_rows<P, NT>(ilog2(L));
  static_assert(W >= 1 && W * T == NT, "tile must fill the workgroup");
  const bool mfast_in = d.kind != MANY_SINGLE;
  const bool mfast_out = d.kind == MANY_B;
  int m = mfast_in ? tid % W : tid / T;
  int t = mfast_in ? tid / W : tid % T;
  const int m_st = mfast_out ? tid % W : tid / T;
  const int t_st = mfast_out ? tid / W : tid % T;
  const bool first = d.kind != MANY_B;
  const bool last = d.kind != MANY_A;
  const uint32_t sgn_in = (first && a.inverse) ? 0x80000000u : 0u;
#pragma unroll
  for (int q = 0; q < PP; ++q) v[q].y = __uint_as_float(__float_as_uint(v[q].y) ^ sgn_in);

  run_stages<L, P, W, 0, 1>(v, xch, m, t, m_st, t_st, mfast_in != mfast_out, twl);

  float scale;
  if (d.kind == MANY_SINGLE)
    scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)L : 1.f);
  else if (d.kind == MANY_A)
    scale = (a.inverse && !a.use_scale) ? 1.f / (float)(1 << d.lg1) : 1.f;
  else
    scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)(1 << (d.lgN - d.lg1)) : 1.f);
  const uint32_t sgn_out = (last && a.inverse) ? 0x80000000u : 0u;
  const uint32_t line_st = (uint32_t)(d.b * W + m);
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    float2 y = v[q];
    if (d.kind == MANY_A) {
      if constexpr (kRows) {
        y = cmul(y, cmul(tw_base, rowl[m * PP + q]));
      } else {
        const uint32_t jj = line_st * (uint32_t)(t + q * T);
        const float2* lo = a.tw + d.tw_lo;
        const float2* hi = lo + ((int64_t)1 << d.lg1);
        y = cmul(y, cmul(hi[jj >> d.lg1], lo[jj & ((1u << d.lg1) - 1u)]));
      }
    }
    y = cscale(y, scale);
    y.y = __uint_as_float(__float_as_uint(y.y) ^ sgn_out);
    v[q] = y;
  }
}

// Stores of an item whose outputs xcompute left in v.  `base` is the lane's
// line offset for one-pass items.
template <int L, int P, int NT, typename TS>
__device__ __forceinline__ void xstore(const ManyArgs& a, const ManyItemX& d, const float2* v, int64_t base,
                                       int tid) {
  using S = Sched<L, P>;
  constexpr int T = S::T;
  constexpr int PP = S::PP;
  constexpr int W = NT / T;
  const bool mfast_out = d.kind == MANY_B;
  const int m = mfast_out ? tid % W : tid / T;
  const int t = mfast_out ? tid / W : tid % T;
  TS* dst = reinterpret_cast<TS*>(a.out);
  int64_t obase, oelem = 1;
  bool ok;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    obase = base;
  } else {
    const int64_t N1 = (int64_t)1 << d.lg1, N2 = (int64_t)1 << (d.lgN - d.lg1);
    const int64_t line = (int64_t)d.b * W + m;
    if (d.kind == MANY_A) {
      ok = line < N2;
      obase = d.off + line * N1;  // T[n2*N1 + k1]
    } else {
      ok = line < N1;
      obase = d.off + line;  // X[k1 + N1*k2]
      oelem = N1;
    }
  }
  if (ok) {
    if (d.nt) {
#pragma unroll
      for (int q = 0; q < PP; ++q) store_nt(dst + obase + (int64_t)(t + q * T) * oelem, v[q]);
    } else {
#pragma unroll
      for (int q = 0; q < PP; ++q) store_c(dst + obase + (int64_t)(t + q * T) * oelem, v[q]);
    }
  }
}

// Descriptor of queue slot i, read with scalar loads (i is uniform).
__device__ __forceinline__ ManyItemX xitem(const ManyArgs& a, int i, int hi) {
  ManyItemX d{};
  d.kind = -1;
  d.lg = 0;
  if (i < hi) {
    // constant address space: uniform loads from it are scalar loads
    typedef const int32_t __attribute__((address_space(4)))* cptr;
    const cptr p = (cptr)(a.itx + __builtin_amdgcn_readfirstlane(i));
    int32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = p[k];
    __builtin_memcpy(&d, w, sizeof(d));
  }
  return d;
}

// Line offset of this lane's line in a one-pass item (lines past the tile's
// last read its first line).
template <int P>
__device__ __forceinline__ int64_t xbase(const ManyArgs& a, const ManyItemX& d, int tid) {
  const int lt = d.lg - (d.lg < ilog2(P) ? d.lg : ilog2(P));
  const int m = tid >> lt;
  return a.order_off[d.a + (m < d.b ? m : 0)];
}

#define MANY_XCD_SWITCH(LG, CALL)                          \
  switch (LG) {                                            \
    case 1: { constexpr int L = 2; CALL; } break;          \
    case 2: { constexpr int L = 4; CALL; } break;          \
    case 3: { constexpr int L = 8; CALL; } break;          \
    case 4: { constexpr int L = 16; CALL; } break;         \
    case 5: { constexpr int L = 32; CALL; } break;         \
    case 6: { constexpr int L = 64; CALL; } break;         \
    case 7: { constexpr int L = 128; CALL; } break;        \
    case 8: { constexpr int L = 256; CALL; } break;        \
    case 9: { constexpr int L = 512; CALL; } break;        \
    case 10: { constexpr int L = 1024; CALL; } break;      \
    case 11: { constexpr int L = 2048; CALL; } break;      \
    case 12: { constexpr int L = 4096; CALL; } break;      \
    default: break;                                        \
  }

// One loop iteration handles three items: it stores the results of the
// previous item p (left in registers), transforms the current item c (whose
// points were loaded during p) and issues the loads of the next item n.  So
// every vector-memory operation is issued about one item before anything
// waits for it, and the one full wait at the top of each iteration (for c's
// points) costs nothing even though it also covers p's stores, issued an
// iteration earlier: the pipelining does not depend on the compiler
// computing exact wait counts across the many item paths.
// Launch `a.phase` runs the items q_off[phase] .. q_off[phase+1]-1.
template <typename TS, int P, int NT, int MAXLG>
__global__ void __launch_bounds__(NT, 512 / NT) k_many_2l(ManyArgs a) {
  static_assert(NT * P >= (1 << MAXLG) && MAXLG <= 12, "tile lengths 2 .. 2^12");
  constexpr int XN = many_lds_max<P, NT, MAXLG>();
  constexpr int TWN = many_tw_total<P, MAXLG>();
  __shared__ float2 lds[XN + TWN + 2 * NT];
  __shared__ int s_idx[2], s_last;
  float2* xch = lds;
  float2* twl = lds + XN;
  float2* rowl = lds + XN + TWN;
  const int tid = threadIdx.x;
  int* heads = a.ws + kManyWsHeader + a.n_xforms;  // [phase]: queue head; [8 + phase]: exits
  const int ph = a.phase;
  const int lo = a.q_off[ph], hi = a.q_off[ph + 1];
  int* head = heads + ph;
  int* exits = heads + 8 + ph;
  constexpr int kNoClaim = 1 << 30;

  // The first two items are fixed: g and G + g for workgroup g of G.  Every
  // workgroup starts at once, and 2G claims on the one queue head at the
  // start would be served one after another (several microseconds for the
  // last in line); later claims come spread over the launch.  Claim k
  // (0-based) then names item 2G + k.
  const int G = (int)gridDim.x;
  // The first claim goes out before anything else: a claim issued behind
  // this workgroup's first loads can reach the queue head after other
  // workgroups' second claims, and then some get four items of a launch
  // whose items would go three to every workgroup.
  int claim = kNoClaim;  // thread 0: raw value of the claim in flight
  if (tid == 0) claim = atomicAdd(head, 1);
  int c = min(lo + (int)blockIdx.x, hi);
  int n = min(lo + G + (int)blockIdx.x, hi);
  ManyItemX dc = xitem(a, c, hi);
  ManyItemX dn = xitem(a, n, hi);
  int64_t base_c = 0, base_n = 0;
  if (c < hi && dc.kind == MANY_SINGLE) base_c = xbase<P>(a, dc, tid);

  // stage twiddles: the prefix of the plan's LDS image that this launch's
  // lengths read, loaded while the first item's loads are in flight (every
  // lane loads an entry; entries past the prefix are not written)
  constexpr int K = (TWN + NT - 1) / NT;
  const int img = min(a.tw_img_len, a.tw_img_len_ph[ph]);
  float2 tmp[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k * NT < img) tmp[k] = a.tw_img[min(tid + k * NT, img - 1)];
  XPre<P> pre;
  if (c < hi && dc.lg >= 1) xprefetch<P, NT, TS>(a, dc, base_c, pre, tid);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (tid + k * NT < img) twl[tid + k * NT] = tmp[k];
  // (the barrier at the top of the first iteration makes them visible)
  if (n < hi && dn.kind == MANY_SINGLE) base_n = xbase<P>(a, dn, tid);

  float2 v[P];
  ManyItemX dp{};
  dp.kind = -1;
  dp.lg = 0;
  int64_t base_p = 0;
  int par = 0;

  while (c < hi) {
    // ---- top: every memory operation issued by the previous iteration done
    vm_wait<0>();
    // stores of the previous item
    if (dp.kind >= 0) {
      MANY_XCD_SWITCH(dp.lg, (xstore<L, P, NT, TS>(a, dp, v, base_p, tid)));
    }
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = pre.v[k];
    float2 tw_base = make_float2(1.f, 0.f);
    if (dc.kind == MANY_A && dc.lg >= 1 && many_step_rows<P, NT>(dc.lg)) {
      const int lpp = dc.lg < ilog2(P) ? dc.lg : ilog2(P);
      const int wpp = (NT << (2 * lpp)) >> dc.lg;  // W * PP <= 2 * NT
      rowl[tid] = pre.rown[0];
      if (tid + NT < wpp) rowl[tid + NT] = pre.rown[1];
      tw_base = cmul(pre.hin, pre.lon);
    }
    // the index of the item after n
    if (tid == 0) s_idx[par] = min(lo + 2 * G + claim, hi);
    lds_barrier();  // also: step rows visible
    const int n2 = s_idx[par];
    par ^= 1;
    claim = kNoClaim;
    if (n2 < hi && tid == 0) claim = atomicAdd(head, 1);
    if (n < hi && dn.lg >= 1) xprefetch<P, NT, TS>(a, dn, base_n, pre, tid);
    const ManyItemX dn2 = xitem(a, n2, hi);

    // ---- the current item
    if (dc.lg == 0) {
      many_tile1<NT, TS>(a, ManyItem{dc.kind, dc.lg, dc.a, dc.b}, tid);
    } else {
      MANY_XCD_SWITCH(dc.lg, (xcompute<L, P, NT>(a, dc, v, xch, twl + ManyTwOff<P, (ilog2(L) > 0 ? ilog2(L) : 1)>::value, rowl, tw_base, tid)));
    }
    // line offsets of item n2 (one-pass items)
    int64_t base_n2 = 0;
    if (n2 < hi && dn2.kind == MANY_SINGLE) base_n2 = xbase<P>(a, dn2, tid);
    lds_barrier();  // LDS reads of this item done before the next one writes

    dp = dc;
    base_p = base_c;
    if (dc.lg == 0) dp.kind = -1;  // stored already
    c = n;
    dc = dn;
    base_c = base_n;
    n = n2;
    dn = dn2;
    base_n = base_n2;
  }
  // the last item's stores
  if (dp.kind >= 0) {
    MANY_XCD_SWITCH(dp.lg, (xstore<L, P, NT, TS>(a, dp, v, base_p, tid)));
  }
  // The last workgroup out resets this launch's queue head for the next exec.
  __syncthreads();
  if (tid == 0) {
    const int fin = __hip_atomic_fetch_add(exits, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = fin == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_last && tid == 0) {
    __hip_atomic_store(head, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(exits, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Both launches of an exec: first passes and one-pass tiles, then second
// passes (the second launch is skipped when no transform is split).
template <typename TS, int P, int NT, int MAXLG>
hipError_t launch_many_2l(const ManyArgs& a, int grid, hipStream_t s) {
  for (int ph = 0; ph < 2; ++ph) {
    ManyArgs b = a;
    b.phase = ph;
    if (ph == 1 && a.n_phase2 == 0) break;
    hipLaunchKernelGGL((k_many_2l<TS, P, NT, MAXLG>), dim3(grid), dim3(NT), 0, s, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS, int P, int NT, int MAXLG>
int blocks_many_2l() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_many_2l<TS, P, NT, MAXLG>, NT, 0) != hipSuccess) return 0;
  return n;
}

template <typename TS, int P, int NT, int MAXLG>
hipError_t launch_many_pipe(const ManyArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_many_pipe<TS, P, NT, MAXLG>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <typename TS, int P, int NT, int MAXLG>
int blocks_many_pipe() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_many_pipe<TS, P, NT, MAXLG>, NT, 0) != hipSuccess)
    return 0;
  return n;
}

template <typename TS, int P, int NT>
hipError_t launch_many(const ManyArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_many<TS, P, NT>), dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <typename TS, int P, int NT>
int blocks_many() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_many<TS, P, NT>, NT, 0) != hipSuccess) return 0;
  return n;
}

#define MANY_VARIANT(TS, DT, P, NT) \
  {DT, P, NT, 0, kManyMaxLg, &launch_many<TS, P, NT>, &blocks_many<TS, P, NT>}
// pipelined: 512 lanes (tiles up to 2^12) or 256 lanes (tiles up to 2^11,
// half the LDS; its registers still keep it to one workgroup per CU)
#define MANY_PIPE(TS, DT, P, NT, MAXLG) \
  {DT, P, NT, 1, MAXLG, &launch_many_pipe<TS, P, NT, MAXLG>, &blocks_many_pipe<TS, P, NT, MAXLG>}
// two launches (kernel boundary between the passes): 512 lanes, tiles up to 2^12
#define MANY_2L(TS, DT, P, NT, MAXLG) \
  {DT, P, NT, 2, MAXLG, &launch_many_2l<TS, P, NT, MAXLG>, &blocks_many_2l<TS, P, NT, MAXLG>}

static const ManyVariant kManyVariants[] = {
    MANY_VARIANT(float2, DT_C64, 16, 256),   MANY_VARIANT(float2, DT_C64, 8, 256),
    MANY_VARIANT(float2, DT_C64, 16, 512),   MANY_VARIANT(__half2, DT_C16F, 16, 256),
    MANY_VARIANT(__half2, DT_C16F, 8, 256),  MANY_VARIANT(c16bf, DT_C16BF, 16, 256),
    MANY_VARIANT(c16bf, DT_C16BF, 8, 256),   MANY_PIPE(float2, DT_C64, 16, 512, 12),
    MANY_PIPE(__half2, DT_C16F, 16, 512, 12),    MANY_PIPE(c16bf, DT_C16BF, 16, 512, 12),
    MANY_PIPE(float2, DT_C64, 16, 256, 11),      MANY_PIPE(__half2, DT_C16F, 16, 256, 11),
    MANY_PIPE(c16bf, DT_C16BF, 16, 256, 11),
    MANY_2L(float2, DT_C64, 16, 512, 12),        MANY_2L(__half2, DT_C16F, 16, 512, 12),
    MANY_2L(c16bf, DT_C16BF, 16, 512, 12),
    // 256 lanes, tiles up to 2^11: half the LDS, two workgroups per CU
    MANY_2L(float2, DT_C64, 16, 256, 11),        MANY_2L(__half2, DT_C16F, 16, 256, 11),
    MANY_2L(c16bf, DT_C16BF, 16, 256, 11),
};

int many_variant_count() { return (int)(sizeof(kManyVariants) / sizeof(kManyVariants[0])); }
const ManyVariant* many_variant(int i) {
  return (i >= 0 && i < many_variant_count()) ? &kManyVariants[i] : nullptr;
}

}  // namespace mfft
