// Persistent kernel for many transforms of uneven power-of-two lengths.
#include "fft_device.hpp"
#include "many.hpp"
#include "variants.hpp"

namespace mfft {

// LDS needed by a tile of length 2^lg: W = NT/T lines, padded layout.
template <int P, int NT>
__host__ __device__ constexpr int many_lds_len(int lg) {
  return lg == 0 ? NT
                 : (NT / ((1 << lg) / ((P < (1 << lg)) ? P : (1 << lg)))) *
                       ((1 << lg) + ((1 << lg) >> 4) + 1);
}
template <int P, int NT>
__host__ __device__ constexpr int many_lds_max(int lg = 0) {
  return lg > kManyMaxLg ? 0
                         : (many_lds_len<P, NT>(lg) > many_lds_max<P, NT>(lg + 1)
                                ? many_lds_len<P, NT>(lg)
                                : many_lds_max<P, NT>(lg + 1));
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
  int xid = d.a;
  if (d.kind == MANY_SINGLE) {
    ok = m < d.b;
    xid = ok ? a.order[d.a + m] : 0;
    ibase = a.xf[xid].off;
  } else {
    const ManyXform x = a.xf[xid];
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
    xid = ok ? a.order[d.a + m] : 0;
    obase = a.xf[xid].off;
    scale = a.use_scale ? a.scale : (a.inverse ? 1.f / (float)L : 1.f);
  } else {
    const ManyXform x = a.xf[xid];
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
  int* watchdog = a.ws + 2;
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

#define MANY_VARIANT(TS, DT, P, NT) {DT, P, NT, &launch_many<TS, P, NT>, &blocks_many<TS, P, NT>}

static const ManyVariant kManyVariants[] = {
    MANY_VARIANT(float2, DT_C64, 16, 256),   MANY_VARIANT(float2, DT_C64, 8, 256),
    MANY_VARIANT(float2, DT_C64, 16, 512),   MANY_VARIANT(__half2, DT_C16F, 16, 256),
    MANY_VARIANT(__half2, DT_C16F, 8, 256),  MANY_VARIANT(c16bf, DT_C16BF, 16, 256),
    MANY_VARIANT(c16bf, DT_C16BF, 8, 256),
};

int many_variant_count() { return (int)(sizeof(kManyVariants) / sizeof(kManyVariants[0])); }
const ManyVariant* many_variant(int i) {
  return (i >= 0 && i < many_variant_count()) ? &kManyVariants[i] : nullptr;
}

}  // namespace mfft
