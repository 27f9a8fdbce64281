// Batched transforms of uneven power-of-two lengths in one persistent launch.
//
// The paper synchronises its passes with kernel boundaries ("we call the
// kernel function three times to make sure synchronization when we use
// global memory", Sec. 2.3.3).  Here one launch of resident workgroups pulls
// work items from a device queue instead; the boundary between the two passes
// of a split transform becomes a per-transform completion counter that the
// first-pass tiles release and the second-pass tiles acquire.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace mfft {

enum ManyKind { MANY_SINGLE = 0, MANY_A = 1, MANY_B = 2 };

// One work item = one workgroup-sized tile.
//   MANY_SINGLE: b lines of length 2^lg; line m is transform order[a + m]
//   MANY_A:      first pass of transform a, tile b (columns b*W .. b*W+W-1)
//   MANY_B:      second pass of transform a, tile b
struct ManyItem {
  int32_t kind, lg, a, b;
};

// One transform: length 2^lg at element offset `off` of the packed buffer;
// split transforms use N1 = 2^lg1 (first pass) and N2 = 2^(lg - lg1), have
// nA first-pass tiles, and read the inter-pass tables at tw_lo (2^lg1
// entries W_N^j) and tw_lo + 2^lg1 (2^(lg-lg1) entries W_N^{j*N1}).
struct ManyXform {
  int64_t off;
  int64_t tw_lo;
  int64_t tw_step;  // [N2][P] entries W_N^{n2*q*(N1/P)} (first pass of a split, N1 >= P)
  int32_t lg, lg1, nA, pad;
};

constexpr int kManyMaxLg = 12;  // longest single-tile length: 2^12 points

// Work item of the two-launch kernel: everything its loads, butterflies and
// stores need, so that one scalar load per item fetches it.
struct ManyItemX {
  int32_t kind, lg;  // MANY_*; log2 of the tile's line length
  int32_t a;         // transform (first/second pass) or first order slot (one pass)
  int32_t b;         // tile (first/second pass) or lines in the tile (one pass)
  int64_t off;       // element offset of the transform (first/second pass)
  int64_t tw_lo;     // first pass: W_N^j tables (lo at tw_lo, hi at tw_lo + N1)
  int64_t tw_step;   // first pass: step rows W_N^{n2*q*(N1/P)}
  int32_t lg1, lgN;  // log2 N1 and log2 N (first/second pass)
  int32_t nt;        // stores with the nontemporal hint
  int32_t pad[3];
};
static_assert(sizeof(ManyItemX) == 64, "one 64-byte record per item");

constexpr int kManyMaxQueues = 16;  // ints after the counters: queue heads and exit counts

struct ManyArgs {
  const void* in;
  void* out;
  const ManyItem* items;
  const ManyXform* xf;
  const int32_t* order;
  const int64_t* order_off;           // element offset of transform order[i]
  const float2* tw;                   // base of the plan's tables
  int64_t stage_off[kManyMaxLg + 1];  // stage table of a 2^lg tile
  int32_t n_items, n_xforms;
  int32_t* ws;                        // workspace (layout above kManyWsHeader)
  float scale;                        // used when use_scale != 0
  int32_t use_scale;                  // 0: per-transform default (1 or 1/N)
  int32_t inverse;
  int64_t wait_ticks;  // bound of one dependency wait, 100 MHz ticks
  int32_t tw_used;     // bit lg set: the plan has 2^lg tiles (stage table present)
  // pipelined kernel: the stage twiddles of every used length, laid out as
  // the kernel keeps them in LDS (copied there contiguously at launch)
  const float2* tw_img;
  int32_t tw_img_len;
  // two-launch kernel: items in launch order, launch p running items
  // q_off[p] .. q_off[p+1]-1 (p = phase: 0 first passes and one-pass tiles,
  // 1 second passes); n_phase2 = q_off[2] - q_off[1]
  const ManyItemX* itx;
  const int32_t* q_off;
  int32_t phase, n_phase2;
  int32_t tw_img_len_ph[2];  // two-launch kernel: image entries each launch's lengths need
  int32_t* watchdog;  // flag set when a bounded wait expires
};

// Workspace: [0] queue head (shared-queue kernel), [1] exits, [2] watchdog,
// [3] unused, then one completion counter per transform, then
// kManyMaxQueues ints for the two-launch kernel (queue head of launch p at
// [p], its exit count at [8 + p]).
constexpr int kManyWsHeader = 4;  // ints before the per-transform counters

struct ManyVariant {
  int dtype, P, threads;
  int pipe;    // 1: software-pipelined; 2: software-pipelined, two launches per exec
  int max_lg;  // longest one-tile length, 2^max_lg
  hipError_t (*launch)(const ManyArgs&, int grid, hipStream_t);
  int (*max_blocks_per_cu)();
};

// LDS image of the pipelined kernel's stage twiddles (P points per lane):
// entry i holds table element map[i] (an index into the plan's twiddle
// table), or nothing (-1: row padding, unused lengths).  Returns the number
// of entries the kernel copies (up to the longest used length).
int many_tw_image_map(const int64_t* stage_off, int32_t tw_used, int P, int max_lg,
                      std::vector<int32_t>* map);
hipError_t launch_gather_f2(float2* dst, const float2* src, const int32_t* map, int n, hipStream_t s);
// Entries of the pipelined kernels' stage-twiddle image (P points per lane)
// that tiles of length up to 2^max_lg read: the image holds the lengths in
// increasing order, so this is a prefix.
int many_tw_image_prefix(int P, int max_lg);

// Compiled persistent-kernel variants (storage type x points per lane x
// workgroup size).
int many_variant_count();
const ManyVariant* many_variant(int i);

// Host-side plan state (owned by fft_plan_s).
struct ManyPlan {
  bool active = false;
  const ManyVariant* var = nullptr;
  ManyItem* d_items = nullptr;
  ManyItemX* d_itx = nullptr;
  int32_t* d_q_off = nullptr;
  ManyXform* d_xf = nullptr;
  int32_t* d_order = nullptr;
  int64_t* d_order_off = nullptr;
  float2* d_tw = nullptr;
  float2* d_tw_img = nullptr;
  ManyArgs args{};
  int64_t count = 0, n_items = 0;
  int64_t points = 0, pass_points = 0, packed_bytes = 0;
  double flops = 0;
  int grid = 0;
  int dtype = 0;
  bool has_split = false;
  bool gpu_twiddles = false;
};

size_t many_workspace_bytes(const ManyPlan& mp);
int many_alloc_workspace(const ManyPlan& mp, void** ws, size_t* bytes);
hipError_t many_reset_workspace(const ManyPlan& mp, void* ws);
// `watchdog`: the flag word bounded waits set (NULL: the one in `ws`).
hipError_t many_launch(const ManyPlan& mp, const void* in, void* out, void* ws, int32_t* watchdog,
                       float scale, bool use_scale, bool inverse, hipStream_t s);
void many_free(ManyPlan& mp);

}  // namespace mfft
