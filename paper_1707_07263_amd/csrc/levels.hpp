// One global-memory radix-2 kernel per butterfly level (the method of
// Sec. 2.2 that the LDS-resident passes replace), for the ablation plans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfft {

struct LevelsArgs {
  const void* in;
  void* out;
  void* buf;          // batch * N elements, plan-owned ping-pong buffer
  int64_t batch;
  int lgN;            // >= 1
  int dtype;          // 0 complex64, 1 fp16 pairs, 2 bf16 pairs
  const float2* tw;   // W_N^m, m < N/2
  float scale;        // caller's scale, applied by the last level
  bool user_scale;    // false: 1 forward, 1/2 per level inverse (1/N in all)
  bool inverse;
  int cus;
};

hipError_t launch_levels(const LevelsArgs& a, hipStream_t st);

}  // namespace mfft
