// Deterministic sums of per-wave partial vectors (the MLP weight gradients):
// out[p] += sum over waves w of partial[w][p].  Stage 1: group g of
// kSumGroups adds waves g, g + kSumGroups, ... in that order into tmp[g][p];
// stage 2 adds the groups in order.  The order is fixed by the wave count, so
// repeated runs give the same bits, and the work is spread over
// kSumGroups x P threads instead of P.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace ngprt {

constexpr int kSumGroups = 64;

static __global__ void partial_group_sums_kernel(const float* __restrict__ partial, int64_t n_waves, int P,
                                                 float* __restrict__ tmp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (p >= P) return;
  float a = 0.0f;
  for (int64_t w = g; w < n_waves; w += kSumGroups) a += partial[w * P + p];
  tmp[int64_t(g) * P + p] = a;
}

static __global__ void partial_final_sums_kernel(const float* __restrict__ tmp, int P, float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float a = 0.0f;
  for (int g = 0; g < kSumGroups; ++g) a += tmp[int64_t(g) * P + p];
  out[p] += a;
}

// tmp: kSumGroups * P floats of workspace
static inline int launch_partial_sums(ngprt_ctx* ctx, const float* partial, int64_t n_waves, int P, float* tmp,
                                      float* out, hipStream_t st) {
  const unsigned bx = unsigned((P + 255) / 256);
  hipLaunchKernelGGL(partial_group_sums_kernel, dim3(bx, kSumGroups), dim3(256), 0, st, partial, n_waves, P, tmp);
  int rc = check_launch(ctx, "partial_group_sums_kernel");
  if (rc) return rc;
  hipLaunchKernelGGL(partial_final_sums_kernel, dim3(bx), dim3(256), 0, st, tmp, P, out);
  return check_launch(ctx, "partial_final_sums_kernel");
}

}  // namespace ngprt
