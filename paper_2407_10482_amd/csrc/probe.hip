// Random-gather probe: the gather ceiling of this device for the scene's own
// table layout.  Each lane stands for one sample: per level it gathers eight
// feature rows and logits at pseudo-random entries of that level (all eight
// independent, or four random entries each with its x-neighbour e ^ 1, which
// is how the spatial hash places the two x-adjacent corners of a cell when
// the cell's x index is even), dequantises them as the render does and
// writes their sum, so no load can be dropped.  Requested bytes per sample
// are L * 8 * (row + logit bytes), the same figure as a render sample.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace ngprt {

// 32-bit integer mixer (xor-shift / multiply finaliser)
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

template <int DT>
__global__ void __launch_bounds__(256) gather_probe_kernel(SceneArgs S, int64_t n, uint32_t seed,
                                                           int pairs, float* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t key = mix32(uint32_t(p) ^ mix32(seed ^ uint32_t(p >> 32)));
  float acc = 0.0f;
  for (int l = 0; l < S.L; ++l) {
    const void* fb = feat_level<DT>(S.feat, l, S.log2T);
    const void* lb = logit_level<DT>(S.logit, l, S.log2T);
    uint32_t idx[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t r = mix32(key + uint32_t(l * 8 + (pairs ? (k >> 1) : k)) * 0x9E3779B9u) & S.mask;
      idx[k] = pairs ? (r ^ uint32_t(k & 1)) : r;
    }
    float ch[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) ch[j] = 0.0f;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      float v[4][8], lg[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Store<DT>::feat(fb, idx[4 * g + k], v[k]);
        lg[k] = Store<DT>::logit(lb, idx[4 * g + k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ch[8] += lg[k];
#pragma unroll
        for (int j = 0; j < 8; ++j) ch[j] += v[k][j];
      }
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) acc += (DT == DT_FP8 ? S.scale[l][j] * ch[j] : ch[j]);
  }
  out[p] = acc;
}

int launch_gather_probe(ngprt_ctx* ctx, int64_t n, uint32_t seed, int pairs, float* out, hipStream_t s) {
  const SceneArgs S = scene_args(ctx);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > int64_t(0x7FFFFFFF)) return fail(ctx, NGPRT_E_SHAPE, "too many points for one launch");
  dim3 g = dim3(unsigned(blocks)), b = dim3(256);
  switch (ctx->desc.table_dtype) {
    case DT_F32: hipLaunchKernelGGL(gather_probe_kernel<DT_F32>, g, b, 0, s, S, n, seed, pairs, out); break;
    case DT_BF16: hipLaunchKernelGGL(gather_probe_kernel<DT_BF16>, g, b, 0, s, S, n, seed, pairs, out); break;
    case DT_FP8: hipLaunchKernelGGL(gather_probe_kernel<DT_FP8>, g, b, 0, s, S, n, seed, pairs, out); break;
    default: return fail(ctx, NGPRT_E_DTYPE, "unknown table dtype");
  }
  return check_launch(ctx, "gather_probe_kernel");
}

}  // namespace ngprt
