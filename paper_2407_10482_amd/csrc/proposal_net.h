// Inference of the per-ray sample-interval proposal network by one wave for
// its 64 rays (an extension beyond the paper), shared by the render kernel's
// prologue and the stand-alone inference kernel.
//
// Network: r = [o; d] -> Fourier features sin/cos(2^k pi r_j), k = 0..3
// (feature 8j + 2k = sin, 8j + 2k + 1 = cos; 48) -> 64 -> 64 -> 4 with ReLU
// hidden layers; outputs t_near, t_far, t_term and a confidence logit.
//
// Every product is v_mfma_f32_16x16x16_bf16 (bfloat16 operands, float32
// accumulation), computed as D = W X^T with the hidden units as rows and 16
// rays as columns.  Lane l holds A[l % 16][4 (l / 16) + e], B[4 (l / 16) + e][l % 16]
// (e = 0..3) and receives D[4 (l / 16) + r][l % 16] (r = 0..3), so a layer's
// output tile (16 hidden units x 16 rays), after bias, ReLU and rounding to
// bfloat16, is already the next layer's B operand for the K-chunk of those 16
// units: activations never leave registers.  The weights come pre-arranged
// as A operands (PropTiles), one 8-byte load per lane per tile, read through
// the cache (16 KB for the whole network).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace ngprt {

typedef float pn_f32x4 __attribute__((ext_vector_type(4)));
typedef short pn_bf16x4 __attribute__((ext_vector_type(4)));

// A-operand tiles: layer 1 (m, kc) at m * 3 + kc (m = 0..3 rows of 16
// hidden units, kc = 0..2 chunks of 16 inputs); layer 2 at 12 + m * 4 + kc;
// layer 3 at 28 + kc (rows 4..15 zero).  Tile t, lane l: W[16 m + l % 16][16 kc
// + 4 (l / 16) + e], e = 0..3, as four bfloat16 (round to nearest even).
constexpr int kPropTiles = 32;
constexpr int kPropBias = 132;     // b1[64], b2[64], b3[4] (float32)

__device__ __forceinline__ pn_bf16x4 pn_tile(const uint2* __restrict__ w, int tile, int lane) {
  const uint2 q = w[tile * 64 + lane];
  pn_bf16x4 a;
  a[0] = (short)(q.x & 0xFFFFu);
  a[1] = (short)(q.x >> 16);
  a[2] = (short)(q.y & 0xFFFFu);
  a[3] = (short)(q.y >> 16);
  return a;
}

__device__ __forceinline__ pn_bf16x4 pn_pack(float a, float b, float c, float d) {
  pn_bf16x4 v;
  v[0] = (short)bf16_rne(a);
  v[1] = (short)bf16_rne(b);
  v[2] = (short)bf16_rne(c);
  v[3] = (short)bf16_rne(d);
  return v;
}

// out4: this wave's LDS slab of at least 256 floats.  On return (after the
// caller's barrier) out4[4 i + c] holds output c of ray ray_base + i, the
// confidence already through the sigmoid.  Rays at or beyond n encode a zero
// input.  Every lane of the wave must call this.
__device__ __forceinline__ void prop_infer_wave(const uint2* __restrict__ w, const float* __restrict__ bias,
                                                const float* __restrict__ O, const float* __restrict__ D,
                                                int64_t ray_base, int64_t n, int lane, float* out4) {
  const int j = lane & 15, s = lane >> 4;
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    // the weight loads are the same for every ray tile; an opaque copy of the
    // pointer keeps the compiler from hoisting all 32 of them (64 registers)
    // out of this loop
    const uint2* wt = w;
    asm volatile("" : "+s"(wt));
    const int64_t ray = ray_base + 16 * t + j;
    const bool ok = ray < n;
    // K-chunk kc of the encoding holds features 16 kc + 4 s + e: input
    // component 2 kc + s / 2, frequencies 2 (s % 2) and 2 (s % 2) + 1
    pn_bf16x4 benc[3];
#pragma unroll
    for (int kc = 0; kc < 3; ++kc) {
      const int comp = 2 * kc + (s >> 1);
      const float* src = comp < 3 ? O : D;
      const float r = ok ? src[3 * (ok ? ray : 0) + (comp < 3 ? comp : comp - 3)] : 0.0f;
      const int k0 = 2 * (s & 1);
      const float a0 = float(1 << k0) * r, a1 = float(2 << k0) * r;
      benc[kc] = pn_pack(sinpif(a0), cospif(a0), sinpif(a1), cospif(a1));
    }
    pn_bf16x4 h1[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      pn_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < 3; ++kc)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pn_tile(wt, m * 3 + kc, lane), benc[kc], acc, 0, 0, 0);
      const float* b = bias + 16 * m + 4 * s;
      h1[m] = pn_pack(fmaxf(acc[0] + b[0], 0.0f), fmaxf(acc[1] + b[1], 0.0f), fmaxf(acc[2] + b[2], 0.0f),
                      fmaxf(acc[3] + b[3], 0.0f));
    }
    pn_bf16x4 h2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      pn_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pn_tile(wt, 12 + m * 4 + kc, lane), h1[kc], acc, 0, 0, 0);
      const float* b = bias + 64 + 16 * m + 4 * s;
      h2[m] = pn_pack(fmaxf(acc[0] + b[0], 0.0f), fmaxf(acc[1] + b[1], 0.0f), fmaxf(acc[2] + b[2], 0.0f),
                      fmaxf(acc[3] + b[3], 0.0f));
    }
    pn_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pn_tile(wt, 28 + kc, lane), h2[kc], acc, 0, 0, 0);
    if (s == 0) {
      float* dst = out4 + 4 * (16 * t + j);
      dst[0] = acc[0] + bias[128];
      dst[1] = acc[1] + bias[129];
      dst[2] = acc[2] + bias[130];
      dst[3] = 1.0f / (1.0f + __expf(-(acc[3] + bias[131])));
    }
  }
}

}  // namespace ngprt
