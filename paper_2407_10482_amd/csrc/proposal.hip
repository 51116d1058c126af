// Learned per-ray sample-interval proposal (an extension beyond the paper).
//
// Network: r = [o; d] -> Fourier features sin/cos(2^k pi r_j), k = 0..3 (48)
// -> 64 -> 64 -> 4 (ReLU hidden), outputs t_near, t_far, t_term and a
// confidence logit.  Parameters (float32 master, caller-owned, 7556 values):
// W1[64][48], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
//
// One wave owns 64 rays.  Every product is a 16x16 tile of
// v_mfma_f32_16x16x16_bf16 (bfloat16 operands, float32 accumulation): the
// layers as D = W X^T (K = input features), the backward as W^T G^T, and
// the weight gradients as G^T X with K = the wave's 64 rays.  Activations
// and gradients live in LDS feature-major ([feature][ray], bfloat16), so the
// weight-gradient operands are contiguous along K.  Per-wave gradient
// partials are summed by a second kernel in a fixed order; Adam then updates
// the float32 master copy.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "proposal_net.h"

namespace ngprt {

typedef float pf32x4 __attribute__((ext_vector_type(4)));
typedef short pbf16x4 __attribute__((ext_vector_type(4)));

constexpr int kPIn = 48, kPH = 64, kPOut = 4;
constexpr int kPW1 = 0, kPB1 = 3072, kPW2 = 3136, kPB2 = 7232, kPW3 = 7296, kPB3 = 7552;
constexpr int kPParams = 7556;
constexpr int kPPartial = kPParams + 1;          // + loss

struct PropLds {
  uint16_t enc[kPIn * 64];     // [feature][ray]
  uint16_t h1[kPH * 64];
  uint16_t h2[kPH * 64];
  float out[kPOut * 64];
  uint16_t gout[16 * 64];      // rows 4..15 zero
  uint16_t gz2[kPH * 64];
  uint16_t gz1[kPH * 64];
};

// D(16x16) += sum_kc A[i][16kc + k] B[16kc + k][j]; fa(i, k), fb(k, j) return bf16 bits.
template <class FA, class FB>
__device__ __forceinline__ pf32x4 mm_tile(int n_kc, FA fa, FB fb, int lane) {
  const int i = lane & 15, s = lane >> 4;
  pf32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < n_kc; ++kc) {
    pbf16x4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = kc * 16 + 4 * s + e;
      a[e] = (short)fa(i, k);
      b[e] = (short)fb(k, i);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// sum over the 16 lanes that share (lane >> 4)
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float sum64(float v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Forward of the wave's 64 rays into L.out (float32 outputs before the sigmoid).
__device__ __forceinline__ void prop_forward(PropLds& L, const float* __restrict__ P,
                                             const uint16_t* __restrict__ Wb, const float* o,
                                             const float* d, bool in_range, int lane) {
  // Fourier features of this lane's ray
  float r[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    r[j] = in_range ? o[j] : 0.0f;
    r[3 + j] = in_range ? d[j] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float a = float(1 << k) * r[j];
      L.enc[(8 * j + 2 * k) * 64 + lane] = bf16_rne(sinpif(a));
      L.enc[(8 * j + 2 * k + 1) * 64 + lane] = bf16_rne(cospif(a));
    }
  }
  __syncthreads();
  const int s = lane >> 4, col = lane & 15;
  // layer 1: h1 = relu(W1 enc + b1)
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt) {
      pf32x4 acc = mm_tile(
          3, [&](int i, int k) { return Wb[kPW1 + (mt * 16 + i) * kPIn + k]; },
          [&](int k, int j) { return L.enc[k * 64 + nt * 16 + j]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = mt * 16 + 4 * s + q;
        L.h1[row * 64 + nt * 16 + col] = bf16_rne(fmaxf(acc[q] + P[kPB1 + row], 0.0f));
      }
    }
  __syncthreads();
  // layer 2
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt) {
      pf32x4 acc = mm_tile(
          4, [&](int i, int k) { return Wb[kPW2 + (mt * 16 + i) * kPH + k]; },
          [&](int k, int j) { return L.h1[k * 64 + nt * 16 + j]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = mt * 16 + 4 * s + q;
        L.h2[row * 64 + nt * 16 + col] = bf16_rne(fmaxf(acc[q] + P[kPB2 + row], 0.0f));
      }
    }
  __syncthreads();
  // layer 3 (4 outputs, rows 4..15 of the tile zero)
  for (int nt = 0; nt < 4; ++nt) {
    pf32x4 acc = mm_tile(
        4, [&](int i, int k) { return i < kPOut ? Wb[kPW3 + i * kPH + k] : (uint16_t)0; },
        [&](int k, int j) { return L.h2[k * 64 + nt * 16 + j]; }, lane);
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) L.out[q * 64 + nt * 16 + col] = acc[q] + P[kPB3 + q];
    }
  }
  __syncthreads();
}

// Float32 master weights -> the A-operand tiles and biases of
// prop_infer_wave (proposal_net.h): 32 tiles x 64 lanes of four bfloat16,
// then b1, b2, b3 as float32.
__global__ void prop_arrange_kernel(const float* __restrict__ P, uint2* __restrict__ tiles,
                                    float* __restrict__ bias) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kPropTiles * 64) {
    const int tile = t >> 6, lane = t & 63;
    const int i = lane & 15, k0 = 4 * (lane >> 4);
    int base, row, col, ld;
    bool zero = false;
    if (tile < 12) {             // layer 1: W1[64][48]
      base = kPW1; ld = kPIn; row = 16 * (tile / 3) + i; col = 16 * (tile % 3) + k0;
    } else if (tile < 28) {      // layer 2: W2[64][64]
      const int q = tile - 12;
      base = kPW2; ld = kPH; row = 16 * (q / 4) + i; col = 16 * (q % 4) + k0;
    } else {                     // layer 3: W3[4][64], rows 4..15 zero
      base = kPW3; ld = kPH; row = i; col = 16 * (tile - 28) + k0;
      zero = i >= kPOut;
    }
    uint16_t h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = zero ? (uint16_t)0 : bf16_rne(P[base + (zero ? 0 : row) * ld + col + e]);
    tiles[t] = make_uint2(uint32_t(h[0]) | (uint32_t(h[1]) << 16), uint32_t(h[2]) | (uint32_t(h[3]) << 16));
  }
  if (t < kPropBias) bias[t] = t < 64 ? P[kPB1 + t] : (t < 128 ? P[kPB2 + t - 64] : P[kPB3 + t - 128]);
}

// Stand-alone inference: four waves per workgroup, one wave per 64 rays.
__global__ void __launch_bounds__(256) prop_infer_kernel(int64_t n, const float* __restrict__ O,
                                                         const float* __restrict__ D,
                                                         const uint2* __restrict__ tiles,
                                                         const float* __restrict__ bias,
                                                         float* __restrict__ out) {
  __shared__ float out4_all[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ray_base = (int64_t(blockIdx.x) * 4 + wave) * 64;
  prop_infer_wave(tiles, bias, O, D, ray_base, n, lane, out4_all[wave]);
  __syncthreads();
  const int64_t ray = ray_base + lane;
  if (ray < n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) out[ray * 4 + c] = out4_all[wave][4 * lane + c];
  }
}

// Labels [n][4]: t_near, t_far, t_term, valid (1/0).  phase 1: pinball
// losses on t_near (quantile 0.05) and t_far (0.95), squared error on t_term;
// phase >= 2: + confidence cross-entropy with target = valid and
// [out0 - margin, out1 + margin] contains [t_near, t_far].  Loss terms are
// divided by n (the batch).
__global__ void __launch_bounds__(64) prop_train_kernel(int64_t n, const float* __restrict__ O,
                                                        const float* __restrict__ D,
                                                        const float* __restrict__ labels,
                                                        int phase, float margin,
                                                        const float* __restrict__ P,
                                                        const uint16_t* __restrict__ Wb,
                                                        float* __restrict__ partial) {
  __shared__ PropLds L;
  const int lane = threadIdx.x;
  const int64_t ray = int64_t(blockIdx.x) * 64 + lane;
  const bool in_range = ray < n;
  prop_forward(L, P, Wb, O + 3 * (in_range ? ray : 0), D + 3 * (in_range ? ray : 0), in_range, lane);
  const int s = lane >> 4, col = lane & 15;
  float* part = partial + int64_t(blockIdx.x) * kPPartial;
  const float inv_n = 1.0f / float(n);

  // loss and dL/dout for this lane's ray
  float go[4] = {0.f, 0.f, 0.f, 0.f};
  float loss = 0.0f;
  if (in_range) {
    const float* y = labels + ray * 4;
    const bool valid = y[3] != 0.0f;
    float ov[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) ov[c] = L.out[c * 64 + lane];
    if (valid) {
      // t_near: pinball loss at quantile 0.05; t_far: at 0.95; t_term: squared error
      const float r0 = y[0] - ov[0], r1 = y[1] - ov[1], df = ov[2] - y[2];
      loss += (r0 >= 0.0f ? 0.05f * r0 : -0.95f * r0) + (r1 >= 0.0f ? 0.95f * r1 : -0.05f * r1) + df * df;
      go[0] = (ov[0] > y[0] ? 0.95f : -0.05f) * inv_n;
      go[1] = (ov[1] > y[1] ? 0.05f : -0.95f) * inv_n;
      go[2] = 2.0f * df * inv_n;
    }
    if (phase >= 2) {
      const float tgt = (valid && ov[0] - margin <= y[0] && ov[1] + margin >= y[1]) ? 1.0f : 0.0f;
      const float sg = 1.0f / (1.0f + __expf(-ov[3]));
      loss += -(tgt * __logf(sg + 1e-12f) + (1.0f - tgt) * __logf(1.0f - sg + 1e-12f));
      go[3] = (sg - tgt) * inv_n;
    }
  }
  loss = sum64(loss * inv_n);
#pragma unroll
  for (int c = 0; c < 16; ++c) L.gout[c * 64 + lane] = c < 4 ? bf16_rne(go[c < 4 ? c : 0]) : (uint16_t)0;
  {
    float b3[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) b3[c] = sum64(go[c]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) part[kPB3 + c] = b3[c];
      part[kPParams] = loss;
    }
  }
  __syncthreads();
  // gz2 = (W3^T gout) * [h2 > 0]
  for (int mt = 0; mt < 4; ++mt) {
    float bsum[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nt = 0; nt < 4; ++nt) {
      pf32x4 acc = mm_tile(
          1, [&](int i, int k) { return k < kPOut ? Wb[kPW3 + k * kPH + mt * 16 + i] : (uint16_t)0; },
          [&](int k, int j) { return L.gout[k * 64 + nt * 16 + j]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = mt * 16 + 4 * s + q, rc = nt * 16 + col;
        const float g = bf16_to_f32(L.h2[row * 64 + rc]) > 0.0f ? acc[q] : 0.0f;
        L.gz2[row * 64 + rc] = bf16_rne(g);
        bsum[q] += g;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float t = sum16(bsum[q]);
      if (col == 0) part[kPB2 + mt * 16 + 4 * s + q] = t;
    }
  }
  __syncthreads();
  // gz1 = (W2^T gz2) * [h1 > 0]
  for (int mt = 0; mt < 4; ++mt) {
    float bsum[4] = {0.f, 0.f, 0.f, 0.f};
    for (int nt = 0; nt < 4; ++nt) {
      pf32x4 acc = mm_tile(
          4, [&](int i, int k) { return Wb[kPW2 + k * kPH + mt * 16 + i]; },
          [&](int k, int j) { return L.gz2[k * 64 + nt * 16 + j]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = mt * 16 + 4 * s + q, rc = nt * 16 + col;
        const float g = bf16_to_f32(L.h1[row * 64 + rc]) > 0.0f ? acc[q] : 0.0f;
        L.gz1[row * 64 + rc] = bf16_rne(g);
        bsum[q] += g;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float t = sum16(bsum[q]);
      if (col == 0) part[kPB1 + mt * 16 + 4 * s + q] = t;
    }
  }
  __syncthreads();
  // weight gradients, K = the wave's rays
  for (int nt = 0; nt < 4; ++nt) {          // dW3[4][64]
    pf32x4 acc = mm_tile(
        4, [&](int i, int k) { return L.gout[i * 64 + k]; },
        [&](int k, int j) { return L.h2[(nt * 16 + j) * 64 + k]; }, lane);
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) part[kPW3 + q * kPH + nt * 16 + col] = acc[q];
    }
  }
  for (int mt = 0; mt < 4; ++mt)             // dW2[64][64]
    for (int nt = 0; nt < 4; ++nt) {
      pf32x4 acc = mm_tile(
          4, [&](int i, int k) { return L.gz2[(mt * 16 + i) * 64 + k]; },
          [&](int k, int j) { return L.h1[(nt * 16 + j) * 64 + k]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) part[kPW2 + (mt * 16 + 4 * s + q) * kPH + nt * 16 + col] = acc[q];
    }
  for (int mt = 0; mt < 4; ++mt)             // dW1[64][48]
    for (int nt = 0; nt < 3; ++nt) {
      pf32x4 acc = mm_tile(
          4, [&](int i, int k) { return L.gz1[(mt * 16 + i) * 64 + k]; },
          [&](int k, int j) { return L.enc[(nt * 16 + j) * 64 + k]; }, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) part[kPW1 + (mt * 16 + 4 * s + q) * kPIn + nt * 16 + col] = acc[q];
    }
}

__global__ void prop_reduce_kernel(const float* __restrict__ partial, int64_t n_waves,
                                   float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kPPartial) return;
  float a = 0.0f;
  for (int64_t w = 0; w < n_waves; ++w) a += partial[w * kPPartial + p];
  if (p < kPParams) grad[p] = a;
  else if (loss) loss[0] += a;
}

__global__ void prop_cast_kernel(const float* __restrict__ P, uint16_t* __restrict__ Wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kPParams) Wb[p] = bf16_rne(P[p]);
}

static int ensure_prop_buffers(ngprt_ctx* ctx, int64_t n_waves, hipStream_t st) {
  // each buffer on its own, so that a failed call leaves nothing half made
  if ((!ctx->prop_wb &&
       dev_malloc_async((void**)&ctx->prop_wb, kPParams * sizeof(uint16_t), st) != hipSuccess) ||
      (!ctx->prop_grad && dev_malloc_async((void**)&ctx->prop_grad, kPParams * sizeof(float), st) != hipSuccess)) {
    (void)hipGetLastError();
    return fail(ctx, NGPRT_E_ALLOC, "proposal buffers");
  }
  const size_t need = size_t(n_waves) * kPPartial * sizeof(float);
  if (need > ctx->ws_bytes) {
    if (ctx->ws) (void)hipFreeAsync(ctx->ws, st);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (dev_malloc_async((void**)&ctx->ws, need, st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_ALLOC, "proposal workspace");
    }
    ctx->ws_bytes = need;
  }
  return NGPRT_OK;
}

constexpr size_t kPropNetBytes = size_t(kPropTiles) * 64 * sizeof(uint2) + kPropBias * sizeof(float);

// dst: kPropNetBytes of device memory (tiles, then biases)
int launch_prop_arrange(ngprt_ctx* ctx, const float* P, void* dst, hipStream_t st) {
  uint2* tiles = reinterpret_cast<uint2*>(dst);
  float* bias = reinterpret_cast<float*>(reinterpret_cast<char*>(dst) + size_t(kPropTiles) * 64 * sizeof(uint2));
  hipLaunchKernelGGL(prop_arrange_kernel, dim3((kPropTiles * 64 + 255) / 256), dim3(256), 0, st, P, tiles, bias);
  return check_launch(ctx, "prop_arrange_kernel");
}

int launch_prop_infer(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* P, float* out,
                      hipStream_t st) {
  if (!ctx->prop_tmp && dev_malloc((void**)&ctx->prop_tmp, kPropNetBytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->prop_tmp = nullptr;
    return fail(ctx, NGPRT_E_ALLOC, "proposal inference weights");
  }
  int rc = launch_prop_arrange(ctx, P, ctx->prop_tmp, st);
  if (rc) return rc;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays");
  const uint2* tiles = reinterpret_cast<const uint2*>(ctx->prop_tmp);
  const float* bias = reinterpret_cast<const float*>(reinterpret_cast<const char*>(ctx->prop_tmp) +
                                                     size_t(kPropTiles) * 64 * sizeof(uint2));
  hipLaunchKernelGGL(prop_infer_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, n, o, d, tiles, bias, out);
  return check_launch(ctx, "prop_infer_kernel");
}

int load_proposal(ngprt_ctx* ctx, const float* P, hipStream_t st) {
  if (!ctx->prop_net && dev_malloc((void**)&ctx->prop_net, kPropNetBytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->prop_net = nullptr;
    return fail(ctx, NGPRT_E_ALLOC, "proposal network");
  }
  int rc = launch_prop_arrange(ctx, P, ctx->prop_net, st);
  if (rc) return rc;
  ctx->prop_loaded = true;
  return NGPRT_OK;
}

int launch_prop_train(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* labels,
                      int phase, float margin, float* P, float* m, float* v, int32_t step, float lr,
                      float* loss, float* grad_out, hipStream_t st) {
  const int64_t blocks = (n + 63) / 64;
  if (blocks > (int64_t(1) << 24)) return fail(ctx, NGPRT_E_SHAPE, "batch too large");
  int rc = ensure_prop_buffers(ctx, blocks, st);
  if (rc) return rc;
  hipLaunchKernelGGL(prop_cast_kernel, dim3((kPParams + 255) / 256), dim3(256), 0, st, P,
                     (uint16_t*)ctx->prop_wb);
  if ((rc = check_launch(ctx, "prop_cast_kernel"))) return rc;
  float* partial = reinterpret_cast<float*>(ctx->ws);
  hipLaunchKernelGGL(prop_train_kernel, dim3(unsigned(blocks)), dim3(64), 0, st, n, o, d, labels, phase,
                     margin, P, (const uint16_t*)ctx->prop_wb, partial);
  if ((rc = check_launch(ctx, "prop_train_kernel"))) return rc;
  float* grad = grad_out ? grad_out : reinterpret_cast<float*>(ctx->prop_grad);
  hipLaunchKernelGGL(prop_reduce_kernel, dim3((kPPartial + 255) / 256), dim3(256), 0, st, partial, blocks,
                     grad, loss);
  if ((rc = check_launch(ctx, "prop_reduce_kernel"))) return rc;
  if (m && v) {
    rc = launch_adam(kPParams, P, grad, m, v, step, lr, 0.9f, 0.99f, 1e-8f, st);
    if (rc) return fail(ctx, rc, "adam");
  }
  return NGPRT_OK;
}

}  // namespace ngprt
