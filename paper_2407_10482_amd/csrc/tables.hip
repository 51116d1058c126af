// Hash-table ingest: float32 [L][T][9] -> library layout in the storage dtype.
//
// Library layout: features [L][T][8] (32 B / 16 B / 8 B rows for F32 / BF16 /
// FP8, aligned so one row is one vector load) and logits [L][T].
// BF16: round-to-nearest-even of the float32 pattern (NaN -> 0x7FC0).
// FP8: OCP E4M3FN with one float32 scale per (level, channel):
// s = amax / 448 (1 when amax = 0), code = RNE-saturate(x / s); the encoder
// below is written from the format definition (bias 7, 3 mantissa bits,
// subnormal step 2^-9, largest finite 448, no infinities).
#include <hip/hip_runtime.h>

#include <cstring>

#include "device.h"
#include "internal.h"

namespace ngprt {

__device__ __forceinline__ uint8_t fp8_encode(float x) {
  if (x != x) return 0x7F;
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  uint32_t code;
  if (a >= 448.0f) {
    code = 0x7E;
  } else if (a < 0.015625f) {                     // below 2^-6: subnormal step 2^-9
    code = uint32_t(rintf(a * 512.0f));           // 8 -> 0x08, the smallest normal
  } else {
    int e = int((__float_as_uint(a) >> 23) & 0xFFu) - 127;          // -6 .. 8
    float y = a * __uint_as_float(uint32_t(127 - e) << 23);          // a / 2^e in [1, 2)
    uint32_t m = uint32_t(rintf((y - 1.0f) * 8.0f));
    if (m == 8) { m = 0; ++e; }
    code = (uint32_t(e + 7) << 3) | m;
    if (code > 0x7E) code = 0x7E;
  }
  return uint8_t(code | sign);
}

__global__ void split_f32_kernel(const float* __restrict__ src, float* __restrict__ feat,
                                 float* __restrict__ logit, int64_t n_entries) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_entries) return;
  const float* s = src + i * 9;
  for (int j = 0; j < 8; ++j) feat[i * 8 + j] = s[j];
  logit[i] = s[8];
}

__global__ void split_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ feat,
                                  uint16_t* __restrict__ logit, int64_t n_entries) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_entries) return;
  const float* s = src + i * 9;
  for (int j = 0; j < 8; ++j) feat[i * 8 + j] = bf16_rne(s[j]);
  logit[i] = bf16_rne(s[8]);
}

// amax[l][c] as the bit pattern of a non-negative float (ordered like uint32)
__global__ void amax_kernel(const float* __restrict__ src, uint32_t* __restrict__ amax, int64_t T,
                            int L) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  __shared__ uint32_t part[9];
  const int l = int(blockIdx.y);
  if (threadIdx.x < 9) part[threadIdx.x] = 0;
  __syncthreads();
  if (i < T) {
    const float* s = src + (int64_t(l) * T + i) * 9;
    for (int c = 0; c < 9; ++c) {
      float a = fabsf(s[c]);
      if (a == a) atomicMax(&part[c], __float_as_uint(a));
    }
  }
  __syncthreads();
  if (threadIdx.x < 9) atomicMax(&amax[l * 9 + threadIdx.x], part[threadIdx.x]);
}

struct Scales9 {
  float s[kMaxLevels][9] = {};
};

__global__ void split_fp8_kernel(const float* __restrict__ src, uint8_t* __restrict__ feat,
                                 uint8_t* __restrict__ logit, int64_t T, Scales9 sc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int l = int(blockIdx.y);
  if (i >= T) return;
  const int64_t e = int64_t(l) * T + i;
  const float* s = src + e * 9;
  for (int j = 0; j < 8; ++j) feat[e * 8 + j] = fp8_encode(s[j] / sc.s[l][j]);
  logit[e] = fp8_encode(s[8] / sc.s[l][8]);
}

template <typename Tv>
__global__ void join_kernel(const Tv* __restrict__ feat, const Tv* __restrict__ logit, Tv* __restrict__ dst,
                            int64_t n_entries) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_entries) return;
  for (int j = 0; j < 8; ++j) dst[i * 9 + j] = feat[i * 8 + j];
  dst[i * 9 + 8] = logit[i];
}

int launch_load_tables(ngprt_ctx* ctx, const float* src, hipStream_t st) {
  const int L = ctx->desc.n_levels;
  const int64_t T = ctx->T;
  const int64_t n = int64_t(L) * T;
  const unsigned nb = unsigned((n + 255) / 256);
  for (int l = 0; l < kMaxLevels; ++l)
    for (int c = 0; c < 9; ++c) ctx->scales_host[l][c] = 1.0f;
  switch (ctx->desc.table_dtype) {
    case DT_F32: {
      hipLaunchKernelGGL(split_f32_kernel, dim3(nb), dim3(256), 0, st, src, (float*)ctx->feat,
                         (float*)ctx->logit, n);
      return check_launch(ctx, "split_f32_kernel");
    }
    case DT_BF16: {
      hipLaunchKernelGGL(split_bf16_kernel, dim3(nb), dim3(256), 0, st, src, (uint16_t*)ctx->feat,
                         (uint16_t*)ctx->logit, n);
      return check_launch(ctx, "split_bf16_kernel");
    }
    case DT_FP8: {
      uint32_t* amax = reinterpret_cast<uint32_t*>(ctx->scales_dev);
      if (hipMemsetAsync(amax, 0, sizeof(uint32_t) * L * 9, st) != hipSuccess)
        return check_launch(ctx, "hipMemsetAsync");
      dim3 g(unsigned((T + 255) / 256), unsigned(L));
      hipLaunchKernelGGL(amax_kernel, g, dim3(256), 0, st, src, amax, T, L);
      int rc = check_launch(ctx, "amax_kernel");
      if (rc) return rc;
      uint32_t host_amax[kMaxLevels * 9];
      if (hipMemcpyAsync(host_amax, amax, sizeof(uint32_t) * L * 9, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return check_launch(ctx, "amax readback");
      Scales9 sc;
      for (int l = 0; l < kMaxLevels; ++l)
        for (int c = 0; c < 9; ++c) sc.s[l][c] = 1.0f;
      for (int l = 0; l < L; ++l)
        for (int c = 0; c < 9; ++c) {
          float a;
          std::memcpy(&a, &host_amax[l * 9 + c], 4);
          float s = a / 448.0f;
          sc.s[l][c] = (a == 0.0f) ? 1.0f : s;
          ctx->scales_host[l][c] = sc.s[l][c];
        }
      // keep the scales on the device as floats (for export)
      if (hipMemcpyAsync(ctx->scales_dev, &ctx->scales_host[0][0], sizeof(float) * L * 9,
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return check_launch(ctx, "scale upload");
      hipLaunchKernelGGL(split_fp8_kernel, g, dim3(256), 0, st, src, (uint8_t*)ctx->feat,
                         (uint8_t*)ctx->logit, T, sc);
      rc = check_launch(ctx, "split_fp8_kernel");
      if (rc) return rc;
      // the host copy of the scales must outlive the async upload
      if (hipStreamSynchronize(st) != hipSuccess) return check_launch(ctx, "scale upload");
      return NGPRT_OK;
    }
    default:
      return fail(ctx, NGPRT_E_DTYPE, "unknown table dtype");
  }
}

int launch_export_tables(ngprt_ctx* ctx, void* codes, float* scales, hipStream_t st) {
  const int64_t n = int64_t(ctx->desc.n_levels) * ctx->T;
  const unsigned nb = unsigned((n + 255) / 256);
  switch (ctx->desc.table_dtype) {
    case DT_F32:
      hipLaunchKernelGGL(join_kernel<float>, dim3(nb), dim3(256), 0, st, (const float*)ctx->feat,
                         (const float*)ctx->logit, (float*)codes, n);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(join_kernel<uint16_t>, dim3(nb), dim3(256), 0, st, (const uint16_t*)ctx->feat,
                         (const uint16_t*)ctx->logit, (uint16_t*)codes, n);
      break;
    default:
      hipLaunchKernelGGL(join_kernel<uint8_t>, dim3(nb), dim3(256), 0, st, (const uint8_t*)ctx->feat,
                         (const uint8_t*)ctx->logit, (uint8_t*)codes, n);
      break;
  }
  int rc = check_launch(ctx, "join_kernel");
  if (rc) return rc;
  if (scales) {
    if (hipMemcpyAsync(scales, ctx->scales_dev, sizeof(float) * ctx->desc.n_levels * 9,
                       hipMemcpyDeviceToDevice, st) != hipSuccess)
      return check_launch(ctx, "scale export");
  }
  return NGPRT_OK;
}

// Baked model: coarse atlas [n_blocks][512][C] float32 -> rows of Cpad
// floats (zero padded) so a row is whole float4 loads.
__global__ void pack_atlas_kernel(const float* __restrict__ src, float* __restrict__ dst, int64_t rows,
                                  int C, int Cpad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * Cpad) return;
  const int64_t r = i / Cpad;
  const int c = int(i - r * Cpad);
  dst[i] = c < C ? src[r * C + c] : 0.0f;
}

int launch_pack_atlas(ngprt_ctx* ctx, const float* atlas, int64_t n_blocks, hipStream_t st) {
  const int C = coarse_channels(ctx->desc), Cpad = coarse_row_floats(C);
  const int64_t total = n_blocks * 512 * Cpad;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "atlas too large");
  hipLaunchKernelGGL(pack_atlas_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, atlas, ctx->catlas,
                     n_blocks * 512, C, Cpad);
  return check_launch(ctx, "pack_atlas_kernel");
}

}  // namespace ngprt
