// View-dependent deferred MLP (Eq. 5; supplement "Network Design"):
// C = sigmoid(C_d + MLP_psi(C_d, F, SH(d))), MLP_psi 23 -> 64 -> 64 -> 3 with
// ReLU hidden layers, SH(d) the 16 real spherical harmonics of degrees 0..3
// of the normalised view direction.
//
// A separate pass after the march: the render kernel leaves C_d and F in the
// caller's output buffers, and this kernel runs the MLP over all rays.  One
// workgroup = 16 waves sharing one copy of the weights, pre-arranged at load
// time in the order the MFMA sequence consumes them (one 64-float record per
// instruction, lane l reading element l), staged once per workgroup in LDS
// (35 KB of weights + 6 KB of inputs per wave: 131 KB, one workgroup and
// four waves per SIMD on a CU); the grid holds only as many workgroups as
// stay resident together, each taking groups of 1024 rays in turn.  Per wave
// the 64 rays are 4 column blocks of 16; every layer is a
// chain of v_mfma_f32_16x16x4f32 with the hidden units as rows and the rays
// as columns; the hidden index handed to the next layer is permuted (k-slot
// s of chunk (m, r) = unit 16 m + 4 s + r) so each layer consumes the
// previous accumulators in place.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "reduce.h"

namespace ngprt {

typedef float f32x4v __attribute__((ext_vector_type(4)));

// MFMA operand records: layer 1 (4 output blocks x 6 K-chunks), layer 2
// (4 output blocks x 16 chunks), layer 3 (16 chunks), then the biases laid
// out per lane: b0 [4 blocks][64 lanes][4], b1 likewise, b2 [64 lanes][4].
constexpr int kL1Rec = 4 * 6, kL2Rec = 4 * 16, kL3Rec = 16;
constexpr int kViewRecFloats = (kL1Rec + kL2Rec + kL3Rec) * 64 + (4 + 4 + 1) * 64 * 4;   // 8960
static_assert(kViewRecFloats == kMlpViewRec, "record size");

// Rearrange the flattened parameters W0[64][23], b0[64], W1[64][64], b1[64],
// W2[3][64], b2[3] into the MFMA records (one thread per record float).
__global__ void view_mlp_arrange_kernel(const float* __restrict__ P, float* __restrict__ rec) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kViewRecFloats) return;
  const float* W0 = P;
  const float* b0 = W0 + 64 * 23;
  const float* W1 = b0 + 64;
  const float* b1 = W1 + 64 * 64;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 3 * 64;
  const int lane = t & 63, i = lane & 15, s = lane >> 4;
  int rix = t >> 6;
  float v = 0.0f;
  if (rix < kL1Rec) {                                    // layer 1: (mo, c)
    const int mo = rix / 6, c = rix % 6, k = 4 * c + s;
    v = k < 23 ? W0[(mo * 16 + i) * 23 + k] : 0.0f;
  } else if ((rix -= kL1Rec) < kL2Rec) {                 // layer 2: (mo, m, r)
    const int mo = rix / 16, m = (rix / 4) % 4, r = rix % 4;
    v = W1[(mo * 16 + i) * 64 + m * 16 + 4 * s + r];
  } else if ((rix -= kL2Rec) < kL3Rec) {                 // layer 3: (m, r)
    const int m = rix / 4, r = rix % 4;
    v = i < 3 ? W2[i * 64 + m * 16 + 4 * s + r] : 0.0f;
  } else {                                               // biases per lane
    const int b = t - (kL1Rec + kL2Rec + kL3Rec) * 64;   // [9][64][4]
    const int blk = b / 256, ln = (b / 4) % 64, r = b % 4, unit = 4 * (ln >> 4) + r;
    if (blk < 4) v = b0[blk * 16 + unit];
    else if (blk < 8) v = b1[(blk - 4) * 16 + unit];
    else v = unit < 3 ? b2[unit] : 0.0f;
  }
  rec[t] = v;
}

__device__ __forceinline__ void sh16(float x, float y, float z, float* Y) {
  // real spherical harmonics, degrees 0..3 (orthonormal, no Condon-Shortley phase)
  const float c0 = 0.28209479177387814f;                 // 1/2 sqrt(1/pi)
  const float c1 = 0.4886025119029199f;                  // sqrt(3/(4 pi))
  const float c2a = 1.0925484305920792f;                 // 1/2 sqrt(15/pi)
  const float c2b = 0.31539156525252005f;                // 1/4 sqrt(5/pi)
  const float c2c = 0.5462742152960396f;                 // 1/4 sqrt(15/pi)
  const float c3a = 0.5900435899266435f;                 // 1/4 sqrt(35/(2 pi))
  const float c3b = 2.890611442640554f;                  // 1/2 sqrt(105/pi)
  const float c3c = 0.4570457994644658f;                 // 1/4 sqrt(21/(2 pi))
  const float c3d = 0.3731763325901154f;                 // 1/4 sqrt(7/pi)
  const float c3e = 1.445305721320277f;                  // 1/4 sqrt(105/pi)
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = c0;
  Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
  Y[4] = c2a * x * y; Y[5] = c2a * y * z; Y[6] = c2b * (3.0f * zz - 1.0f);
  Y[7] = c2a * x * z; Y[8] = c2c * (xx - yy);
  Y[9] = c3a * y * (3.0f * xx - yy); Y[10] = c3b * x * y * z; Y[11] = c3c * y * (5.0f * zz - 1.0f);
  Y[12] = c3d * z * (5.0f * zz - 3.0f); Y[13] = c3c * x * (5.0f * zz - 1.0f);
  Y[14] = c3e * z * (xx - yy); Y[15] = c3a * x * (xx - 3.0f * yy);
}

constexpr int kViewWaves = 16;                    // waves per workgroup of view_mlp_kernel

__global__ void __launch_bounds__(64 * kViewWaves) view_mlp_kernel(int64_t n, const float* __restrict__ D,
                                                       const float* __restrict__ c_d,
                                                       const float* __restrict__ feat,
                                                       const float* __restrict__ rec,
                                                       float* __restrict__ rgb) {
  __shared__ float W[kViewRecFloats];
  __shared__ float xin_all[kViewWaves][24 * 64];
  for (int t = threadIdx.x; t < kViewRecFloats; t += 64 * kViewWaves) W[t] = rec[t];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* xin = xin_all[wave];
  const int i = lane & 15, s = lane >> 4;
  const float* R1 = W;
  const float* R2 = W + kL1Rec * 64;
  const float* R3 = R2 + kL2Rec * 64;
  const float* B = R3 + kL3Rec * 64;
  const int64_t groups = (n + 64 * kViewWaves - 1) / (64 * kViewWaves);
  // the group loop is uniform across the workgroup, so its barriers are too
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
  const int64_t ray_base = (g * kViewWaves + wave) * 64;
  const int64_t ray = ray_base + lane;
  float x[24];
#pragma unroll
  for (int j = 0; j < 24; ++j) x[j] = 0.0f;
  if (ray < n) {
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] = c_d[ray * 3 + j];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[3 + j] = feat[ray * 4 + j];
    float d0 = D[ray * 3], d1 = D[ray * 3 + 1], d2 = D[ray * 3 + 2];
    const float nn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
    if (nn > 0.0f && isfinite(nn)) sh16(d0 / nn, d1 / nn, d2 / nn, x + 7);
  }
  // every wave has read the previous group's inputs (and, the first time,
  // the weights are in place) before the slabs are written again
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 24; ++j) xin[j * 64 + lane] = x[j];
  __syncthreads();
  for (int rb = 0; rb < 4; ++rb) {
    const int col = rb * 16 + i;
    float h1[4][4], h2[4][4];
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      f32x4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int c = 0; c < 6; ++c)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(R1[(mo * 6 + c) * 64 + lane], xin[(4 * c + s) * 64 + col],
                                                   acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[mo][r] = fmaxf(acc[r] + B[(mo * 64 + lane) * 4 + r], 0.0f);
    }
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      f32x4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(R2[((mo * 4 + m) * 4 + r) * 64 + lane], h1[m][r], acc, 0,
                                                     0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[mo][r] = fmaxf(acc[r] + B[((4 + mo) * 64 + lane) * 4 + r], 0.0f);
    }
    f32x4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(R3[(m * 4 + r) * 64 + lane], h2[m][r], acc, 0, 0, 0);
    if (s == 0) {
      const int64_t gr = ray_base + col;
      if (gr < n) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const float z = xin[j * 64 + col] + (acc[j] + B[(8 * 64 + lane) * 4 + j]);
          rgb[gr * 3 + j] = 1.0f / (1.0f + __expf(-z));
        }
      }
    }
  }
  }
}

// ---------------------------------------------------------------------------
// Backward of the view-dependent MLP (a training extension).  One wave =
// one workgroup = 64 rays, a lane per ray; the weights come from the
// flattened parameters by uniform (scalar) loads.  Per lane: the forward
// again (activation rows a1, a2 in LDS, ReLU masks as bits), gz = dL/drgb
// * rgb (1 - rgb), g2 = (W2^T gz) masked, g1 = (W1^T g2) masked, each
// gradient row written over the activation rows whose last reader is done
// (g2 over a2 after dW2, g1 over a1 after dW1: two 64-row buffers, 45 KB of
// LDS per wave, three waves per CU),
// dL/dC_d = gz + (W0^T g1)[0..2], dL/dF = (W0^T g1)[3..6].  The weight
// gradients are sums over the wave's rays of outer products, taken on
// v_mfma_f32_16x16x4f32 with the rays as K, and written as one 5891-float
// partial per wave; the partials are then added in a fixed order (reduce.h).
constexpr int kVP = 65;                                  // LDS row pitch (bank spread)
constexpr int kW0 = 0, kB0 = 64 * 23, kW1 = kB0 + 64, kB1 = kW1 + 64 * 64, kW2 = kB1 + 64,
              kB2 = kW2 + 3 * 64;
static_assert(kB2 + 3 == kMlpViewParams, "parameter layout");

// D[ia + i][jb + j] = sum over the wave's 64 rays r of A[r][ia + i] * B[r][jb + j]
// (i, j < 16); lane l gets D[ia + 4 (l / 16) + q][jb + l % 16], q = 0..3.
__device__ __forceinline__ f32x4v outer16(const float* A, int pa, int ia, const float* B, int pb, int jb,
                                          int lane) {
  const int i = lane & 15, s = lane >> 4;
  f32x4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int r = 4 * c + s;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r * pa + ia + i], B[r * pb + jb + i], acc, 0, 0, 0);
  }
  return acc;
}

__global__ void __launch_bounds__(64) view_mlp_backward_kernel(int64_t n, const float* __restrict__ D,
                                                               const float* __restrict__ c_d,
                                                               const float* __restrict__ feat,
                                                               const float* __restrict__ grad_rgb,
                                                               const float* __restrict__ P,
                                                               float* __restrict__ grad_cf,
                                                               float* __restrict__ partial) {
  __shared__ float sA[64 * kVP];       // a1, then g1
  __shared__ float sB[64 * kVP];       // a2, then g2
  __shared__ float sX[64 * 32];        // x (23 used, zero padded)
  __shared__ float sG[64 * 16];        // gz (3 used, zero padded)
  const int lane = threadIdx.x;
  const int64_t ray = int64_t(blockIdx.x) * 64 + lane;
  const bool ok = ray < n;
  float x[23];
#pragma unroll
  for (int j = 0; j < 23; ++j) x[j] = 0.0f;
  float g[3] = {0.0f, 0.0f, 0.0f};
  if (ok) {
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] = c_d[ray * 3 + j];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[3 + j] = feat[ray * 4 + j];
    const float d0 = D[ray * 3], d1 = D[ray * 3 + 1], d2 = D[ray * 3 + 2];
    const float nn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
    if (nn > 0.0f && isfinite(nn)) sh16(d0 / nn, d1 / nn, d2 / nn, x + 7);
#pragma unroll
    for (int j = 0; j < 3; ++j) g[j] = grad_rgb[ray * 3 + j];
  }
  float* rowA = sA + lane * kVP;
  float* rowB = sB + lane * kVP;
  float* rowX = sX + lane * 32;
  float* rowG = sG + lane * 16;
#pragma unroll
  for (int j = 0; j < 32; ++j) rowX[j] = j < 23 ? x[j < 23 ? j : 0] : 0.0f;
#pragma unroll
  for (int j = 0; j < 16; ++j) rowG[j] = 0.0f;
  // forward
  uint64_t m1 = 0, m2 = 0;
  for (int j = 0; j < 64; ++j) {
    float z = P[kB0 + j];
#pragma unroll
    for (int k = 0; k < 23; ++k) z = __builtin_fmaf(P[kW0 + j * 23 + k], x[k], z);
    m1 |= uint64_t(z > 0.0f) << j;
    rowA[j] = fmaxf(z, 0.0f);
  }
  for (int i = 0; i < 64; ++i) {
    float z = P[kB1 + i];
    for (int j = 0; j < 64; ++j) z = __builtin_fmaf(P[kW1 + i * 64 + j], rowA[j], z);
    m2 |= uint64_t(z > 0.0f) << i;
    rowB[i] = fmaxf(z, 0.0f);
  }
  float gz[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float o = P[kB2 + c];
    for (int i = 0; i < 64; ++i) o = __builtin_fmaf(P[kW2 + c * 64 + i], rowB[i], o);
    const float C = 1.0f / (1.0f + __expf(-(x[c] + o)));
    gz[c] = g[c] * C * (1.0f - C);
    rowG[c] = gz[c];
  }
  __syncthreads();
  float* part = partial + int64_t(blockIdx.x) * kMlpViewParams;
  const int qi = lane >> 4, col = lane & 15;
  // dW2 [3][64] = sum gz (x) a2; db2
#pragma unroll
  for (int jb = 0; jb < 64; jb += 16) {
    f32x4v r = outer16(sG, 16, 0, sB, kVP, jb, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * qi + q;
      if (c < 3) part[kW2 + c * 64 + jb + col] = r[q];
    }
  }
  if (lane < 3) {
    float a = 0.0f;
    for (int r = 0; r < 64; ++r) a += sG[r * 16 + lane];
    part[kB2 + lane] = a;
  }
  __syncthreads();
  // g2 (over a2's rows: dW2 was their last reader)
  for (int i = 0; i < 64; ++i) {
    float a = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) a = __builtin_fmaf(P[kW2 + c * 64 + i], gz[c], a);
    rowB[i] = ((m2 >> i) & 1) ? a : 0.0f;
  }
  __syncthreads();
  // dW1 [64][64] = sum g2 (x) a1; db1
#pragma unroll
  for (int ia = 0; ia < 64; ia += 16) {
#pragma unroll
    for (int jb = 0; jb < 64; jb += 16) {
      f32x4v r = outer16(sB, kVP, ia, sA, kVP, jb, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) part[kW1 + (ia + 4 * qi + q) * 64 + jb + col] = r[q];
    }
  }
  {
    float a = 0.0f;
    for (int r = 0; r < 64; ++r) a += sB[r * kVP + lane];
    part[kB1 + lane] = a;
  }
  __syncthreads();
  // g1 (over a1's rows: dW1 was their last reader) and the input gradients
  float gx[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int j = 0; j < 64; ++j) {
    float a = 0.0f;
    for (int i = 0; i < 64; ++i) a = __builtin_fmaf(P[kW1 + i * 64 + j], rowB[i], a);
    const float g1 = ((m1 >> j) & 1) ? a : 0.0f;
    rowA[j] = g1;
#pragma unroll
    for (int k = 0; k < 7; ++k) gx[k] = __builtin_fmaf(P[kW0 + j * 23 + k], g1, gx[k]);
  }
  if (ok) {
#pragma unroll
    for (int c = 0; c < 3; ++c) grad_cf[ray * 7 + c] = gz[c] + gx[c];
#pragma unroll
    for (int k = 3; k < 7; ++k) grad_cf[ray * 7 + k] = gx[k];
  }
  __syncthreads();
  // dW0 [64][23] = sum g1 (x) x; db0
#pragma unroll
  for (int ia = 0; ia < 64; ia += 16) {
#pragma unroll
    for (int jb = 0; jb < 32; jb += 16) {
      f32x4v r = outer16(sA, kVP, ia, sX, 32, jb, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = jb + col;
        if (k < 23) part[kW0 + (ia + 4 * qi + q) * 23 + k] = r[q];
      }
    }
  }
  {
    float a = 0.0f;
    for (int r = 0; r < 64; ++r) a += sA[r * kVP + lane];
    part[kB0 + lane] = a;
  }
}

int launch_view_mlp_backward(ngprt_ctx* ctx, int64_t n, const float* d, const float* c_d, const float* feat,
                             const float* grad_rgb, float* grad_cf, float* gmlp, hipStream_t st) {
  const int64_t waves = (n + 63) / 64;
  if (waves > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays for one launch");
  const size_t need = (size_t(waves) + kSumGroups) * kMlpViewParams * sizeof(float);
  if (need > ctx->ws_bytes) {
    if (ctx->ws) (void)hipFreeAsync(ctx->ws, st);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (dev_malloc_async((void**)&ctx->ws, need, st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_ALLOC, "view MLP backward workspace allocation failed");
    }
    ctx->ws_bytes = need;
  }
  float* partial = reinterpret_cast<float*>(ctx->ws);
  hipLaunchKernelGGL(view_mlp_backward_kernel, dim3(unsigned(waves)), dim3(64), 0, st, n, d, c_d, feat, grad_rgb,
                     ctx->mlp, grad_cf, partial);
  int rc = check_launch(ctx, "view_mlp_backward_kernel");
  if (rc) return rc;
  return launch_partial_sums(ctx, partial, waves, kMlpViewParams, partial + size_t(waves) * kMlpViewParams, gmlp,
                             st);
}

int launch_view_mlp_arrange(ngprt_ctx* ctx, const float* params, hipStream_t st) {
  hipLaunchKernelGGL(view_mlp_arrange_kernel, dim3((kViewRecFloats + 255) / 256), dim3(256), 0, st, params,
                     ctx->mlp_rec);
  return check_launch(ctx, "view_mlp_arrange_kernel");
}

int launch_view_mlp(ngprt_ctx* ctx, int64_t n, const float* d, const float* c_d, const float* feat,
                    float* rgb, hipStream_t st) {
  if (n <= 0) return NGPRT_OK;
  if (ctx->vmlp_resident <= 0) {
    // workgroups of view_mlp_kernel that stay resident together on the device
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, view_mlp_kernel, 64 * kViewWaves, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        per_cu <= 0 || cus <= 0) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_HIP, "view_mlp_kernel occupancy query failed");
    }
    ctx->vmlp_resident = per_cu * cus;
  }
  const int64_t groups = (n + 64 * kViewWaves - 1) / (64 * kViewWaves);
  const int64_t blocks = groups < ctx->vmlp_resident ? groups : ctx->vmlp_resident;
  hipLaunchKernelGGL(view_mlp_kernel, dim3(unsigned(blocks)), dim3(64 * kViewWaves), 0, st, n, d, c_d, feat,
                     ctx->mlp_rec, rgb);
  return check_launch(ctx, "view_mlp_kernel");
}

}  // namespace ngprt
