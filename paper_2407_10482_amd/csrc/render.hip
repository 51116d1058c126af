// Render kernels: occupancy-distance march, hashed lookup + attention,
// front-to-back compositing, and the deferred MLP on MFMA.
//
// One lane owns one ray; a wave owns 64 rays (an 8x8 pixel tile when the
// caller orders rays tile-major, which keeps the coarse-level gathers of a
// wave on shared cache lines; neighbouring rays also march alike, so the
// wave's lanes finish within a sample or two of each other).  Each iteration every live lane first marches
// to its next occupied lattice point (divergent but cheap: one 2-byte grid
// read per marching point, none inside a known-empty region), then all lanes
// holding a sample evaluate it together (the gather-heavy part runs with the
// wave converged).  After the last ray of the wave finishes, the wave runs
// the deferred MLP for its 64 rays with v_mfma_f32_16x16x4_f32.
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "march.h"
#include "proposal_net.h"

namespace ngprt {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// MODE_RENDER: plain render.  MODE_RENDER_EXT: render that also writes the
// label outputs (t_first / t_far / t_half) and honours a proposal.
// MODE_MARCH: sample lists for parity checks (no MLP).
enum { MODE_RENDER = 0, MODE_MARCH = 1, MODE_RENDER_EXT = 2 };

// Optional per-ray sample-interval proposal [t_near, t_far, t_term,
// confidence], given per ray (prop) or computed by the loaded network in the
// kernel's prologue (net_w): a ray whose confidence reaches conf_thr marches
// only the lattice points with t in [t_near - margin, t_far + margin] (box:
// from lattice index max(0, floor((t_near - margin - t0) / step)); contracted
// domain: points before t_near - margin are visited without a read; without
// use_near from its start).  With far_guard > 0 the far end ends a ray only
// once its transmittance is below far_guard; otherwise it marches on.  A
// proposed ray that takes no sample in its interval marches again from its
// start as the plain march (its samples are then the plain render's; its
// read count includes both marches).
struct ProposalArgs {
  const float* prop;     // [n][4] (NULL: no per-ray proposal given)
  const uint2* net_w;    // loaded network: A-operand tiles (NULL: none)
  const float* net_b;    // its biases
  float* prop_out;       // [n][4] the network's outputs (NULL-able)
  float conf_thr;
  float margin;
  int use_near;
  float far_guard;
  int32_t* fallback;     // [n] 1 where the plain march ran after a proposal (NULL-able)
};

struct MarchRecord {
  int32_t* sample_k;
  int32_t* n_samples;
  int32_t* n_reads;
  int cap;
};

// Deferred MLP of the 64 rays of this wave (Eq. 5), 7 -> 16 -> 16 -> 3 on
// v_mfma_f32_16x16x4_f32.  xin: this wave's LDS slab [8][64] holding
// (C_d, F, 0) of every lane's ray.  Layout of the 16x16x4 product D = A B:
// lane l supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[4*(l/16) + r][l%16], r = 0..3.  The hidden index handed from one layer
// to the next is permuted (k-slot s of chunk c = unit 4s + c) so every layer
// consumes the previous layer's accumulators in place.
__device__ __forceinline__ void wave_mlp(const float* __restrict__ P, const float* xin, int lane,
                                         int64_t ray_base, int64_t n, float* __restrict__ rgb) {
  const int i = lane & 15, s = lane >> 4;
  float a1[2], a2[4], a3[4];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    int k = 4 * c + s;
    a1[c] = (k < 7) ? P[i * 7 + k] : 0.0f;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    a2[c] = P[128 + i * 16 + 4 * s + c];
    a3[c] = (i < 3) ? P[400 + i * 16 + 4 * s + c] : 0.0f;
  }
  float b0[4], b1[4], b2[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    b0[r] = P[112 + 4 * s + r];
    b1[r] = P[384 + 4 * s + r];
    b2[r] = (4 * s + r < 3) ? P[448 + 4 * s + r] : 0.0f;
  }
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int ray = blk * 16 + i;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 2; ++c)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[c], xin[(4 * c + s) * 64 + ray], acc, 0, 0, 0);
    float h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = fmaxf(acc[r] + b0[r], 0.0f);
    acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[c], h[c], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = fmaxf(acc[r] + b1[r], 0.0f);
    acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[c], h[c], acc, 0, 0, 0);
    if (s == 0) {
      const int64_t gr = ray_base + ray;
      if (gr < n) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          float z = xin[j * 64 + ray] + (acc[j] + b2[j]);
          rgb[gr * 3 + j] = 1.0f / (1.0f + __expf(-z));
        }
      }
    }
  }
}

// Occupancy floor of the render kernel (waves per SIMD; the 16-level kernels
// fit 4 with ~126 VGPRs).  Giving each XCD one contiguous eighth of the rays
// measured slower on the 8-view 1080p workload (54.2 -> 61.9 ms): the XCDs
// then work on different views at once and share no Infinity Cache lines.
#ifndef NGPRT_RENDER_WAVES_PER_EU
#define NGPRT_RENDER_WAVES_PER_EU 4
#endif
#ifndef NGPRT_XCD_CHUNK
#define NGPRT_XCD_CHUNK 0
#endif

// MODEL: bit 0 = baked feature model, bit 1 = occupancy pyramid march,
// bit 2 = the baked model's ablation aggregations
template <int DOM, int DT, int LMAX, int MODE, int MODEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NGPRT_RENDER_WAVES_PER_EU)))
render_kernel(SceneArgs S, int64_t n, const float* __restrict__ O,
                                                     const float* __restrict__ D, RayOut out,
                                                     MarchRecord rec, const float* __restrict__ mlp,
                                                     int naive, ProposalArgs pa) {
  __shared__ float xin_all[4][8 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#if NGPRT_XCD_CHUNK > 0
  // workgroups are dispatched round-robin over the 8 XCDs: give each XCD runs
  // of NGPRT_XCD_CHUNK consecutive ray tiles-of-4 (neighbouring rays share
  // cache lines in its L2) while all XCDs still sweep the same image region
  // (their L2 misses share Infinity Cache lines); the last partial round of
  // 8 * chunk workgroups keeps the identity placement
  constexpr unsigned C = NGPRT_XCD_CHUNK;
  const unsigned xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;
  const unsigned full = gridDim.x / (8u * C);
  const unsigned block = (slot / C < full) ? (slot / C) * (8u * C) + xcd * C + (slot % C) : blockIdx.x;
#else
  const unsigned block = blockIdx.x;
#endif
  const int64_t ray_base = (int64_t(block) * 4 + wave) * 64;
  const int64_t ray = ray_base + lane;
  const bool in_range = ray < n;

  MarchState m;
  const float* oray = O + 3 * (in_range ? ray : 0);
  const float* dray = D + 3 * (in_range ? ray : 0);
  march_init<DOM>(S, oray, dray, in_range, m);
  constexpr bool EXT = MODE == MODE_RENDER_EXT;
  bool proposed = false, fell_back = false;
  if (EXT && (pa.prop || pa.net_w)) {
    float q[4];
    if (pa.net_w) {
      // the loaded network, run by the wave for its 64 rays (uniform branch:
      // every wave of the grid takes it)
      float* out4 = xin_all[wave];
      prop_infer_wave(pa.net_w, pa.net_b, O, D, ray_base, n, lane, out4);
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = out4[4 * lane + c];
      __syncthreads();
      if (pa.prop_out && in_range) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pa.prop_out[4 * ray + c] = q[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = in_range ? pa.prop[4 * ray + c] : 0.0f;
    }
    if (in_range && !m.done && q[3] >= pa.conf_thr) {
      m.t_hi = q[1] + pa.margin;
      if (pa.use_near) {
        const float lo = q[0] - pa.margin;
        if (DOM == DOM_BOX) {
          const float kf = floorf((lo - m.t0) / S.step);
          m.k = kf > 0.0f ? (kf < (float)kMaxLattice ? (int)kf : kMaxLattice) : 0;
        } else {
          m.t_lo = lo;
        }
      }
      proposed = true;
    }
  }
  float T = 1.0f, cd[3] = {0.f, 0.f, 0.f}, fv[4] = {0.f, 0.f, 0.f, 0.f}, depth = 0.0f;
  // labels: t of the first sample, of the sample after which T < 0.5, and of
  // the sample after which T < 1e-3 (the proposal's far end)
  float t_first = 0.0f, t_last = 0.0f, t_half = 0.0f, t_far = 0.0f;
  bool half_set = false, far_set = false;
  // distortion regulariser: running sums of w, w m and w (m W_< - S_<), and w^2
  float dW = 0.0f, dS = 0.0f, dP = 0.0f, dQ = 0.0f;
  int ns = 0, reads = 0;

  for (;;) {
    float u[3], ts;
    int ks;
    bool have = march_next<DOM, (MODEL & 2) != 0, EXT>(S, m, naive != 0, reads, u, ts, ks);
    if (EXT && !have && proposed && !fell_back) {
      if (ns == 0) {
        // the proposed interval holds no occupied lattice point: march again
        // from the start as the plain march
        march_init<DOM>(S, oray, dray, in_range, m);
        fell_back = true;
        have = march_next<DOM, (MODEL & 2) != 0, EXT>(S, m, naive != 0, reads, u, ts, ks);
      } else if (m.stopped_at_hi && pa.far_guard > 0.0f && !(T < pa.far_guard)) {
        // at the proposed far end with too much transmittance left: march on
        m.t_hi = __int_as_float(0x7F800000);
        m.done = false;
        m.stopped_at_hi = false;
        have = march_next<DOM, (MODEL & 2) != 0, EXT>(S, m, naive != 0, reads, u, ts, ks);
      }
    }
    if (__ballot(have) == 0) break;
    if (have) {
      float f[8];
      eval_sample<MODEL & 5, DT, LMAX>(S, u, f);
      const float sigma = exp32(f[0]);
      const float e = exp32(-(sigma * S.step));
      const float alpha = 1.0f - e;
      const float w = T * alpha;
#pragma unroll
      for (int j = 0; j < 3; ++j) cd[j] = __builtin_fmaf(w, f[1 + j], cd[j]);
#pragma unroll
      for (int j = 0; j < 4; ++j) fv[j] = __builtin_fmaf(w, f[4 + j], fv[j]);
      depth = __builtin_fmaf(w, ts, depth);
      if (MODE == MODE_MARCH && ns < rec.cap) rec.sample_k[ray * rec.cap + ns] = ks;
      T = T * e;
      if (EXT) {
        const float mid = ((float)ks + 0.5f) * S.step;
        dP = __builtin_fmaf(w, mid * dW - dS, dP);
        dQ = __builtin_fmaf(w, w, dQ);
        dW = dW + w;
        dS = __builtin_fmaf(w, mid, dS);
        if (ns == 0) t_first = ts;
        t_last = ts;
        if (!half_set && T < 0.5f) { t_half = ts; half_set = true; }
        if (!far_set && T < 1e-3f) { t_far = ts; far_set = true; }
      }
      ++ns;
      if (T < S.thr || ns >= S.max_samples) m.done = true;
    }
  }
  if (!half_set) t_half = t_last;
  if (!far_set) t_far = t_last;

  if (MODE == MODE_MARCH) {
    if (in_range) {
      for (int j = ns; j < rec.cap; ++j) rec.sample_k[ray * rec.cap + j] = -1;
      if (rec.n_samples) rec.n_samples[ray] = ns;
      if (rec.n_reads) rec.n_reads[ray] = reads;
    }
    return;
  }
  if (in_range) {
    if (out.c_d) { for (int j = 0; j < 3; ++j) out.c_d[ray * 3 + j] = cd[j]; }
    if (out.feat) { for (int j = 0; j < 4; ++j) out.feat[ray * 4 + j] = fv[j]; }
    if (out.t_final) out.t_final[ray] = T;
    if (out.depth) out.depth[ray] = depth;
    if (out.n_samples) out.n_samples[ray] = ns;
    if (out.n_reads) out.n_reads[ray] = reads;
    if (EXT) {
      if (out.t_first) out.t_first[ray] = t_first;
      if (out.t_far) out.t_far[ray] = t_far;
      if (out.t_half) out.t_half[ray] = t_half;
      if (out.dist_loss) out.dist_loss[ray] = 2.0f * dP + dQ * (S.step * (1.0f / 3.0f));
      if (pa.fallback) pa.fallback[ray] = fell_back ? 1 : 0;
    }
  }
  float* xin = xin_all[wave];
  xin[0 * 64 + lane] = cd[0];
  xin[1 * 64 + lane] = cd[1];
  xin[2 * 64 + lane] = cd[2];
  xin[3 * 64 + lane] = fv[0];
  xin[4 * 64 + lane] = fv[1];
  xin[5 * 64 + lane] = fv[2];
  xin[6 * 64 + lane] = fv[3];
  xin[7 * 64 + lane] = 0.0f;
  __syncthreads();
  if (!S.view_mlp) wave_mlp(mlp, xin, lane, ray_base, n, out.rgb);
}

template <int DT, int LMAX, int MODEL>
__global__ void __launch_bounds__(256) eval_points_kernel(SceneArgs S, int64_t n,
                                                          const float* __restrict__ pos,
                                                          int32_t* idx, float* fused, float* weights) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  float u[3];
  for (int a = 0; a < 3; ++a) u[a] = (p[a] - S.lo) * S.inv_ext;
  float f[8], w[LMAX];
  int32_t id[LMAX * 8];
  eval_sample<MODEL, DT, LMAX, true>(S, u, f, w, id);
  if (fused)
    for (int j = 0; j < 8; ++j) fused[i * 8 + j] = f[j];
  if (weights)
    for (int l = 0; l < S.L; ++l) weights[i * S.L + l] = w[l];
  if (idx)
    for (int l = 0; l < S.L; ++l)
      for (int k = 0; k < 8; ++k) idx[(i * S.L + l) * 8 + k] = id[l * 8 + k];
}

// ---------------------------------------------------------------------------
// dispatch

template <int MODE, int DOM, int DT>
static void dispatch_l(const SceneArgs& S, dim3 g, hipStream_t st, int64_t n, const float* o,
                       const float* d, const RayOut& out, const MarchRecord& rec,
                       const float* mlp, int naive, const ProposalArgs& pa) {
  if (S.model == 1 && S.gen) {
    // the ablation aggregations: float32 tables only (checked at create)
    if constexpr (DT == DT_F32) {
      if (S.pyr_n > 0)
        hipLaunchKernelGGL((render_kernel<DOM, DT, 4, MODE, 7>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                           mlp, naive, pa);
      else
        hipLaunchKernelGGL((render_kernel<DOM, DT, 4, MODE, 5>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                           mlp, naive, pa);
    }
  } else if (S.model == 1 && S.L <= 2) {
    // at most two fine levels: coarse rows of at most 12 channels
    if (S.pyr_n > 0)
      hipLaunchKernelGGL((render_kernel<DOM, DT, 2, MODE, 3>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                         mlp, naive, pa);
    else
      hipLaunchKernelGGL((render_kernel<DOM, DT, 2, MODE, 1>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                         mlp, naive, pa);
  } else if (S.model == 1 && S.pyr_n > 0)
    hipLaunchKernelGGL((render_kernel<DOM, DT, 4, MODE, 3>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                       mlp, naive, pa);
  else if (S.model == 1)
    hipLaunchKernelGGL((render_kernel<DOM, DT, 4, MODE, 1>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                       mlp, naive, pa);
  else if (S.pyr_n > 0)
    hipLaunchKernelGGL((render_kernel<DOM, DT, 16, MODE, 2>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                       mlp, naive, pa);
  else if (S.L <= 8)
    hipLaunchKernelGGL((render_kernel<DOM, DT, 8, MODE, 0>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                       mlp, naive, pa);
  else
    hipLaunchKernelGGL((render_kernel<DOM, DT, 16, MODE, 0>), g, dim3(256), 0, st, S, n, o, d, out, rec,
                       mlp, naive, pa);
}

template <int MODE>
static void dispatch(const SceneArgs& S, int dom, int dt, dim3 g, hipStream_t st, int64_t n,
                     const float* o, const float* d, const RayOut& out, const MarchRecord& rec,
                     const float* mlp, int naive, const ProposalArgs& pa) {
#define NGPRT_CASE(DOMV, DTV)                                                       \
  if (dom == DOMV && dt == DTV) {                                                   \
    dispatch_l<MODE, DOMV, DTV>(S, g, st, n, o, d, out, rec, mlp, naive, pa);       \
    return;                                                                         \
  }
  NGPRT_CASE(DOM_BOX, DT_F32)
  NGPRT_CASE(DOM_BOX, DT_BF16)
  NGPRT_CASE(DOM_BOX, DT_FP8)
  NGPRT_CASE(DOM_CONTRACT, DT_F32)
  NGPRT_CASE(DOM_CONTRACT, DT_BF16)
  NGPRT_CASE(DOM_CONTRACT, DT_FP8)
#undef NGPRT_CASE
}

int launch_render(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const RayOut& out,
                  const float* prop, bool use_net, float* prop_out, const ngprt_proposal_cfg& pc,
                  int32_t* fallback, hipStream_t st) {
  SceneArgs S = scene_args(ctx);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays for one launch");
  MarchRecord rec{nullptr, nullptr, nullptr, 0};
  const uint2* net_w = use_net ? reinterpret_cast<const uint2*>(ctx->prop_net) : nullptr;
  const float* net_b = use_net ? reinterpret_cast<const float*>(
                                     reinterpret_cast<const char*>(ctx->prop_net) + kPropTiles * 64 * 8)
                               : nullptr;
  ProposalArgs pa{prop,         net_w,           net_b,        use_net ? prop_out : nullptr,
                  pc.conf_threshold, pc.margin, pc.use_near, pc.far_guard, fallback};
  const bool ext = prop || use_net || out.t_first || out.t_far || out.t_half || out.dist_loss;
  if (ext)
    dispatch<MODE_RENDER_EXT>(S, ctx->desc.domain, ctx->desc.table_dtype, dim3(unsigned(blocks)), st, n,
                              o, d, out, rec, ctx->mlp, 0, pa);
  else
    dispatch<MODE_RENDER>(S, ctx->desc.domain, ctx->desc.table_dtype, dim3(unsigned(blocks)), st, n, o,
                          d, out, rec, ctx->mlp, 0, pa);
  int rc = check_launch(ctx, "render_kernel");
  if (rc == NGPRT_OK && S.view_mlp) rc = launch_view_mlp(ctx, n, d, out.c_d, out.feat, out.rgb, st);
  return rc;
}

int launch_march(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, int32_t cap,
                 int32_t* sk, int32_t* ns, int32_t* nr, int naive, hipStream_t st) {
  SceneArgs S = scene_args(ctx);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays for one launch");
  MarchRecord rec{sk, ns, nr, cap};
  RayOut out{};
  ProposalArgs pa{nullptr, nullptr, nullptr, nullptr, 0.0f, 0.0f, 0, 0.0f, nullptr};
  dispatch<MODE_MARCH>(S, ctx->desc.domain, ctx->desc.table_dtype, dim3(unsigned(blocks)), st, n, o,
                       d, out, rec, ctx->mlp, naive, pa);
  return check_launch(ctx, "march_kernel");
}

int launch_eval_points(ngprt_ctx* ctx, int64_t n, const float* pos, int32_t* idx, float* fused,
                       float* weights, hipStream_t st) {
  SceneArgs S = scene_args(ctx);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many points for one launch");
  dim3 g = dim3(unsigned(blocks));
  const int dt = ctx->desc.table_dtype;
#define NGPRT_EV(DTV, LM, MD)                                                                   \
  hipLaunchKernelGGL((eval_points_kernel<DTV, LM, MD>), g, dim3(256), 0, st, S, n, pos, idx, fused, \
                     weights)
#define NGPRT_EV_DT(DTV)                   \
  if (dt == DTV) {                         \
    if (S.model == 1) NGPRT_EV(DTV, 4, 1); \
    else if (S.L <= 8) NGPRT_EV(DTV, 8, 0); \
    else NGPRT_EV(DTV, 16, 0);              \
  }
  if (S.model == 1 && S.gen)   // the ablation aggregations: float32 tables only (checked at create)
    NGPRT_EV(DT_F32, 4, 5);
  else {
    NGPRT_EV_DT(DT_F32)
  }
  NGPRT_EV_DT(DT_BF16)
  NGPRT_EV_DT(DT_FP8)
#undef NGPRT_EV_DT
#undef NGPRT_EV
  return check_launch(ctx, "eval_points_kernel");
}

}  // namespace ngprt
