// Backward of the render path (a training extension; the paper trains its
// model but states no gradient code).  FP32 tables only.
//
// Forward state is recomputed per ray instead of stored per sample:
//  pass 1  re-march the ray: composited C_d and F (Eq. 2, Eq. 5), or take
//          the forward's per-ray C_d and F when the caller hands them over
//          (the same float32 values; not with the regulariser, whose sums
//          this pass also forms); then, per
//          lane, the deferred MLP forward and backward give dL/dC_d, dL/dF,
//          and per-ray outer products whose sum over the wave's 64 rays is
//          taken on v_mfma_f32_16x16x4_f32 (K = rays) and written as one
//          451-float partial per wave (with the view-dependent MLP, dL/dC_d
//          and dL/dF come per ray from its own backward instead, `ups`);
//  pass 2  re-march again with the same decisions; at each sample
//          dL/dsigma_i = delta (T_{i+1} s_i - (S - P_i)) with
//          s_i = dL/dC_d . c_i + dL/dF . v_i, S = dL/dC_d . C_d + dL/dF . F and
//          P_i the running sum of w_j s_j; then the softmax adjoint
//          dL/da_l = w_l (dL/df . v_l - dL/df . f) and the trilinear scatter of
//          every level's 9-channel gradient into its 8 corner entries with
//          hardware float atomics (order-nondeterministic sums).  The wave
//          first sums the contributions to equal entries (neighbouring rays'
//          samples share cells) so one lane issues each entry's atomics:
//          per corner slot the 64 (entry, lane) words are sorted across the
//          wave (a bitonic network on DPP and swizzle lane moves), runs of
//          equal entries are summed by a segmented scan, and the last lane
//          of each run issues the atomics.  Measured on 2^18-ray training
//          batches (backward kernel): 16 x 2^19 tables 174 -> 92 ms, 8 x 2^14
//          35 -> 14 ms against one pass per distinct entry with a butterfly
//          sum each; spreading each run's 9 channel atomics over neighbouring
//          lanes of one instruction (scatter_runs) then 92 -> 20 ms and
//          14 -> 7 ms.
//          The baked model scatters into its fine levels and coarse atlas
//          rows instead (baked_scatter).  In the deterministic mode each
//          contribution goes to a record of its own instead (det.hip).
// The per-wave MLP partials are then added in a fixed order (reduce.h).
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "internal.h"
#include "march.h"
#include "reduce.h"

namespace ngprt {

typedef float bf32x4 __attribute__((ext_vector_type(4)));

constexpr int kPad = 17;   // LDS row pitch of the per-wave staging (bank spread)

// Levels of at least this resolution merge equal table entries across the
// wave by sorting (wave_sort_merge); coarser levels, where a wave's samples
// share a handful of cells, by the leader loop (one pass per distinct entry).
#ifndef NGPRT_BW_SORT_MIN_RES
#define NGPRT_BW_SORT_MIN_RES 16
#endif

// value of lane (lane ^ J) for every lane of a full wave; J = 1, 2, 4, 8 by
// DPP lane moves (quad_perm, row_half_mirror, row_mirror), 16 by ds_swizzle,
// 32 by ds_bpermute
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane) {
  const int x = int(v);
  if constexpr (J == 1) return uint32_t(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));
  if constexpr (J == 2) return uint32_t(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));
  if constexpr (J == 4) {
    const int h = __builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false);   // i ^ 7 within 8
    return uint32_t(__builtin_amdgcn_update_dpp(h, h, 0x1B, 0xF, 0xF, false)); // then ^ 3
  }
  if constexpr (J == 8) {
    const int m = __builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false);   // i ^ 15 within 16
    return uint32_t(__builtin_amdgcn_update_dpp(m, m, 0x141, 0xF, 0xF, false)); // then ^ 7
  }
  if constexpr (J == 16) return uint32_t(__builtin_amdgcn_ds_swizzle(x, 0x401F));
  return uint32_t(__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, x));
}

constexpr int kStageRow = 17;   // staged run: up to 16 values and the key

// The atomics of a merged level.  The 9 (NV) channels of each run's row go to
// neighbouring lanes of one atomic instruction, so an instruction carries the
// rows of about 7 runs, 9 consecutive floats each: the tail lanes (one per
// run) stage key and values in this wave's LDS slab `stage` (64 x 17 words),
// then lane q of each pass adds value q % NV of run q / NV.  Measured on
// 2^18-ray training batches (backward kernel, 16 x 2^19 / 8 x 2^14 tables):
// 91.6 / 14.5 ms with 9 one-lane-per-run instructions, 19.8 / 7.0 ms spread
// (the same-line atomics of one instruction are combined on their way to
// memory).
// Rows are `stride` floats apart (9 for the tables, C for the coarse atlas);
// only the first nv <= NV channels are added.
template <int NV>
__device__ __forceinline__ void scatter_runs(float* __restrict__ gbase, bool tail, uint32_t key, const float x[NV],
                                             int lane, float* stage, int stride = 9, int nv = NV) {
  static_assert(NV < kStageRow, "a staged row holds the values and the key");
  const uint64_t tm = __ballot(tail);
  const int m = __popcll(tm);
  if (tail) {
    const int rank = __builtin_amdgcn_mbcnt_hi(uint32_t(tm >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(tm), 0));
    float* row = stage + rank * kStageRow;
#pragma unroll
    for (int j = 0; j < NV; ++j) row[j] = x[j];
    row[kStageRow - 1] = __uint_as_float(key);
  }
  // the other lanes' staged rows are read below: a wave-scope fence orders
  // the LDS stores before the loads (and the next call's stores after them)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  for (int q = lane; q < nv * m; q += 64) {
    const int t = q / nv, c = q - t * nv;
    const float* row = stage + t * kStageRow;
    unsafeAtomicAdd(gbase + size_t(__float_as_uint(row[kStageRow - 1])) * size_t(stride) + c, row[c]);
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// one compare-exchange stage of a bitonic sort over the wave's 64 lanes
template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_stage(uint32_t v, int lane) {
  const uint32_t o = lane_xor<J>(v, lane);
  const bool keep_min = ((lane & J) == 0) == ((lane & K) == 0);
  const uint32_t lo = v < o ? v : o, hi = v < o ? o : v;
  return keep_min ? lo : hi;
}

// Sums the NV values of the wave's lanes that hold the same key (an entry
// index below 2^26; lanes with active = false take no part).  Sorting the
// words (key << 6 | lane) puts equal keys on neighbouring lanes; each lane
// fetches the values of the lane whose word it holds, runs of equal keys are
// summed by a scan (skipped when no key repeats) and the last lane of each
// run returns true with the run's key and sum in key, v.  Every lane of the
// wave must call this with all 64 lanes active.
template <int NV>
__device__ __forceinline__ bool wave_sort_merge(uint32_t& key, bool active, float v[NV], int lane) {
  uint32_t w = active ? ((key << 6) | uint32_t(lane)) : 0xFFFFFFFFu;
  w = bitonic_stage<2, 1>(w, lane);
  w = bitonic_stage<4, 2>(w, lane);   w = bitonic_stage<4, 1>(w, lane);
  w = bitonic_stage<8, 4>(w, lane);   w = bitonic_stage<8, 2>(w, lane);   w = bitonic_stage<8, 1>(w, lane);
  w = bitonic_stage<16, 8>(w, lane);  w = bitonic_stage<16, 4>(w, lane);  w = bitonic_stage<16, 2>(w, lane);
  w = bitonic_stage<16, 1>(w, lane);
  w = bitonic_stage<32, 16>(w, lane); w = bitonic_stage<32, 8>(w, lane);  w = bitonic_stage<32, 4>(w, lane);
  w = bitonic_stage<32, 2>(w, lane);  w = bitonic_stage<32, 1>(w, lane);
  w = bitonic_stage<64, 32>(w, lane); w = bitonic_stage<64, 16>(w, lane); w = bitonic_stage<64, 8>(w, lane);
  w = bitonic_stage<64, 4>(w, lane);  w = bitonic_stage<64, 2>(w, lane);  w = bitonic_stage<64, 1>(w, lane);
  const bool valid = w != 0xFFFFFFFFu;
  const int src = int(w & 63u);
  const uint32_t k = w >> 6;
  float x[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j)
    x[j] = __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v[j])));
  // neighbours' keys (sentinels sort last, so a valid lane's successor is
  // either valid or the sentinel)
  const uint32_t next = uint32_t(__builtin_amdgcn_ds_bpermute(((lane + 1) & 63) << 2, int(k)));
  const bool tail = valid && (lane == 63 || next != k);
  // segmented inclusive scan over runs of equal keys (Hillis-Steele), only
  // as far as the longest run needs
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t pk = uint32_t(__builtin_amdgcn_ds_bpermute(((lane - d) & 63) << 2, int(k)));
    const bool same = valid && lane >= d && pk == k;
    if (__ballot(same) == 0) break;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const float o = __int_as_float(__builtin_amdgcn_ds_bpermute(((lane - d) & 63) << 2, __float_as_int(x[j])));
      x[j] = same ? x[j] + o : x[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = x[j];
  key = k;
  return tail;
}

// D[i][j] = sum over the wave's 64 rays r of A_r[i] * B_r[j] (i, j < 16).
// sA, sB: [64][kPad].  Lane l returns D[4*(l/16) + q][l%16], q = 0..3.
__device__ __forceinline__ bf32x4 wave_outer_sum(const float* sA, const float* sB, int lane) {
  const int i = lane & 15, s = lane >> 4;
  bf32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int r = 4 * c + s;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sA[r * kPad + i], sB[r * kPad + i], acc, 0, 0, 0);
  }
  return acc;
}

// Corner k of a cell for a loop counter k that is the same on every lane:
// picked from registers by selects, where indexing the arrays with k would
// put them in per-lane scratch memory (a store per level and a load per
// corner through the vector memory pipeline).
__device__ __forceinline__ void corner_pick(const Corners& c, int k, uint32_t& idx, float& w) {
  idx = c.idx[0];
  w = c.w[0];
#pragma unroll
  for (int j = 1; j < 8; ++j) {
    idx = k == j ? c.idx[j] : idx;
    w = k == j ? c.w[j] : w;
  }
}

// Adjoint of the baked feature construction at one sample (Sec. 4.2 Eq. 7-8):
// with f_0 = f~_0 + sum_l g(omega_l) s_l and f_j = f~_j + sum_l g(beta_l) v_lj
// (j >= 1), dL/df (gf) gives
//   fine level l:  dL/dv_l0 = gf_0 g(omega_l),  dL/dv_lj = gf_j g(beta_l),
//   coarse row:    dL/df~_j = gf_j,
//                  dL/domega_l = gf_0 s_l g'(omega_l),
//                  dL/dbeta_l = sum_{j>=1} gf_j v_lj g'(beta_l),
// each spread trilinearly over its 8 corners; g' = g (1 - g).  Vertices of
// empty blocks take the default vector and receive no gradient.  Every lane
// of the wave takes part (have = false: no contribution) so that equal
// entries are summed across the wave before one lane issues their atomics.
// gtab: [L][T][9] (channel 8, the hash model's logit, untouched); gatlas:
// [n_blocks][8][8][8][C], C = 8 + 2 L.
template <int LMAX>
__device__ __forceinline__ void baked_scatter(const SceneArgs& S, const float u[3], bool have, const float gf[8],
                                              float* __restrict__ gtab, float* __restrict__ gatlas,
                                              float* stage) {
  static_assert(LMAX <= 4, "the coarse row holds at most 16 channels");
  constexpr int CMAX = 8 + 2 * LMAX;
  const int C = 8 + 2 * S.L;
  int i0[3];
  float fr[3], gr[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float p = u[a] * S.LCf;
    int i = (int)floorf(p);
    i = i < 0 ? 0 : (i > S.LC - 1 ? S.LC - 1 : i);
    i0[a] = i;
    fr[a] = __builtin_fmaf(u[a], S.LCf, -(float)i);
    gr[a] = 1.0f - fr[a];
  }
  // interpolated attention parameters (coarse channels 8 .. 8 + 2L)
  float ap[2 * LMAX];
#pragma unroll
  for (int j = 0; j < 2 * LMAX; ++j) ap[j] = 0.0f;
  if (have) {
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
      const int vx = i0[0] + bx, vy = i0[1] + by, vz = i0[2] + bz;
      const int bid = S.cidx[((vz >> 3) * S.nb + (vy >> 3)) * S.nb + (vx >> 3)];
      const float wk = ((bx ? fr[0] : gr[0]) * (by ? fr[1] : gr[1])) * (bz ? fr[2] : gr[2]);
      float v[8];
      if (bid >= 0) {
        const float4* row = reinterpret_cast<const float4*>(
            S.catlas + (size_t(bid) * 512 + size_t(((vz & 7) * 8 + (vy & 7)) * 8 + (vx & 7))) * S.Cpad);
        const float4 q2 = row[2];
        const float4 q3 = S.Cpad > 12 ? row[3] : make_float4(0.f, 0.f, 0.f, 0.f);
        v[0] = q2.x; v[1] = q2.y; v[2] = q2.z; v[3] = q2.w;
        v[4] = q3.x; v[5] = q3.y; v[6] = q3.z; v[7] = q3.w;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = S.cdef[8 + j];
      }
#pragma unroll
      for (int j = 0; j < 2 * LMAX; ++j) ap[j] = __builtin_fmaf(wk, v[j], ap[j]);
    }
  }
  float gco[CMAX];
#pragma unroll
  for (int j = 0; j < 8; ++j) gco[j] = have ? gf[j] : 0.0f;
#pragma unroll
  for (int j = 8; j < CMAX; ++j) gco[j] = 0.0f;
  const size_t T_entries = size_t(1) << S.log2T;
  // fine levels: values for the gate gradients, then the 8-channel scatter
#pragma unroll
  for (int l = 0; l < LMAX; ++l) {
    if (l >= S.L) break;
    Corners c;
    level_corners(u, S.N[l], S.Nf[l], S.mask, c);
    float gv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) gv[j] = 0.0f;
    if (have) {
      const void* fb = feat_level<DT_F32>(S.feat, l, S.log2T);
      float acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float v[8];
        Store<DT_F32>::feat(fb, c.idx[k], v);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_fmaf(c.w[k], v[j], acc[j]);
      }
      const float gw = sigmoid32(ap[2 * l]), gb = sigmoid32(ap[2 * l + 1]);
      float tb = 0.0f;
#pragma unroll
      for (int j = 1; j < 8; ++j) tb = __builtin_fmaf(gf[j], acc[j], tb);
      gco[8 + 2 * l] = gf[0] * acc[0] * (gw * (1.0f - gw));
      gco[9 + 2 * l] = tb * (gb * (1.0f - gb));
      gv[0] = gf[0] * gw;
#pragma unroll
      for (int j = 1; j < 8; ++j) gv[j] = gf[j] * gb;
    }
    float* gbase = gtab + (size_t(l) * T_entries) * 9;
    const int lane = threadIdx.x & 63;
    if (S.N[l] >= NGPRT_BW_SORT_MIN_RES) {
#pragma unroll 1
      for (int k = 0; k < 8; ++k) {
        uint32_t key;
        float wk;
        corner_pick(c, k, key, wk);
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = wk * gv[j];
        const bool tail = wave_sort_merge<8>(key, have, x, lane);
        scatter_runs<8>(gbase, tail, key, x, lane, stage);
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      bool pending = have;
      uint64_t pm = __ballot(pending);
      while (pm) {
        const int leader = __ffsll((unsigned long long)pm) - 1;
        const uint32_t key = __shfl(c.idx[k], leader, 64);
        const bool mine = pending && c.idx[k] == key;
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = mine ? c.w[k] * gv[j] : 0.0f;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) x[j] += __shfl_xor(x[j], off, 64);
        }
        if (lane == leader) {
          float* dst = gbase + size_t(key) * 9;
#pragma unroll
          for (int j = 0; j < 8; ++j) unsafeAtomicAdd(dst + j, x[j]);
        }
        pending = pending && !mine;
        pm = __ballot(pending);
      }
    }
  }
  // coarse rows: one vertex = (atlas row, local offset)
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
    const int vx = i0[0] + bx, vy = i0[1] + by, vz = i0[2] + bz;
    const int bid = have ? S.cidx[((vz >> 3) * S.nb + (vy >> 3)) * S.nb + (vx >> 3)] : -1;
    const int loc = ((vz & 7) * 8 + (vy & 7)) * 8 + (vx & 7);
    const float wk = ((bx ? fr[0] : gr[0]) * (by ? fr[1] : gr[1])) * (bz ? fr[2] : gr[2]);
    if (S.n_blocks <= (1 << 17)) {
      // vertex key bid * 512 + loc < 2^26: sorted merge and spread atomics
      uint32_t key = bid >= 0 ? uint32_t(bid) * 512u + uint32_t(loc) : 0u;
      float x[CMAX];
#pragma unroll
      for (int j = 0; j < CMAX; ++j) x[j] = wk * gco[j];
      const bool tail = wave_sort_merge<CMAX>(key, bid >= 0, x, lane);
      scatter_runs<CMAX>(gatlas, tail, key, x, lane, stage, C, C);
      continue;
    }
    bool pending = bid >= 0;
    uint64_t pm = __ballot(pending);
    while (pm) {
      const int leader = __ffsll((unsigned long long)pm) - 1;
      const int kb = __shfl(bid, leader, 64), kl = __shfl(loc, leader, 64);
      const bool mine = pending && bid == kb && loc == kl;
      float x[CMAX];
#pragma unroll
      for (int j = 0; j < CMAX; ++j) x[j] = mine ? wk * gco[j] : 0.0f;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int j = 0; j < CMAX; ++j) x[j] += __shfl_xor(x[j], off, 64);
      }
      if ((threadIdx.x & 63) == leader) {
        float* dst = gatlas + (size_t(kb) * 512 + size_t(kl)) * size_t(C);
#pragma unroll
        for (int j = 0; j < CMAX; ++j)
          if (j < C) unsafeAtomicAdd(dst + j, x[j]);
      }
      pending = pending && !mine;
      pm = __ballot(pending);
    }
  }
}

template <int DOM, int LMAX, bool PYR, int MODEL>
__global__ void __launch_bounds__(256) backward_kernel(SceneArgs S, int64_t n, const float* __restrict__ O,
                                                       const float* __restrict__ D,
                                                       const float* __restrict__ grad_rgb,
                                                       const float* __restrict__ grad_dist,
                                                       const float* __restrict__ ups,
                                                       const float* __restrict__ fcd,
                                                       const float* __restrict__ ffv,
                                                       float* __restrict__ gtab, float* __restrict__ gatlas,
                                                       float* __restrict__ partial,
                                                       const float* __restrict__ P, DetRecords det) {
  __shared__ float sA_all[4][64 * kPad];
  __shared__ float sB_all[4][64 * kPad];
  __shared__ float stage_all[4][64 * kStageRow];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t ray = (int64_t(blockIdx.x) * 4 + wave) * 64 + lane;
  const bool in_range = ray < n;
  const float* o = O + 3 * (in_range ? ray : 0);
  const float* d = D + 3 * (in_range ? ray : 0);

  // distortion regulariser (dL/d dist_loss of this ray, 0 if none): running
  // sums of w, w m, w (m W_< - S_<) and w^2 over the samples
  const float gdist = (grad_dist && in_range) ? grad_dist[ray] : 0.0f;
  float dW = 0.0f, dS = 0.0f, dP = 0.0f, dQ = 0.0f;

  // ---------------- pass 1: forward (or the forward's C_d and F, given:
  // the same float32 values, so pass 1 is skipped; not with the regulariser,
  // whose sums pass 1 also takes)
  MarchState m;
  float T = 1.0f, cd[3] = {0.f, 0.f, 0.f}, fv[4] = {0.f, 0.f, 0.f, 0.f};
  int ns = 0, reads = 0;
  if (fcd) {
    if (in_range) {
#pragma unroll
      for (int j = 0; j < 3; ++j) cd[j] = fcd[ray * 3 + j];
#pragma unroll
      for (int j = 0; j < 4; ++j) fv[j] = ffv[ray * 4 + j];
    }
  } else {
  march_init<DOM>(S, o, d, in_range, m);
  for (;;) {
    float u[3], ts;
    int ks;
    bool have = march_next<DOM, PYR>(S, m, false, reads, u, ts, ks);
    if (__ballot(have) == 0) break;
    if (have) {
      float f[8];
      eval_sample<MODEL, DT_F32, LMAX>(S, u, f);
      const float sigma = exp32(f[0]);
      const float e = exp32(-(sigma * S.step));
      const float w = T * (1.0f - e);
      for (int j = 0; j < 3; ++j) cd[j] = __builtin_fmaf(w, f[1 + j], cd[j]);
      for (int j = 0; j < 4; ++j) fv[j] = __builtin_fmaf(w, f[4 + j], fv[j]);
      if (gdist != 0.0f) {
        const float mid = ((float)ks + 0.5f) * S.step;
        dP = __builtin_fmaf(w, mid * dW - dS, dP);
        dQ = __builtin_fmaf(w, w, dQ);
        dW = dW + w;
        dS = __builtin_fmaf(w, mid, dS);
      }
      T = T * e;
      ++ns;
      if (T < S.thr || ns >= S.max_samples) m.done = true;
    }
  }
  }

  float gcd[3], gfv[4];
  if (ups) {
    // dL/dC_d and dL/dF given per ray (the view-dependent MLP's adjoint):
    // no MLP here, no MLP partials
#pragma unroll
    for (int j = 0; j < 3; ++j) gcd[j] = in_range ? ups[ray * 7 + j] : 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) gfv[j] = in_range ? ups[ray * 7 + 3 + j] : 0.0f;
  } else {
    // ---------------- deferred MLP forward + backward (per lane)
    float x[8] = {cd[0], cd[1], cd[2], fv[0], fv[1], fv[2], fv[3], 1.0f};
    float z1[16], h1[16], z2[16], h2[16], oo[3];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float a = P[112 + i];
#pragma unroll
      for (int k = 0; k < 7; ++k) a = __builtin_fmaf(P[i * 7 + k], x[k], a);
      z1[i] = a;
      h1[i] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float a = P[384 + i];
#pragma unroll
      for (int k = 0; k < 16; ++k) a = __builtin_fmaf(P[128 + i * 16 + k], h1[k], a);
      z2[i] = a;
      h2[i] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float a = P[448 + i];
#pragma unroll
      for (int k = 0; k < 16; ++k) a = __builtin_fmaf(P[400 + i * 16 + k], h2[k], a);
      oo[i] = a;
    }
    float gz[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float C = 1.0f / (1.0f + __expf(-(cd[j] + oo[j])));
      const float g = in_range ? grad_rgb[ray * 3 + j] : 0.0f;
      gz[j] = g * C * (1.0f - C);
    }
    float gz2[16], gz1[16], gx[7];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a = 0.0f;
#pragma unroll
      for (int i = 0; i < 3; ++i) a = __builtin_fmaf(P[400 + i * 16 + k], gz[i], a);
      gz2[k] = z2[k] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float a = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) a = __builtin_fmaf(P[128 + i * 16 + k], gz2[i], a);
      gz1[k] = z1[k] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      float a = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) a = __builtin_fmaf(P[i * 7 + k], gz1[i], a);
      gx[k] = a;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) gcd[j] = gz[j] + gx[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) gfv[j] = gx[3 + j];

    // ---------------- MLP weight gradients: sums over the wave on MFMA
    float* sA = sA_all[wave];
    float* sB = sB_all[wave];
    float* part = partial + (int64_t(blockIdx.x) * 4 + wave) * kMlpParams;
    const int qi = lane >> 4, col = lane & 15;
    // W0 (16 x 7) and b0 (column 7 of x is 1)
#pragma unroll
    for (int i = 0; i < 16; ++i) sA[lane * kPad + i] = gz1[i];
#pragma unroll
    for (int j = 0; j < 16; ++j) sB[lane * kPad + j] = j < 8 ? x[j < 8 ? j : 0] : 0.0f;
    __syncthreads();
    {
      bf32x4 r = wave_outer_sum(sA, sB, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * qi + q;
        if (col < 7) part[i * 7 + col] = r[q];
        else if (col == 7) part[112 + i] = r[q];
      }
    }
    __syncthreads();
    // W1 (16 x 16) and b1
#pragma unroll
    for (int i = 0; i < 16; ++i) sA[lane * kPad + i] = gz2[i];
#pragma unroll
    for (int j = 0; j < 16; ++j) sB[lane * kPad + j] = h1[j];
    __syncthreads();
    {
      bf32x4 r = wave_outer_sum(sA, sB, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) part[128 + (4 * qi + q) * 16 + col] = r[q];
      if (lane < 16) {
        float a = 0.0f;
        for (int rr = 0; rr < 64; ++rr) a += sA[rr * kPad + lane];
        part[384 + lane] = a;
      }
    }
    __syncthreads();
    // W2 (3 x 16) and b2
#pragma unroll
    for (int i = 0; i < 16; ++i) sA[lane * kPad + i] = i < 3 ? gz[i < 3 ? i : 0] : 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) sB[lane * kPad + j] = h2[j];
    __syncthreads();
    {
      bf32x4 r = wave_outer_sum(sA, sB, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * qi + q;
        if (i < 3) part[400 + i * 16 + col] = r[q];
      }
      if (lane < 3) {
        float a = 0.0f;
        for (int rr = 0; rr < 64; ++rr) a += sA[rr * kPad + lane];
        part[448 + lane] = a;
      }
    }
  }
  const float Ldist = 2.0f * dP + dQ * (S.step * (1.0f / 3.0f));
  const float Stot = gdist * (2.0f * Ldist) + (gcd[0] * cd[0] + gcd[1] * cd[1] + gcd[2] * cd[2]) +
                     (gfv[0] * fv[0] + gfv[1] * fv[1] + gfv[2] * fv[2] + gfv[3] * fv[3]);

  // ---------------- pass 2: re-march and scatter
  // Every lane takes part in each iteration (lanes without a sample carry a
  // zero gradient) so that coarse levels can merge equal table entries across
  // the wave before the atomics.
  march_init<DOM>(S, o, d, in_range, m);
  T = 1.0f;
  ns = 0;
  float Pc = 0.0f, rW = 0.0f, rS = 0.0f;
  const size_t T_entries = size_t(1) << S.log2T;
  for (;;) {
    float u[3] = {0.f, 0.f, 0.f}, ts;
    int ks;
    const bool have = march_next<DOM, PYR>(S, m, false, reads, u, ts, ks);
    if (__ballot(have) == 0) break;
    float gf[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, wl[LMAX], gff = 0.0f;
    if (have) {
      float f[8];
      if constexpr (MODEL == 1) {
        eval_baked<DT_F32, LMAX>(S, u, f);
      } else {
        int32_t idx_unused[LMAX * 8];
        eval_fused<DT_F32, LMAX, true>(S, u, f, wl, idx_unused);
      }
      const float sigma = exp32(f[0]);
      const float e = exp32(-(sigma * S.step));
      const float w = T * (1.0f - e);
      float s = (gcd[0] * f[1] + gcd[1] * f[2] + gcd[2] * f[3]) +
                (gfv[0] * f[4] + gfv[1] * f[5] + gfv[2] * f[6] + gfv[3] * f[7]);
      if (gdist != 0.0f) {
        // dL_dist/dw_i = 2 sum_j w_j |m_i - m_j| + 2/3 step w_i (prefix sums over j < i)
        const float mid = ((float)ks + 0.5f) * S.step;
        const float pair = (mid * rW - rS) + ((dS - rS - w * mid) - mid * (dW - rW - w));
        s = __builtin_fmaf(gdist, 2.0f * pair + (2.0f / 3.0f) * S.step * w, s);
        rW = rW + w;
        rS = __builtin_fmaf(w, mid, rS);
      }
      Pc = __builtin_fmaf(w, s, Pc);
      const float Tn = T * e;
      const float gsig = S.step * (Tn * s - (Stot - Pc));
      gf[0] = sigma * gsig;
      for (int j = 0; j < 3; ++j) gf[1 + j] = w * gcd[j];
      for (int j = 0; j < 4; ++j) gf[4 + j] = w * gfv[j];
#pragma unroll
      for (int j = 0; j < 8; ++j) gff = __builtin_fmaf(gf[j], f[j], gff);
      T = Tn;
      ++ns;
      if (T < S.thr || ns >= S.max_samples) m.done = true;
    } else {
#pragma unroll
      for (int l = 0; l < LMAX; ++l) wl[l] = 0.0f;
    }
    if constexpr (MODEL == 1) {
      baked_scatter<LMAX>(S, u, have, gf, gtab, gatlas, stage_all[wave]);
      continue;
    }
#pragma unroll
    for (int l = 0; l < LMAX; ++l) {
      if (l >= S.L) break;
      Corners c;
      level_corners(u, S.N[l], S.Nf[l], S.mask, c);
      float gv[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) gv[j] = 0.0f;
      if (have) {
        const void* fb = feat_level<DT_F32>(S.feat, l, S.log2T);
        float v[8][8];
#pragma unroll
        for (int k = 0; k < 8; ++k) Store<DT_F32>::feat(fb, c.idx[k], v[k]);
        float gw = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float acc = 0.0f;
#pragma unroll
          for (int k = 0; k < 8; ++k) acc = __builtin_fmaf(c.w[k], v[k][j], acc);
          gw = __builtin_fmaf(gf[j], acc, gw);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) gv[j] = wl[l] * gf[j];
        gv[8] = wl[l] * (gw - gff);
      }
      float* gbase = gtab + (size_t(l) * T_entries) * 9;
      if (det.off) {
        // deterministic mode: every contribution to its own record
        if (have) {
          const int64_t base = ((det.off[ray] + (ns - 1)) * S.L + l) * 8;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int64_t rec = base + k;
            if (rec >= det.n) break;
            det.keys[rec] = uint32_t(l) * uint32_t(T_entries) + c.idx[k];
            det.order[rec] = uint32_t(rec);
#pragma unroll
            for (int j = 0; j < 9; ++j) det.vals[rec * 9 + j] = c.w[k] * gv[j];
          }
        }
      } else if (S.N[l] >= NGPRT_BW_SORT_MIN_RES) {
        // equal entries summed after a sort across the wave; the last lane
        // of each run issues the atomics
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
          uint32_t key;
          float wk;
          corner_pick(c, k, key, wk);
          float x[9];
#pragma unroll
          for (int j = 0; j < 9; ++j) x[j] = wk * gv[j];
          const bool tail = wave_sort_merge<9>(key, have, x, lane);
          scatter_runs<9>(gbase, tail, key, x, lane, stage_all[wave]);
        }
      } else {
        // sum equal entries over the wave; one lane issues the atomics
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          bool pending = have;
          uint64_t pm = __ballot(pending);
          while (pm) {
            const int leader = __ffsll((unsigned long long)pm) - 1;
            const uint32_t key = __shfl(c.idx[k], leader, 64);
            const bool mine = pending && c.idx[k] == key;
            float x[9];
#pragma unroll
            for (int j = 0; j < 9; ++j) x[j] = mine ? c.w[k] * gv[j] : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
              for (int j = 0; j < 9; ++j) x[j] += __shfl_xor(x[j], off, 64);
            }
            if (lane == leader) {
              float* dst = gbase + size_t(key) * 9;
#pragma unroll
              for (int j = 0; j < 9; ++j) unsafeAtomicAdd(dst + j, x[j]);
            }
            pending = pending && !mine;
            pm = __ballot(pending);
          }
        }
      }
    }
  }
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

size_t backward_workspace_bytes(int64_t n) {
  const int64_t n_waves = (n + 255) / 256 * 4;
  return (size_t(n_waves) + kSumGroups) * kMlpParams * sizeof(float);
}

static bool is_baked_model(const ngprt_ctx* ctx) { return ctx->desc.feature_model == NGPRT_MODEL_BAKED; }

int launch_backward(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                    const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                    float* gtab, float* gatlas, float* gmlp, hipStream_t st) {
  if ((n + 255) / 256 > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays for one launch");
  const size_t need = backward_workspace_bytes(n);
  if (need > ctx->ws_bytes) {
    if (ctx->ws) (void)hipFreeAsync(ctx->ws, st);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (dev_malloc_async((void**)&ctx->ws, need, st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_ALLOC, "backward workspace allocation failed");
    }
    ctx->ws_bytes = need;
  }
  if (ctx->det_grad) {
    if (is_baked_model(ctx))
      return fail(ctx, NGPRT_E_UNSUPPORTED, "deterministic gradients are built for the hash model");
    return launch_backward_det(ctx, n, o, d, grad_rgb, grad_dist, ups, fcd, ffv, gtab, gmlp,
                               reinterpret_cast<float*>(ctx->ws), st);
  }
  return launch_backward_ws(ctx, n, o, d, grad_rgb, grad_dist, ups, fcd, ffv, gtab, gatlas, gmlp,
                            reinterpret_cast<float*>(ctx->ws), st);
}

int launch_backward_ws(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                       const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                       float* gtab, float* gatlas, float* gmlp, float* partial, hipStream_t st,
                       const DetRecords& det) {
  SceneArgs S = scene_args(ctx);
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(ctx, NGPRT_E_SHAPE, "too many rays for one launch");
  const int64_t n_waves = blocks * 4;
  dim3 g = dim3(unsigned(blocks));
  const bool box = ctx->desc.domain == DOM_BOX;
#define NGPRT_BW(DOMV, LM, PY, MD)                                                                 \
  hipLaunchKernelGGL((backward_kernel<DOMV, LM, PY, MD>), g, dim3(256), 0, st, S, n, o, d, grad_rgb,   \
                     grad_dist, ups, fcd, ffv, gtab, gatlas, partial, ctx->mlp, det)
  if (S.model == NGPRT_MODEL_BAKED) {
    // L <= 2 fine levels: coarse rows of at most 12 channels, so the wave
    // sums in the coarse scatter carry 12 values instead of 16
    if (S.L <= 2) {
      if (S.pyr_n > 0) {
        if (box) NGPRT_BW(DOM_BOX, 2, true, 1);
        else NGPRT_BW(DOM_CONTRACT, 2, true, 1);
      } else {
        if (box) NGPRT_BW(DOM_BOX, 2, false, 1);
        else NGPRT_BW(DOM_CONTRACT, 2, false, 1);
      }
    } else if (S.pyr_n > 0) {
      if (box) NGPRT_BW(DOM_BOX, 4, true, 1);
      else NGPRT_BW(DOM_CONTRACT, 4, true, 1);
    } else {
      if (box) NGPRT_BW(DOM_BOX, 4, false, 1);
      else NGPRT_BW(DOM_CONTRACT, 4, false, 1);
    }
  } else if (S.pyr_n > 0) {
    if (box) NGPRT_BW(DOM_BOX, 16, true, 0);
    else NGPRT_BW(DOM_CONTRACT, 16, true, 0);
  } else if (S.L <= 8) {
    if (box) NGPRT_BW(DOM_BOX, 8, false, 0);
    else NGPRT_BW(DOM_CONTRACT, 8, false, 0);
  } else {
    if (box) NGPRT_BW(DOM_BOX, 16, false, 0);
    else NGPRT_BW(DOM_CONTRACT, 16, false, 0);
  }
#undef NGPRT_BW
  int rc = check_launch(ctx, "backward_kernel");
  if (rc || ups) return rc;
  return launch_partial_sums(ctx, partial, n_waves, kMlpParams, partial + size_t(n_waves) * kMlpParams, gmlp, st);
}

int launch_adam(int64_t n, float* p, const float* g, float* m, float* v, int32_t step, float lr, float b1,
                float b2, float eps, hipStream_t st) {
  const double c1 = 1.0 / (1.0 - std::pow(double(b1), double(step)));
  const double c2 = 1.0 / (1.0 - std::pow(double(b2), double(step)));
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(adam_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps,
                     float(c1), float(c2));
  return hipGetLastError() == hipSuccess ? NGPRT_OK : NGPRT_E_HIP;
}

}  // namespace ngprt
