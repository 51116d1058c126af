// Device-side building blocks of the NGP-RT render path for gfx950.
//
// Everything on the decision chain (positions, voxel/corner indices,
// trilinear weights, interpolated density and logit, softmax, density
// activation, transmittance) is written with plain float32 operators and
// explicit fused multiply-adds where the chain specifies one (exp32, the
// corner sums, the softmax sums); the library is compiled with
// -ffp-contract=off and correctly rounded division/sqrt, so each operator is
// one IEEE binary32 operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace ngprt {

// ---------------------------------------------------------------------------
// exponential of the decision chain: Cody-Waite reduction by ln 2 (split in a
// 9-bit head and a float32 tail), degree-7 Taylor polynomial of e^r by
// Horner with fused multiply-adds, and exact scaling by 2^k.
// (The special cases branch: a wave almost never diverges on them, and
// taking them by selects after the polynomial measured slower, 154.2 ->
// 149.2 frames/s on the 8-view 1080p workload, for the extra VALU work.)
__device__ __forceinline__ float exp32(float x) {
  if (x != x) return x;
  if (x > 88.0f) return __int_as_float(0x7F800000);
  if (x < -86.0f) return 0.0f;
  const float log2e = __int_as_float(0x3FB8AA3B);
  const float ln2_hi = __int_as_float(0x3F318000);
  const float ln2_lo = __int_as_float(0xB95E8083);
  float k = floorf(__builtin_fmaf(x, log2e, 0.5f));
  float r = __builtin_fmaf(-k, ln2_lo, __builtin_fmaf(-k, ln2_hi, x));
  float p = __int_as_float(0x39500D01);                    // 1/7!
  p = __builtin_fmaf(p, r, __int_as_float(0x3AB60B61));    // 1/6!
  p = __builtin_fmaf(p, r, __int_as_float(0x3C088889));    // 1/5!
  p = __builtin_fmaf(p, r, __int_as_float(0x3D2AAAAB));    // 1/4!
  p = __builtin_fmaf(p, r, __int_as_float(0x3E2AAAAB));    // 1/3!
  p = __builtin_fmaf(p, r, 0.5f);
  p = __builtin_fmaf(p, r, 1.0f);
  p = __builtin_fmaf(p, r, 1.0f);
  int n = (int)k;
  return p * __int_as_float((n + 127) << 23);
}

// float32 -> bfloat16 bits, round to nearest even (NaN -> 0x7FC0).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t b = __float_as_uint(x);
  if (x != x) return 0x7FC0;
  uint32_t lsb = (b >> 16) & 1u;
  return uint16_t((b + 0x7FFFu + lsb) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// Spatial hash of a corner (multi-resolution hash encoding): products modulo
// 2^32, xor, then the low log2(T) bits.
__device__ __forceinline__ uint32_t hash3(uint32_t x, uint32_t y, uint32_t z, uint32_t mask) {
  return ((x * 1u) ^ (y * 2654435761u) ^ (z * 805459861u)) & mask;
}

// ---------------------------------------------------------------------------
// Table storage: features [L][T][8] and logits [L][T] in the storage dtype.

template <int DT> struct Store;

// Read-only views in the constant address space: a load through one with a
// wave-uniform address is a scalar load (scalar cache; no vector-memory
// instruction).  The render kernels never write the tables.
typedef float ev_f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t ev_u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t ev_u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const float c_f32;
typedef __attribute__((address_space(4))) const ev_f32x4 c_f32x4;
typedef __attribute__((address_space(4))) const uint32_t c_u32;
typedef __attribute__((address_space(4))) const ev_u32x2 c_u32x2;
typedef __attribute__((address_space(4))) const ev_u32x4 c_u32x4;

// Accessors take the level's uniform base pointer and a 32-bit entry index,
// so a gather is one global load with a scalar base and a 32-bit offset.
// The _s forms take a wave-uniform index and read by scalar loads.
template <> struct Store<DT_F32> {
  static constexpr int kRow = 32;
  __device__ static __forceinline__ float logit(const void* lbase, uint32_t i) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(lbase) + (i << 2));
  }
  __device__ static __forceinline__ void feat(const void* lbase, uint32_t i, float v[8]) {
    const float4* q = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(lbase) + (i << 5));
    float4 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
  __device__ static __forceinline__ float logit_s(const void* lbase, uint32_t i) {
    return ((c_f32*)lbase)[i];
  }
  __device__ static __forceinline__ void feat_s(const void* lbase, uint32_t i, float v[8]) {
    c_f32x4* q = (c_f32x4*)(reinterpret_cast<const char*>(lbase) + (size_t(i) << 5));
    const ev_f32x4 a = q[0], b = q[1];
    v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
    v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
  }
};

template <> struct Store<DT_BF16> {
  static constexpr int kRow = 16;
  __device__ static __forceinline__ float logit(const void* lbase, uint32_t i) {
    return __uint_as_float(uint32_t(*reinterpret_cast<const uint16_t*>(
                               reinterpret_cast<const char*>(lbase) + (i << 1)))
                           << 16);
  }
  __device__ static __forceinline__ void feat(const void* lbase, uint32_t i, float v[8]) {
    uint4 w = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(lbase) + (i << 4));
    unpack(w.x, w.y, w.z, w.w, v);
  }
  __device__ static __forceinline__ void unpack(uint32_t x, uint32_t y, uint32_t z, uint32_t w,
                                                float v[8]) {
    v[0] = __uint_as_float(x << 16); v[1] = __uint_as_float(x & 0xFFFF0000u);
    v[2] = __uint_as_float(y << 16); v[3] = __uint_as_float(y & 0xFFFF0000u);
    v[4] = __uint_as_float(z << 16); v[5] = __uint_as_float(z & 0xFFFF0000u);
    v[6] = __uint_as_float(w << 16); v[7] = __uint_as_float(w & 0xFFFF0000u);
  }
  // the dword holding the logit (a level holds T >= 16 entries, so the dword
  // lies inside the level)
  __device__ static __forceinline__ float logit_s(const void* lbase, uint32_t i) {
    const uint32_t w = ((c_u32*)lbase)[i >> 1];
    return __uint_as_float((i & 1u) ? (w & 0xFFFF0000u) : (w << 16));
  }
  __device__ static __forceinline__ void feat_s(const void* lbase, uint32_t i, float v[8]) {
    const ev_u32x4 w = *(c_u32x4*)(reinterpret_cast<const char*>(lbase) + (size_t(i) << 4));
    unpack(w[0], w[1], w[2], w[3], v);
  }
};

// OCP E4M3FN codes -> float32 (exact) with gfx950's OCP conversion
// (v_cvt_scalef32_pk_f32_fp8, scale 1): two codes per instruction.
typedef float fp8pair __attribute__((ext_vector_type(2)));

__device__ __forceinline__ fp8pair fp8x2_decode(uint32_t w, bool hi) {
  return hi ? __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)w, 1.0f, true)
            : __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)w, 1.0f, false);
}

template <> struct Store<DT_FP8> {
  static constexpr int kRow = 8;
  __device__ static __forceinline__ float logit(const void* lbase, uint32_t i) {
    return fp8x2_decode(*(reinterpret_cast<const uint8_t*>(lbase) + i), false)[0];
  }
  __device__ static __forceinline__ void feat(const void* lbase, uint32_t i, float v[8]) {
    uint2 w = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(lbase) + (i << 3));
    unpack(w.x, w.y, v);
  }
  __device__ static __forceinline__ void unpack(uint32_t x, uint32_t y, float v[8]) {
    fp8pair a = fp8x2_decode(x, false), b = fp8x2_decode(x, true);
    fp8pair c = fp8x2_decode(y, false), d = fp8x2_decode(y, true);
    v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
    v[4] = c[0]; v[5] = c[1]; v[6] = d[0]; v[7] = d[1];
  }
  // the dword holding the logit (a level holds T >= 16 entries, so the dword
  // lies inside the level)
  __device__ static __forceinline__ float logit_s(const void* lbase, uint32_t i) {
    const uint32_t w = ((c_u32*)lbase)[i >> 2];
    return fp8x2_decode((w >> ((i & 3u) * 8u)) & 0xFFu, false)[0];
  }
  __device__ static __forceinline__ void feat_s(const void* lbase, uint32_t i, float v[8]) {
    const ev_u32x2 w = *(c_u32x2*)(reinterpret_cast<const char*>(lbase) + (size_t(i) << 3));
    unpack(w[0], w[1], v);
  }
};

// level base pointers of the feature and logit arrays
template <int DT>
__device__ __forceinline__ const void* feat_level(const void* feat, int l, int log2T) {
  return reinterpret_cast<const char*>(feat) + ((size_t(l) << log2T) * Store<DT>::kRow);
}
template <int DT>
__device__ __forceinline__ const void* logit_level(const void* logit, int l, int log2T) {
  return reinterpret_cast<const char*>(logit) + ((size_t(l) << log2T) * (Store<DT>::kRow / 8));
}

// ---------------------------------------------------------------------------
// One hash level at grid coordinate u: corner indices and trilinear weights.
struct Corners {
  uint32_t idx[8];
  float w[8];
  uint32_t key0, key1;   // the cell (i0 of each axis, < 2^20): x | y << 20, y >> 12 | z << 8
};

__device__ __forceinline__ void level_corners(const float u[3], int N, float Nf, uint32_t mask,
                                              Corners& c) {
  int i0[3];
  float f[3], g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float p = u[a] * Nf;
    int i = (int)floorf(p);
    i = i < 0 ? 0 : (i > N - 1 ? N - 1 : i);
    i0[a] = i;
    // fraction rounded once: accurate to half an ulp of f at any resolution
    f[a] = __builtin_fmaf(u[a], Nf, -(float)i);
    g[a] = 1.0f - f[a];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
    c.w[k] = ((bx ? f[0] : g[0]) * (by ? f[1] : g[1])) * (bz ? f[2] : g[2]);
    c.idx[k] = hash3(uint32_t(i0[0] + bx), uint32_t(i0[1] + by), uint32_t(i0[2] + bz), mask);
  }
  c.key0 = uint32_t(i0[0]) | (uint32_t(i0[1]) << 20);
  c.key1 = (uint32_t(i0[1]) >> 12) | (uint32_t(i0[2]) << 8);
}

// Lookup + attention at grid coordinate u, in one pass over the levels.
// Per level: 8 corners, each gathering its feature row and logit; the
// interpolated logit a_l enters a softmax across levels (Eq. 8, softmax
// reading) taken with a running maximum m (online softmax, Milakov and
// Gimelshein 2018): d = a_l - m, x = exp32(-|d|); when d > 0 the sums so far
// are scaled by x and e_l = 1 (a_l is the new maximum), else e_l = x; then
// S = fma(S, scale, e_l) and N_j = fma(e_l, v_l[j], N_j * scale).
// fused_j = N_j / S, and S >= 1, so no sample's softmax underflows whatever
// the offset of its logits.  Each corner sum is acc = fma(w_k, v_k, acc)
// from acc = 0, corners in order.  Optionally the
// attention weights exp32(a_l - m) / S [L] and corner indices [L][8].
// When every active lane of the wave samples the same cell of a level (most
// of the time on the coarse levels: the wave's rays are an 8x8 pixel tile),
// the eight rows come in once by scalar loads instead of 24 vector loads;
// the arithmetic is the same.
#ifndef NGPRT_LEVEL_UNROLL
#define NGPRT_LEVEL_UNROLL 1
#endif
// storage types (bit DT) whose lookups read a wave-shared cell by scalar
// loads: F32 only (BF16 and FP8 rows read that way need their unpacking on
// the scalar ALU, and measured slower: 42.6 -> 44.6 ms and 41.3 -> 43.3 ms
// on the 8-view 1080p workload, against 51.3 -> 46.6 ms for F32)
#ifndef NGPRT_SHARED_CELL
#define NGPRT_SHARED_CELL 1
#endif

template <int DT, int LMAX, bool DEBUG = false>
__device__ __forceinline__ void eval_fused(const SceneArgs& S, const float u[3], float fused[8],
                                           float* wout = nullptr, int32_t* idxout = nullptr) {
  float run_max = -__int_as_float(0x7F800000), esum = 0.0f, num0 = 0.0f;
  float num[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // a rolled level loop: per-level constants come in by scalar loads instead
  // of being held in (and spilled from) scalar registers across the march
#pragma unroll NGPRT_LEVEL_UNROLL
  for (int l = 0; l < LMAX; ++l) {
    if (l < S.L) {
      Corners c;
      level_corners(u, S.N[l], S.Nf[l], S.mask, c);
      const void* fb = feat_level<DT>(S.feat, l, S.log2T);
      const void* lb = logit_level<DT>(S.logit, l, S.log2T);
      float acc[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) acc[j] = 0.0f;
      // one cell for the whole wave (common on the coarse levels, where a
      // wave's 64 neighbouring rays sample close together): its eight rows
      // are read once by scalar loads and every lane accumulates from scalar
      // registers, in the same order as the per-lane gather below
      bool shared = false;
      if constexpr ((NGPRT_SHARED_CELL >> DT) & 1) {
        const uint32_t k0 = __builtin_amdgcn_readfirstlane(c.key0);
        const uint32_t k1 = __builtin_amdgcn_readfirstlane(c.key1);
        shared = __ballot(c.key0 != k0 || c.key1 != k1) == 0ull;
      }
      if (shared) {
        uint32_t ik[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          ik[k] = __builtin_amdgcn_readfirstlane(c.idx[k]);
          // opaque, so that the compiler keeps the scalar index instead of
          // substituting the lane's own (equal) vector index
          asm volatile("" : "+s"(ik[k]));
        }
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          float v[4][8], lg[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            Store<DT>::feat_s(fb, ik[4 * g + k], v[k]);
            lg[k] = Store<DT>::logit_s(lb, ik[4 * g + k]);
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float wk = c.w[4 * g + k];
            acc[8] = __builtin_fmaf(wk, lg[k], acc[8]);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_fmaf(wk, v[k][j], acc[j]);
          }
        }
      } else {
        // two groups of four corners keep the gathered rows in flight within
        // the register budget
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          float v[4][8], lg[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            Store<DT>::feat(fb, c.idx[4 * g + k], v[k]);
            lg[k] = Store<DT>::logit(lb, c.idx[4 * g + k]);
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float wk = c.w[4 * g + k];
            acc[8] = __builtin_fmaf(wk, lg[k], acc[8]);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_fmaf(wk, v[k][j], acc[j]);
          }
        }
      }
      if (DT == DT_FP8) {
#pragma unroll
        for (int j = 0; j < 9; ++j) acc[j] = S.scale[l][j] * acc[j];
      }
      const float a = acc[8];
      const float dl = a - run_max;
      const float x = exp32(-fabsf(dl));
      const bool up = dl > 0.0f;
      const float sc = up ? x : 1.0f;
      const float e = up ? 1.0f : x;
      run_max = up ? a : run_max;
      esum = __builtin_fmaf(esum, sc, e);
      num0 = __builtin_fmaf(e, acc[0], num0 * sc);
#pragma unroll
      for (int j = 0; j < 7; ++j) num[j] = __builtin_fmaf(e, acc[1 + j], num[j] * sc);
      if (DEBUG) {
        wout[l] = a;
#pragma unroll
        for (int k = 0; k < 8; ++k) idxout[l * 8 + k] = int32_t(c.idx[k]);
      }
    }
  }
  fused[0] = num0 / esum;
  const float inv = 1.0f / esum;
#pragma unroll
  for (int j = 0; j < 7; ++j) fused[1 + j] = num[j] * inv;
  if (DEBUG) {
#pragma unroll
    for (int l = 0; l < LMAX; ++l)
      if (l < S.L) wout[l] = exp32(wout[l] - run_max) / esum;
  }
}

// ---------------------------------------------------------------------------
// Baked feature model (Sec. 4.1 Eq. 6, Sec. 4.2 Eq. 7-8): a block-sparse
// coarse vertex grid of resolution L_C holds the deferred features f~ and
// the attention parameters a = (omega_l, beta_l); L fine hash levels hold
// 8-channel features f^_l.  f = f~ + [sum_l g(omega_l) sigma^_l,
// sum_l g(beta_l) c^_l, sum_l g(beta_l) v^_l] with g the sigmoid.
//
// Coarse vertex v lives in block (v >> 3) (per axis) at local offset v & 7;
// the block's atlas row comes from the index grid (-1: empty block, whose
// vertices take the default vector).  Atlas rows hold Cpad >= 8 + 2L floats.
// Decision chain: every coarse channel acc = fma(w_k, v_k, acc) (k = 0..7,
// from 0); fine density as the hash levels; g = 1 / (1 + exp32(-a));
// f_0 = f~_0, then f_0 = fma(g_omega_l, sigma^_l, f_0) in level order.
__device__ __forceinline__ float sigmoid32(float a) { return 1.0f / (1.0f + exp32(-a)); }

//
// GEN: the aggregation variants of the ablation (Shared-Att, spatially
// invariant parameters, SUM): level l's two gate parameters are coarse
// channel S.gidx[l][m] or, where that is -1, the constant S.gconst[l][m];
// rows may then be 8 floats.
template <int DT, int LMAX, bool DEBUG = false, bool GEN = false>
__device__ __forceinline__ void eval_baked(const SceneArgs& S, const float u[3], float fused[8],
                                           float* wout = nullptr, int32_t* idxout = nullptr) {
  static_assert(LMAX <= 4, "the coarse row holds at most 16 channels");
  constexpr int CMAX = 8 + 2 * LMAX;
  int i0[3];
  float f[3], g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float p = u[a] * S.LCf;
    int i = (int)floorf(p);
    i = i < 0 ? 0 : (i > S.LC - 1 ? S.LC - 1 : i);
    i0[a] = i;
    f[a] = __builtin_fmaf(u[a], S.LCf, -(float)i);
    g[a] = 1.0f - f[a];
  }
  float co[CMAX];
#pragma unroll
  for (int j = 0; j < CMAX; ++j) co[j] = 0.0f;
  const bool wide = S.Cpad > 12;      // rows of 16 floats (L = 3, 4), else 12
  // corners one after another (rolled): each brings a whole row of up to 16
  // floats, and holding several in flight would spill
#ifndef NGPRT_COARSE_UNROLL
#define NGPRT_COARSE_UNROLL 1
#endif
#pragma unroll NGPRT_COARSE_UNROLL
  for (int k = 0; k < 8; ++k) {
    const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
    const int vx = i0[0] + bx, vy = i0[1] + by, vz = i0[2] + bz;
    const int bid = S.cidx[((vz >> 3) * S.nb + (vy >> 3)) * S.nb + (vx >> 3)];
    const float wk = ((bx ? f[0] : g[0]) * (by ? f[1] : g[1])) * (bz ? f[2] : g[2]);
    float v[16];
    if (bid >= 0) {
      const float4* row = reinterpret_cast<const float4*>(
          S.catlas + (size_t(bid) * 512 + size_t(((vz & 7) * 8 + (vy & 7)) * 8 + (vx & 7))) * S.Cpad);
      float4 q0 = row[0], q1 = row[1];
      float4 q2 = (!GEN || S.Cpad > 8) ? row[2] : make_float4(0.f, 0.f, 0.f, 0.f);
      float4 q3 = wide ? row[3] : make_float4(0.f, 0.f, 0.f, 0.f);
      v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
      v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
      v[8] = q2.x; v[9] = q2.y; v[10] = q2.z; v[11] = q2.w;
      v[12] = q3.x; v[13] = q3.y; v[14] = q3.z; v[15] = q3.w;
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = S.cdef[j];
    }
#pragma unroll
    for (int j = 0; j < CMAX; ++j) co[j] = __builtin_fmaf(wk, v[j], co[j]);
  }
  float f0 = co[0];
  float fc[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) fc[j] = co[1 + j];
  // fine levels, rolled; the level's attention parameters are picked by
  // selects (no dynamically indexed register array)
#pragma unroll 1
  for (int l = 0; l < LMAX; ++l) {
    if (l < S.L) {
      Corners c;
      level_corners(u, S.N[l], S.Nf[l], S.mask, c);
      const void* fb = feat_level<DT>(S.feat, l, S.log2T);
      float acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = 0.0f;
#pragma unroll
      for (int gq = 0; gq < 2; ++gq) {
        float v[4][8];
#pragma unroll
        for (int k = 0; k < 4; ++k) Store<DT>::feat(fb, c.idx[4 * gq + k], v[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float wk = c.w[4 * gq + k];
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[j] = __builtin_fmaf(wk, v[k][j], acc[j]);
        }
      }
      if (DT == DT_FP8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = S.scale[l][j] * acc[j];
      }
      float aw, ab;
      if constexpr (GEN) {
        const int iw = S.gidx[l][0], ib = S.gidx[l][1];
        aw = S.gconst[l][0];
        ab = S.gconst[l][1];
#pragma unroll
        for (int j = 8; j < CMAX; ++j) {
          aw = iw == j ? co[j] : aw;
          ab = ib == j ? co[j] : ab;
        }
      } else {
        aw = co[8];
        ab = co[9];
#pragma unroll
        for (int q = 1; q < LMAX; ++q) {
          aw = l == q ? co[8 + 2 * q] : aw;
          ab = l == q ? co[9 + 2 * q] : ab;
        }
      }
      const float gw = sigmoid32(aw);
      const float gb = sigmoid32(ab);
      f0 = __builtin_fmaf(gw, acc[0], f0);
#pragma unroll
      for (int j = 0; j < 7; ++j) fc[j] = __builtin_fmaf(gb, acc[1 + j], fc[j]);
      if (DEBUG) {
#pragma unroll
        for (int q = 0; q < LMAX; ++q)
          if (q == l) {
            wout[q] = gw;
#pragma unroll
            for (int k = 0; k < 8; ++k) idxout[q * 8 + k] = int32_t(c.idx[k]);
          }
      }
    }
  }
  fused[0] = f0;
#pragma unroll
  for (int j = 0; j < 7; ++j) fused[1 + j] = fc[j];
}

// One sample's fused deferred feature under the scene's feature model.
// MODEL: bit 0 = baked, bit 2 = its ablation aggregations (GEN).
template <int MODEL, int DT, int LMAX, bool DEBUG = false>
__device__ __forceinline__ void eval_sample(const SceneArgs& S, const float u[3], float fused[8],
                                            float* wout = nullptr, int32_t* idxout = nullptr) {
  if constexpr ((MODEL & 1) != 0)
    eval_baked<DT, LMAX, DEBUG, (MODEL & 4) != 0>(S, u, fused, wout, idxout);
  else
    eval_fused<DT, LMAX, DEBUG>(S, u, fused, wout, idxout);
}

}  // namespace ngprt
