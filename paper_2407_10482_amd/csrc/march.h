// Per-ray march over the sample lattice with the occupancy distance grid
// (Sec. 4.3, Eq. 9), shared by the forward and backward kernels.
//
// Box domain: lattice t_k = t0 + k*step inside the cube ROI; a grid read
// returning G = g > 0 proves the next floor(g * (voxel/step) / |d|) - 1
// lattice points empty (they lie within g voxels of the read point, less
// one step), so the march jumps over them without reading.
// Contracted domain: lattice of equal contracted arc length,
// t_{k+1} = t_k + step / |J(x_k) d|, in the image of the contraction
// x -> (2 - 1/|x|) x/|x| (|x| > 1); a read with g > 0 opens a known-empty
// ball of radius g*voxel - voxel/1024 around the read point, and lattice
// points inside it are visited without a read.  Either way the sampled
// lattice points are exactly those an exhaustive occupancy march samples.
#pragma once

#include "device.h"

namespace ngprt {

struct MarchState {
  float o[3], d[3];
  float t0, t1;       // box: entry/exit
  float t;            // contract: current lattice t
  float rho;          // box: (vox/step)/|d|
  float dn, dn2;      // |d|, |d|^2
  float dt_in;        // contract: step / |d|, the lattice spacing inside the unit ball
  int k;              // lattice index of the next point to visit
  int next_read;      // box: first lattice index not known to be empty
  bool has_ball;      // contract: known-empty ball
  float bc[3], br2;
  float t_lo;         // optional start: contract: lattice points with t < t_lo are not read
                      // (box: the caller sets k to the first lattice point at or after it)
  float t_hi;         // optional end: a lattice point with t > t_hi stops the march
  bool stopped_at_hi; // the march ended at t_hi (and can be resumed)
  bool done;
};

template <int DOM>
__device__ __forceinline__ void march_init(const SceneArgs& S, const float* o, const float* d,
                                           bool in_range, MarchState& m) {
  bool valid = in_range;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.o[a] = in_range ? o[a] : 0.0f;
    m.d[a] = in_range ? d[a] : 0.0f;
    valid = valid && isfinite(m.o[a]) && isfinite(m.d[a]);
  }
  m.dn2 = (m.d[0] * m.d[0] + m.d[1] * m.d[1]) + m.d[2] * m.d[2];
  m.dn = sqrtf(m.dn2);
  m.k = 0;
  m.next_read = 0;
  m.has_ball = false;
  m.t = 0.0f;
  m.t_lo = -__int_as_float(0x7F800000);
  m.t_hi = __int_as_float(0x7F800000);
  m.stopped_at_hi = false;
  if (DOM == DOM_BOX) {
    const float lo = S.lo, hi = -S.lo;
    float t0 = 0.0f, t1 = __int_as_float(0x7F800000);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (m.d[a] != 0.0f) {
        float ta = (lo - m.o[a]) / m.d[a];
        float tb = (hi - m.o[a]) / m.d[a];
        t0 = fmaxf(t0, fminf(ta, tb));
        t1 = fminf(t1, fmaxf(ta, tb));
      } else {
        valid = valid && (m.o[a] >= lo) && (m.o[a] <= hi);
      }
    }
    valid = valid && (t0 < t1) && (m.dn2 > 0.0f);
    m.t0 = t0;
    m.t1 = t1;
    m.rho = S.v_over_step / m.dn;
  } else {
    valid = valid && (m.dn2 > 0.0f);
    m.dt_in = S.step / m.dn;
  }
  m.done = !valid;
}

// Grid-domain position -> grid coordinate u in [0,1]^3 and voxel index.
__device__ __forceinline__ uint32_t voxel_of(const SceneArgs& S, const float p[3], float u[3]) {
  int q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = (p[a] - S.lo) * S.inv_ext;
    int i = (int)floorf(u[a] * S.Rf);
    q[a] = i < 0 ? 0 : (i > S.R - 1 ? S.R - 1 : i);
  }
  return uint32_t(q[0]) + uint32_t(S.R) * (uint32_t(q[1]) + uint32_t(S.R) * uint32_t(q[2]));
}

// Occupancy pyramid level j: the cell of grid coordinate u, and whether it
// is empty (levels x fastest, 32 voxels per word).
__device__ __forceinline__ void pyr_cell(const float u[3], int Rj, int q[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int i = (int)floorf(u[a] * (float)Rj);
    q[a] = i < 0 ? 0 : (i > Rj - 1 ? Rj - 1 : i);
  }
}
__device__ __forceinline__ bool pyr_empty(const SceneArgs& S, int j, const float u[3]) {
  const int Rj = S.pyrR[j];
  int q[3];
  pyr_cell(u, Rj, q);
  const uint32_t w = S.pyr[j][(size_t(q[2]) * Rj + q[1]) * size_t(Rj >> 5) + size_t(q[0] >> 5)];
  return !((w >> (q[0] & 31)) & 1u);
}

// Advance this lane's march to its next occupied lattice point.  Returns
// true with (u, ts, ks) set when a sample was found; sets m.done when the
// ray leaves the domain.
// PYR: the scene marches an occupancy pyramid (S.pyr_n > 0) instead of one
// occupancy grid; a template flag so the single-grid march carries none of it.
// LO: honour m.t_lo in the contracted domain (points before it are visited
// without a read).
template <int DOM, bool PYR, bool LO = false>
__device__ __forceinline__ bool march_next(const SceneArgs& S, MarchState& m, bool naive,
                                           int& reads, float u[3], float& ts, int& ks) {
  while (!m.done) {
    if (m.k >= kMaxLattice) { m.done = true; break; }
    float p[3];
    float tcur;
    if (DOM == DOM_BOX) {
      tcur = m.t0 + (float)m.k * S.step;
      if (!(tcur < m.t1)) { m.done = true; break; }
      if (tcur > m.t_hi) { m.done = true; m.stopped_at_hi = true; break; }
#pragma unroll
      for (int a = 0; a < 3; ++a) p[a] = m.o[a] + tcur * m.d[a];
    } else {
      tcur = m.t;
      if (tcur > m.t_hi) { m.done = true; m.stopped_at_hi = true; break; }
      float x[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = m.o[a] + tcur * m.d[a];
      float r2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
      if (!isfinite(r2)) { m.done = true; break; }
      if (r2 > 1.0f) {
        float r = sqrtf(r2);
        float inv_r = 1.0f / r;
        float s = (2.0f - inv_r) * inv_r;
        float xd = ((x[0] * m.d[0] + x[1] * m.d[1]) + x[2] * m.d[2]) * inv_r;
        if (inv_r < S.step && xd >= 0.0f) { m.done = true; break; }
        float perp2 = fmaxf(m.dn2 - xd * xd, 0.0f);
        float rad = xd * (inv_r * inv_r);
        const float jn = sqrtf((s * s) * perp2 + rad * rad);
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] = s * x[a];
        m.t = tcur + S.step / jn;
      } else {
        // inside the unit ball |J d| = |d|: the same quotient, taken once per ray
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] = x[a];
        m.t = tcur + m.dt_in;
      }
    }
    const int kcur = m.k;
    bool need = true;
    if (!naive && DOM == DOM_CONTRACT && m.has_ball) {
      float e0 = p[0] - m.bc[0], e1 = p[1] - m.bc[1], e2 = p[2] - m.bc[2];
      float dd = (e0 * e0 + e1 * e1) + e2 * e2;
      need = !(dd < m.br2);
    }
    m.k = kcur + 1;
    if (!need) continue;
    if (LO && DOM == DOM_CONTRACT && tcur < m.t_lo) continue;
    const uint32_t v = voxel_of(S, p, u);
    if (PYR) {
      // multi-level occupancy (Eq. 9's s_O branch): levels coarse to fine;
      // reads counts marching points (lattice points checked), whatever the
      // number of levels read there
      ++reads;
      // the coarsest empty level decides.  The distance grid's word carries
      // it for the levels at and above the grid's resolution (one read for
      // the code and G); only when all of those are occupied are the finer
      // levels read, coarse to fine.  The exhaustive march reads level 0.
      int lev = -1;
      uint32_t word = 0;
      if (naive) {
        lev = pyr_empty(S, 0, u) ? 0 : -1;
      } else if (S.pwide) {
        // the finest level is the one below the distance grid: the word also
        // holds the voxel's 8 children there (level-0 cell = the voxel's
        // coordinates doubled plus the child offsets, exactly, since u * 2R
        // and u * R differ by a power of two)
        word = S.pwide[v];
        const uint32_t code = (word >> 9) & 7u;
        if (code) {
          lev = int(code);
        } else {
          int q0[3];
          pyr_cell(u, S.pyrR[0], q0);
          const uint32_t c = uint32_t(q0[0] & 1) | (uint32_t(q0[1] & 1) << 1) | (uint32_t(q0[2] & 1) << 2);
          lev = ((word >> (16 + c)) & 1u) ? -1 : 0;
        }
      } else {
        word = S.grid[v];
        const uint32_t code = (word >> 9) & 7u;
        if (code) {
          lev = S.pyr_jg + int(code) - 1;
        } else {
          for (int j = S.pyr_jg - 1; j >= 0; --j)
            if (pyr_empty(S, j, u)) {
              lev = j;
              break;
            }
        }
      }
      if (lev < 0) {
        ts = tcur;
        ks = kcur;
        if (!naive && DOM == DOM_CONTRACT) m.has_ball = false;
        return true;
      }
      if (naive) continue;
      int Rl = S.pyrR[0];
#pragma unroll
      for (int j = 1; j < kMaxPyr; ++j) Rl = lev == j ? S.pyrR[j] : Rl;
      int qe[3];
      pyr_cell(u, Rl, qe);
      const bool use_g = S.use_dist && Rl < S.R;
      const uint32_t g = use_g ? (word & 0xFFu) : 0u;
      const float vj = (-S.lo - S.lo) / (float)Rl;
      if (DOM == DOM_BOX) {
        float te = __int_as_float(0x7F800000);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (m.d[a] != 0.0f) {
            const float b = S.lo + (float)(qe[a] + (m.d[a] > 0.0f ? 1 : 0)) * vj;
            te = fminf(te, (b - m.o[a]) / m.d[a]);
          }
        }
        const float jo = floorf((te - tcur) / S.step);
        int jump = jo >= 1.0f ? (jo < (float)kMaxLattice ? (int)jo : kMaxLattice) : 1;
        if (use_g && g > 0) {
          const float jf = floorf((float)g * m.rho);
          const int jg = jf < (float)kMaxLattice ? (int)jf : kMaxLattice;
          jump = jg > jump ? jg : jump;
        }
        m.k = kcur + jump;
      } else {
        float r = __int_as_float(0x7F800000);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float lower = S.lo + (float)qe[a] * vj;
          const float upper = S.lo + (float)(qe[a] + 1) * vj;
          r = fminf(r, fminf(p[a] - lower, upper - p[a]));
        }
        const float margin = S.vox * 0.0009765625f;
        const float ro = r - margin;
        const float rg = (use_g && g > 0) ? (float)g * S.vox - margin : -__int_as_float(0x7F800000);
        const float rb = fmaxf(ro, rg);
        if (rb > 0.0f) {
          m.br2 = rb * rb;
          m.bc[0] = p[0]; m.bc[1] = p[1]; m.bc[2] = p[2];
          m.has_ball = true;
        } else {
          m.has_ball = false;
        }
      }
      continue;
    }
    const uint32_t word = S.grid[v];
    ++reads;
    if (word & 0x100u) {
      ts = tcur;
      ks = kcur;
      if (!naive && DOM == DOM_CONTRACT) m.has_ball = false;
      return true;
    }
    const uint32_t g = word & 0xFFu;
    if (!naive) {
      if (DOM == DOM_BOX) {
        if (g > 0) {
          const float jf = floorf((float)g * m.rho);
          const int jump = jf < (float)kMaxLattice ? (int)jf : kMaxLattice;
          m.k = kcur + (jump > 1 ? jump : 1);
        }
      } else {
        if (g > 0) {
          float rb = (float)g * S.vox - S.vox * 0.0009765625f;
          m.br2 = rb * rb;
          m.bc[0] = p[0]; m.bc[1] = p[1]; m.bc[2] = p[2];
          m.has_ball = true;
        } else {
          m.has_ball = false;
        }
      }
    }
  }
  return false;
}

}  // namespace ngprt
