// Occupancy distance grid G on the GPU (Sec. 4.3, Eq. 9).
//
// G_p = min(255, floor(box-gap distance from voxel p to the nearest
// occupied voxel)), in voxel units.  The box gap to an occupied voxel q
// equals the Euclidean distance from p to the 3x3x3 block around q, so G is
// the integer square root of the squared Euclidean distance transform of the
// 26-dilated occupancy.  The transform is separable and exact in integers:
// per-row distance along x, then min over y' of f + (y - y')^2, then the
// same along z.  Each pass is a plain brute-force minimum over one grid line
// (R <= 1024), with lanes along x so every load is coalesced.
//
// Packed grid word (uint16): low byte G, bit 8 set when the voxel is occupied.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ngprt {

constexpr int kInf = 1 << 28;

__global__ void dilate_kernel(const uint8_t* __restrict__ occ, uint8_t* __restrict__ dil, int R) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(R) * R * R;
  if (v >= n) return;
  const int x = int(v % R), y = int((v / R) % R), z = int(v / (int64_t(R) * R));
  uint8_t any = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= R) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= R) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx;
        if (xx < 0 || xx >= R) continue;
        any |= occ[(int64_t(zz) * R + yy) * R + xx] != 0;
      }
    }
  }
  dil[v] = any;
}

// one thread per (y, z) row: squared distance along x to the nearest set voxel
__global__ void edt_x_kernel(const uint8_t* __restrict__ dil, int* __restrict__ f, int R) {
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= int64_t(R) * R) return;
  const uint8_t* src = dil + row * R;
  int* dst = f + row * R;
  int last = -1;
  for (int x = 0; x < R; ++x) {
    if (src[x]) last = x;
    dst[x] = last >= 0 ? (x - last) : kInf;
  }
  last = -1;
  for (int x = R - 1; x >= 0; --x) {
    if (src[x]) last = x;
    int dl = dst[x];
    int dr = last >= 0 ? (last - x) : kInf;
    int m = dl < dr ? dl : dr;
    dst[x] = m >= kInf ? kInf : m * m;
  }
}

// f_out[x, y, z] = min_{y'} f_in[x, y', z] + (y - y')^2   (axis = 1)
// f_out[x, y, z] = min_{z'} f_in[x, y, z'] + (z - z')^2   (axis = 2)
__global__ void edt_line_kernel(const int* __restrict__ fin, int* __restrict__ fout, int R, int axis) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(R) * R * R;
  if (v >= n) return;
  const int64_t stride = axis == 1 ? int64_t(R) : int64_t(R) * R;
  const int c = axis == 1 ? int((v / R) % R) : int(v / (int64_t(R) * R));
  const int64_t base = v - int64_t(c) * stride;
  int best = kInf;
  for (int j = 0; j < R; ++j) {
    const int a = fin[base + int64_t(j) * stride];
    const int dd = (c - j) * (c - j);
    const int cand = a + dd;
    best = cand < best ? cand : best;
  }
  fout[v] = best > kInf ? kInf : best;
}

__device__ __forceinline__ int isqrt_exact(int v) {
  int r = (int)sqrtf((float)v);
  while (r > 0 && r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

__global__ void pack_grid_kernel(const uint8_t* __restrict__ occ, const uint8_t* __restrict__ dil,
                                 const int* __restrict__ f, const uint8_t* __restrict__ given,
                                 uint16_t* __restrict__ grid, int64_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint32_t g;
  if (given) {
    g = given[v];
  } else if (dil[v]) {
    g = 0;
  } else {
    int r = isqrt_exact(f[v]);
    g = uint32_t(r > 255 ? 255 : r);
  }
  grid[v] = uint16_t(g | (occ[v] ? 0x100u : 0u));
}

__global__ void unpack_dist_kernel(const uint16_t* __restrict__ grid, uint8_t* __restrict__ out,
                                   int64_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  out[v] = uint8_t(grid[v] & 0xFFu);
}

static unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

int launch_build_distance(ngprt_ctx* ctx, const uint8_t* occ, const uint8_t* dist, hipStream_t st) {
  const int R = ctx->desc.occ_res;
  const int64_t n = int64_t(R) * R * R;
  if (dist) {
    hipLaunchKernelGGL(pack_grid_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, occ, nullptr,
                       nullptr, dist, ctx->grid, n);
    return check_launch(ctx, "pack_grid_kernel");
  }
  uint8_t* dil = nullptr;
  int* f0 = nullptr;
  int* f1 = nullptr;
  if (dev_malloc_async((void**)&dil, size_t(n), st) != hipSuccess ||
      dev_malloc_async((void**)&f0, size_t(n) * sizeof(int), st) != hipSuccess ||
      dev_malloc_async((void**)&f1, size_t(n) * sizeof(int), st) != hipSuccess) {
    if (dil) (void)hipFreeAsync(dil, st);
    if (f0) (void)hipFreeAsync(f0, st);
    (void)hipGetLastError();
    return fail(ctx, NGPRT_E_ALLOC, "distance grid scratch allocation failed");
  }
  int rc = NGPRT_OK;
  hipLaunchKernelGGL(dilate_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, occ, dil, R);
  if ((rc = check_launch(ctx, "dilate_kernel")) == NGPRT_OK) {
    hipLaunchKernelGGL(edt_x_kernel, dim3(blocks_for(int64_t(R) * R, 256)), dim3(256), 0, st, dil,
                       f0, R);
    rc = check_launch(ctx, "edt_x_kernel");
  }
  if (rc == NGPRT_OK) {
    hipLaunchKernelGGL(edt_line_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, f0, f1, R, 1);
    rc = check_launch(ctx, "edt_line_kernel(y)");
  }
  if (rc == NGPRT_OK) {
    hipLaunchKernelGGL(edt_line_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, f1, f0, R, 2);
    rc = check_launch(ctx, "edt_line_kernel(z)");
  }
  if (rc == NGPRT_OK) {
    hipLaunchKernelGGL(pack_grid_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, occ, dil, f0,
                       nullptr, ctx->grid, n);
    rc = check_launch(ctx, "pack_grid_kernel");
  }
  (void)hipFreeAsync(dil, st);
  (void)hipFreeAsync(f0, st);
  (void)hipFreeAsync(f1, st);
  return rc;
}

int launch_export_distance(ngprt_ctx* ctx, uint8_t* out, hipStream_t st) {
  const int R = ctx->desc.occ_res;
  const int64_t n = int64_t(R) * R * R;
  hipLaunchKernelGGL(unpack_dist_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctx->grid, out, n);
  return check_launch(ctx, "unpack_dist_kernel");
}

// ---------------------------------------------------------------------------
// Multi-level occupancy: bit grids (x fastest, 32 voxels per word; R is a
// multiple of 32, so voxel v sits in word v >> 5 at bit v & 31).
__global__ void pyr_pack_kernel(const uint8_t* __restrict__ occ, uint32_t* __restrict__ out,
                                int64_t n_words) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  const uint8_t* src = occ + w * 32;
  uint32_t bits = 0;
  for (int i = 0; i < 32; ++i) bits |= (src[i] != 0 ? 1u : 0u) << i;
  out[w] = bits;
}

// level of resolution Rc from the level of resolution 2 Rc: a voxel is
// occupied when any of its 2x2x2 children is
__global__ void pyr_pool_kernel(const uint32_t* __restrict__ fine, uint32_t* __restrict__ coarse,
                                int Rc) {
  const int64_t wpr = Rc >> 5;                       // words per coarse row
  const int64_t n_words = int64_t(Rc) * Rc * wpr;
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  const int64_t xw = w % wpr;
  const int64_t y = (w / wpr) % Rc;
  const int64_t z = w / (wpr * Rc);
  const int64_t Rf = 2 * int64_t(Rc), wpr_f = Rf >> 5;
  uint64_t acc = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      const int64_t row = ((2 * z + dz) * Rf + (2 * y + dy)) * wpr_f;
      acc |= uint64_t(fine[row + 2 * xw]) | (uint64_t(fine[row + 2 * xw + 1]) << 32);
    }
  uint32_t bits = 0;
  for (int i = 0; i < 32; ++i)
    if ((acc >> (2 * i)) & 3u) bits |= 1u << i;
  coarse[w] = bits;
}

__global__ void pyr_unpack_kernel(const uint32_t* __restrict__ bits, uint8_t* __restrict__ out, int64_t n) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  out[v] = uint8_t((bits[v >> 5] >> (v & 31)) & 1u);
}

// Level codes of the march (Eq. 9's multi-level occupancy): for every voxel
// of the distance grid (pyramid level jg, resolution R), the coarsest level
// j >= jg whose cell holding the voxel is empty, as 1 + j - jg in bits 9-11
// of the voxel's word (0: occupied at every level >= jg).  Level j's cell is
// the voxel's coordinates shifted right by j - jg (the resolutions halve).
// With jg == 1 the finest level holds exactly the voxel's 2x2x2 children:
// wide (when given) gets the word in bits 0-15 and child (dx, dy, dz)'s
// occupancy in bit 16 + dx + 2 dy + 4 dz.
struct PyrLevels {
  const uint32_t* bits[kMaxPyr];
};

__global__ void pyr_code_kernel(uint16_t* __restrict__ grid, uint32_t* __restrict__ wide, int R, int jg,
                                int nl, PyrLevels P) {
  const int64_t n = int64_t(R) * R * R;
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int x = int(v % R), y = int((v / R) % R), z = int(v / (int64_t(R) * R));
  uint32_t code = 0;
  for (int j = nl - 1; j >= jg; --j) {
    const int m = j - jg, Rj = R >> m;
    const int cx = x >> m, cy = y >> m, cz = z >> m;
    const uint32_t w = P.bits[j][(size_t(cz) * Rj + cy) * size_t(Rj >> 5) + size_t(cx >> 5)];
    if (!((w >> (cx & 31)) & 1u)) {
      code = uint32_t(1 + m);
      break;
    }
  }
  const uint16_t word = uint16_t((grid[v] & 0x1FFu) | (code << 9));
  grid[v] = word;
  if (wide) {
    const int Rf = 2 * R, wpr = Rf >> 5;
    uint32_t kids = 0;
    for (int c = 0; c < 8; ++c) {
      const int fx = 2 * x + (c & 1), fy = 2 * y + ((c >> 1) & 1), fz = 2 * z + (c >> 2);
      const uint32_t w = P.bits[0][(size_t(fz) * Rf + fy) * size_t(wpr) + size_t(fx >> 5)];
      kids |= ((w >> (fx & 31)) & 1u) << c;
    }
    wide[v] = uint32_t(word) | (kids << 16);
  }
}

int launch_build_pyramid(ngprt_ctx* ctx, const uint8_t* occ_fine, hipStream_t st) {
  const ngprt_desc& d = ctx->desc;
  const int nl = d.occ_levels;
  for (int j = 0; j < nl; ++j) {
    if (!ctx->pyr[j]) {
      const int64_t Rj = int64_t(d.occ_fine_res) >> j;
      if (dev_malloc((void**)&ctx->pyr[j], size_t(Rj * Rj * Rj / 32) * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, NGPRT_E_ALLOC, "occupancy pyramid allocation failed");
      }
    }
  }
  const int64_t nR = int64_t(d.occ_res) * d.occ_res * d.occ_res;
  if (int64_t(d.occ_fine_res) == 2 * int64_t(d.occ_res) && !ctx->pwide) {
    if (dev_malloc((void**)&ctx->pwide, size_t(nR) * sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_ALLOC, "occupancy pyramid allocation failed");
    }
  }
  const int64_t R0 = d.occ_fine_res;
  const int64_t w0 = R0 * R0 * R0 / 32;
  hipLaunchKernelGGL(pyr_pack_kernel, dim3(blocks_for(w0, 256)), dim3(256), 0, st, occ_fine, ctx->pyr[0], w0);
  int rc = check_launch(ctx, "pyr_pack_kernel");
  for (int j = 1; j < nl && rc == NGPRT_OK; ++j) {
    const int Rc = int(R0 >> j);
    const int64_t wc = int64_t(Rc) * Rc * Rc / 32;
    hipLaunchKernelGGL(pyr_pool_kernel, dim3(blocks_for(wc, 256)), dim3(256), 0, st, ctx->pyr[j - 1],
                       ctx->pyr[j], Rc);
    rc = check_launch(ctx, "pyr_pool_kernel");
  }
  if (rc) return rc;
  // the distance grid comes from the pyramid level of its resolution
  int jg = -1;
  for (int j = 0; j < nl; ++j)
    if ((R0 >> j) == d.occ_res) jg = j;
  if (jg < 0) return fail(ctx, NGPRT_E_SHAPE, "occ_res is not a pyramid resolution");
  const int64_t n = int64_t(d.occ_res) * d.occ_res * d.occ_res;
  uint8_t* tmp = nullptr;
  if (dev_malloc_async((void**)&tmp, size_t(n), st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, NGPRT_E_ALLOC, "pyramid scratch allocation failed");
  }
  hipLaunchKernelGGL(pyr_unpack_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctx->pyr[jg], tmp, n);
  rc = check_launch(ctx, "pyr_unpack_kernel");
  if (rc == NGPRT_OK) rc = launch_build_distance(ctx, tmp, nullptr, st);
  (void)hipFreeAsync(tmp, st);
  if (rc) return rc;
  PyrLevels P = {};
  for (int j = 0; j < nl; ++j) P.bits[j] = ctx->pyr[j];
  uint32_t* wide = jg == 1 ? ctx->pwide : nullptr;
  hipLaunchKernelGGL(pyr_code_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, ctx->grid, wide, d.occ_res, jg,
                     nl, P);
  return check_launch(ctx, "pyr_code_kernel");
}

}  // namespace ngprt
