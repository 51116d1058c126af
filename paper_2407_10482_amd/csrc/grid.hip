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
  if (hipMallocAsync((void**)&dil, size_t(n), st) != hipSuccess ||
      hipMallocAsync((void**)&f0, size_t(n) * sizeof(int), st) != hipSuccess ||
      hipMallocAsync((void**)&f1, size_t(n) * sizeof(int), st) != hipSuccess) {
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

}  // namespace ngprt
