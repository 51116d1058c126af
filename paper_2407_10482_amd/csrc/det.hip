// Deterministic table gradients (a checking aid beside the training
// extension): the backward's float atomics add a wave's merged
// contributions in an order that varies from run to run, so the last bits
// of a table gradient vary too.  In this mode every corner contribution of
// every sample goes to a record of its own at a position fixed by (ray,
// sample, level, corner); a stable radix sort by table entry keeps that
// order within each entry, and one thread per entry sums its records in
// that order.  The table gradient is then the same bit for bit from run to
// run.  The MLP gradient is deterministic in both modes.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <vector>

#include "internal.h"

namespace ngprt {

// One thread per run of equal keys in the sorted records: the run's values,
// taken in record order, summed and added to the entry's gradient row.
__global__ void det_reduce_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ order,
                                  const float* __restrict__ vals, int64_t n, float* __restrict__ gtab) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t key = keys[i];
  if (i > 0 && keys[i - 1] == key) return;
  float s[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t j = i; j < n && keys[j] == key; ++j) {
    const float* v = vals + size_t(order[j]) * 9;
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] += v[c];
  }
  float* g = gtab + size_t(key) * 9;
#pragma unroll
  for (int c = 0; c < 9; ++c) g[c] += s[c];
}

int launch_backward_det(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                        const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                        float* gtab, float* gmlp, float* workspace, hipStream_t st) {
  // samples per ray (the same decisions as the backward's march), and each
  // ray's first sample among all of them
  int32_t* ns_dev = nullptr;
  if (dev_malloc_async((void**)&ns_dev, size_t(n) * sizeof(int32_t), st) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, NGPRT_E_ALLOC, "sample count allocation failed");
  }
  int rc = launch_march(ctx, n, o, d, 0, nullptr, ns_dev, nullptr, 0, st);
  std::vector<int32_t> ns(size_t(n), 0);
  if (rc == NGPRT_OK &&
      (hipMemcpyAsync(ns.data(), ns_dev, size_t(n) * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = check_launch(ctx, "sample count download");
  (void)hipFreeAsync(ns_dev, st);
  if (rc) return rc;
  std::vector<int64_t> off(static_cast<size_t>(n));
  int64_t total = 0;
  for (int64_t r = 0; r < n; ++r) {
    off[size_t(r)] = total;
    total += ns[size_t(r)];
  }
  const int64_t n_rec = total * ctx->desc.n_levels * 8;
  if (n_rec > NGPRT_DET_MAX_RECORDS)
    return fail(ctx, NGPRT_E_SHAPE, "too many contributions for deterministic gradients: split the batch");
  const int end_bit = 32 - __builtin_clz(uint32_t(ctx->desc.n_levels) * uint32_t(ctx->T) - 1u);

  DetRecords det;
  int64_t* off_dev = nullptr;
  uint32_t *keys_out = nullptr, *order_out = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  const size_t rec = size_t(n_rec > 0 ? n_rec : 1);
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, det.keys, keys_out, det.order, order_out,
                                         int(n_rec), 0, end_bit, st) != hipSuccess)
    return check_launch(ctx, "radix sort size query");
  bool ok = dev_malloc_async((void**)&off_dev, size_t(n) * sizeof(int64_t), st) == hipSuccess &&
            dev_malloc_async((void**)&det.keys, rec * sizeof(uint32_t), st) == hipSuccess &&
            dev_malloc_async((void**)&det.order, rec * sizeof(uint32_t), st) == hipSuccess &&
            dev_malloc_async((void**)&det.vals, rec * 9 * sizeof(float), st) == hipSuccess &&
            dev_malloc_async((void**)&keys_out, rec * sizeof(uint32_t), st) == hipSuccess &&
            dev_malloc_async((void**)&order_out, rec * sizeof(uint32_t), st) == hipSuccess &&
            dev_malloc_async(&temp, temp_bytes > 0 ? temp_bytes : 1, st) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    rc = fail(ctx, NGPRT_E_ALLOC, "deterministic gradient records allocation failed");
  }
  if (rc == NGPRT_OK &&
      hipMemcpyAsync(off_dev, off.data(), size_t(n) * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = check_launch(ctx, "ray offsets upload");
  if (rc == NGPRT_OK) {
    det.off = off_dev;
    det.n = n_rec;
    rc = launch_backward_ws(ctx, n, o, d, grad_rgb, grad_dist, ups, fcd, ffv, gtab, nullptr, gmlp, workspace,
                            st, det);
  }
  if (rc == NGPRT_OK && n_rec > 0) {
    if (hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, det.keys, keys_out, det.order, order_out,
                                           int(n_rec), 0, end_bit, st) != hipSuccess)
      rc = check_launch(ctx, "radix sort");
  }
  if (rc == NGPRT_OK && n_rec > 0) {
    hipLaunchKernelGGL(det_reduce_kernel, dim3(unsigned((n_rec + 255) / 256)), dim3(256), 0, st, keys_out,
                       order_out, det.vals, n_rec, gtab);
    rc = check_launch(ctx, "det_reduce_kernel");
  }
  // the host offsets are freed on return: finish their upload first
  if (hipStreamSynchronize(st) != hipSuccess && rc == NGPRT_OK) rc = check_launch(ctx, "deterministic backward");
  for (void* p : {(void*)off_dev, (void*)det.keys, (void*)det.order, (void*)det.vals, (void*)keys_out,
                  (void*)order_out, temp})
    if (p) (void)hipFreeAsync(p, st);
  return rc;
}

}  // namespace ngprt
