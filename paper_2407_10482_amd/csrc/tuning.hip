// Marching-step auto-tuning of the paper's training (supplement, "Auto-tuning
// of Marching Step Size", Eq. S3): after each batch, with N the batch's mean
// number of evaluated samples per ray, gamma <- min(1, (1 + kappa) gamma) when
// N >= N_min, else max(gamma_min, (1 - kappa) gamma); the marching step is
// gamma * s0.  The mean comes from the per-ray sample counts a render wrote,
// summed on the GPU in a fixed order (per-block partial sums, then one block
// over the partials), so repeated calls give the same gamma.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ngprt {

constexpr int kCountBlocks = 1024;

__global__ void __launch_bounds__(256) count_partial_kernel(const int32_t* __restrict__ counts, int64_t n,
                                                            long long* __restrict__ partial) {
  __shared__ long long red[256];
  long long a = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    a += counts[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) count_final_kernel(const long long* __restrict__ partial, int nb,
                                                          long long* __restrict__ total) {
  __shared__ long long red[256];
  long long a = 0;
  for (int i = threadIdx.x; i < nb; i += 256) a += partial[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = red[0];
}

int sum_counts(ngprt_ctx* ctx, int64_t n, const int32_t* counts, long long* host_total, hipStream_t st) {
  if (!ctx->count_ws) {
    if (dev_malloc((void**)&ctx->count_ws, (kCountBlocks + 1) * sizeof(long long)) != hipSuccess) {
      (void)hipGetLastError();
      ctx->count_ws = nullptr;
      return fail(ctx, NGPRT_E_ALLOC, "sample-count workspace");
    }
  }
  long long* partial = reinterpret_cast<long long*>(ctx->count_ws);
  const int64_t want = (n + 255) / 256;
  const int nb = int(want < kCountBlocks ? want : kCountBlocks);
  hipLaunchKernelGGL(count_partial_kernel, dim3(nb), dim3(256), 0, st, counts, n, partial);
  int rc = check_launch(ctx, "count_partial_kernel");
  if (rc) return rc;
  hipLaunchKernelGGL(count_final_kernel, dim3(1), dim3(256), 0, st, partial, nb, partial + kCountBlocks);
  if ((rc = check_launch(ctx, "count_final_kernel"))) return rc;
  if (hipMemcpyAsync(host_total, partial + kCountBlocks, sizeof(long long), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    const hipError_t e = hipGetLastError();
    return fail(ctx, NGPRT_E_HIP, std::string("sample-count read-back: ") + hipGetErrorString(e));
  }
  return NGPRT_OK;
}

}  // namespace ngprt
