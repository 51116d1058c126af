// Allocation-free variant of the hash-model render backward, for callers
// that cannot allocate device memory (code under stream capture, tight
// training loops, hosts that forbid allocation).
//
// Its workspace (one MLP-gradient partial per wave of 64 rays plus the
// fixed-order group sums, see reduce.h) lives in a file-scope device array
// of fixed size instead of the context's grow-on-demand buffer.  Every GPU
// that loads the library holds its own copy of the array until the process
// ends; its device address is looked up once per device, with that device
// current, when the first context on it is created, and only that address
// is handed to kernels.  Every element of the workspace is written before it
// is read in a call, so nothing needs clearing between calls.  All calls on
// one GPU share the array: calls that overlap on one GPU (two streams, two
// threads, two contexts) race and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace ngprt {

namespace {

constexpr int kMaxDevices = 64;
constexpr int64_t kScratchFloats = int64_t(NGPRT_NOALLOC_SCRATCH_BYTES) / 4;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};          // device address of `scratch` on each device

}  // namespace

static __device__ __align__(256) float scratch[kScratchFloats];

// Looks up this device's copy of `scratch`; the device of ctx must be current.
int init_static_scratch(ngprt_ctx* ctx) {
  const int dev = ctx->device;
  if (dev < 0 || dev >= kMaxDevices) return fail(ctx, NGPRT_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev]) return NGPRT_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(ctx, NGPRT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch[dev] = ptr;
  return NGPRT_OK;
}

static void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch[dev];
}

}  // namespace ngprt

using namespace ngprt;

extern "C" int ngprt_render_backward_noalloc(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                                             const float* dev_dirs, const float* dev_grad_rgb,
                                             const float* dev_grad_dist, float* dev_grad_tables,
                                             float* dev_grad_mlp, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays > NGPRT_NOALLOC_MAX_RAYS)
    return fail(ctx, NGPRT_E_SHAPE,
                "ngprt_render_backward_noalloc takes at most NGPRT_NOALLOC_MAX_RAYS (524288) rays per call");
  if (n_rays == 0) return NGPRT_OK;
  if (ctx->det_grad)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "deterministic gradients allocate their records");
  int rc = check_backward_args(ctx, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_tables, dev_grad_mlp);
  if (rc) return rc;
  if (backward_workspace_bytes(n_rays) > size_t(NGPRT_NOALLOC_SCRATCH_BYTES))
    return fail(ctx, NGPRT_E_SHAPE, "workspace exceeds the static scratch");
  void* ws = scratch_of(ctx->device);
  if (!ws) return fail(ctx, NGPRT_E_HIP, "the static scratch of this device was not found at ngprt_create");
  return launch_backward_ws(ctx, n_rays, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_dist, nullptr, nullptr,
                            nullptr, dev_grad_tables, nullptr, dev_grad_mlp, reinterpret_cast<float*>(ws),
                            (hipStream_t)stream);
}
