// C ABI entry points: validation, context and scene ownership, dispatch.
// Validation is pure host code so it runs (and is tested) without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace ngprt {

int fail(ngprt_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int check_launch(ngprt_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ctx, NGPRT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return NGPRT_OK;
}

SceneArgs scene_args(const ngprt_ctx* ctx) {
  const ngprt_desc& d = ctx->desc;
  SceneArgs S;
  std::memset(&S, 0, sizeof(S));
  S.L = d.n_levels;
  S.log2T = d.log2_table_size;
  S.mask = uint32_t((int64_t(1) << d.log2_table_size) - 1);
  for (int l = 0; l < kMaxLevels; ++l) {
    S.N[l] = l < d.n_levels ? d.resolutions[l] : 1;
    S.Nf[l] = float(S.N[l]);
    for (int c = 0; c < 9; ++c) S.scale[l][c] = ctx->scales_host[l][c];
  }
  S.feat = ctx->feat;
  S.logit = ctx->logit;
  S.grid = ctx->grid;
  S.R = d.occ_res;
  S.Rf = float(d.occ_res);
  S.lo = -d.roi_half;
  S.inv_ext = 1.0f / (d.roi_half - (-d.roi_half));
  S.vox = (d.roi_half - (-d.roi_half)) / float(d.occ_res);
  S.v_over_step = S.vox / d.step;
  S.step = d.step;
  S.thr = d.t_threshold;
  S.max_samples = d.max_samples;
  S.pyr_n = d.occ_levels > 0 ? d.occ_levels : 0;
  S.use_dist = d.use_distance;
  S.pyr_jg = 0;
  for (int j = 0; j < kMaxPyr; ++j) {
    S.pyrR[j] = j < S.pyr_n ? (d.occ_fine_res >> j) : 32;
    S.pyr[j] = j < S.pyr_n ? ctx->pyr[j] : nullptr;
    if (j < S.pyr_n && S.pyrR[j] == d.occ_res) S.pyr_jg = j;
  }
  S.pwide = S.pyr_n > 0 && S.pyr_jg == 1 ? ctx->pwide : nullptr;
  S.view_mlp = d.mlp_hidden == 64 ? 1 : 0;
  S.model = d.feature_model;
  if (d.feature_model == NGPRT_MODEL_BAKED) {
    S.LC = d.coarse_res;
    S.LCf = float(d.coarse_res);
    S.nb = (d.coarse_res + 1 + 7) / 8;
    S.Cpad = coarse_row_floats(coarse_channels(d));
    S.cidx = ctx->cidx;
    S.catlas = ctx->catlas;
    S.n_blocks = ctx->n_blocks;
    for (int j = 0; j < 16; ++j) S.cdef[j] = ctx->cdef[j];
    S.gen = d.aggregation != NGPRT_AGG_SEPARATE_V ? 1 : 0;
    for (int l = 0; l < 4; ++l) {
      int iw = 8 + 2 * l, ib = 9 + 2 * l;      // Separate-Att (V)
      float cw = 0.0f, cb = 0.0f;
      switch (d.aggregation) {
        case NGPRT_AGG_SHARED_V: iw = ib = 8 + l; break;
        case NGPRT_AGG_SEPARATE_INV:
          iw = ib = -1;
          cw = d.gate_params[2 * l];
          cb = d.gate_params[2 * l + 1];
          break;
        case NGPRT_AGG_SHARED_INV: iw = ib = -1; cw = cb = d.gate_params[l]; break;
        case NGPRT_AGG_SUM: iw = ib = -1; cw = cb = INFINITY; break;
        default: break;
      }
      S.gidx[l][0] = iw;
      S.gidx[l][1] = ib;
      S.gconst[l][0] = cw;
      S.gconst[l][1] = cb;
    }
  }
  return S;
}

static bool is_view_mlp(const ngprt_desc* d) { return d->mlp_hidden == 64; }
static int mlp_param_count(const ngprt_desc* d) { return is_view_mlp(d) ? kMlpViewParams : kMlpParams; }

static size_t dtype_bytes(int dt) { return dt == DT_F32 ? 4 : (dt == DT_BF16 ? 2 : 1); }

// armed: the number of device allocations still to succeed before one fails
static std::atomic<int64_t> g_fail_alloc_after{-1};

static bool injected_alloc_failure() {
  int64_t k = g_fail_alloc_after.load();
  while (k >= 0) {
    if (g_fail_alloc_after.compare_exchange_weak(k, k - 1)) return k == 0;
  }
  return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  if (injected_alloc_failure()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s) {
  if (injected_alloc_failure()) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, s);
}

}  // namespace ngprt

using namespace ngprt;

extern "C" {

const char* ngprt_status_string(int status) {
  switch (status) {
    case NGPRT_OK: return "NGPRT_OK";
    case NGPRT_E_INVALID_ARG: return "NGPRT_E_INVALID_ARG";
    case NGPRT_E_SHAPE: return "NGPRT_E_SHAPE";
    case NGPRT_E_DTYPE: return "NGPRT_E_DTYPE";
    case NGPRT_E_NOT_LOADED: return "NGPRT_E_NOT_LOADED";
    case NGPRT_E_ALLOC: return "NGPRT_E_ALLOC";
    case NGPRT_E_HIP: return "NGPRT_E_HIP";
    case NGPRT_E_UNSUPPORTED: return "NGPRT_E_UNSUPPORTED";
    default: return "NGPRT_E_UNKNOWN";
  }
}

const char* ngprt_last_error(const ngprt_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

static bool is_pow2_float(float x) {
  if (!(x > 0.0f) || !std::isfinite(x)) return false;
  int e;
  return std::frexp(x, &e) == 0.5f;
}

int ngprt_validate_desc(const ngprt_desc* d) {
  if (!d) return NGPRT_E_INVALID_ARG;
  if (d->n_levels < 1 || d->n_levels > NGPRT_MAX_LEVELS) return NGPRT_E_SHAPE;
  for (int l = 0; l < d->n_levels; ++l)
    if (d->resolutions[l] < 1 || d->resolutions[l] > (1 << 20)) return NGPRT_E_SHAPE;
  if (d->log2_table_size < 4 || d->log2_table_size > 24) return NGPRT_E_SHAPE;
  if (d->table_dtype < 0 || d->table_dtype > 2) return NGPRT_E_DTYPE;
  if (d->domain != NGPRT_ROI_BOX && d->domain != NGPRT_ROI_CONTRACT) return NGPRT_E_INVALID_ARG;
  if (!is_pow2_float(d->roi_half)) return NGPRT_E_INVALID_ARG;
  if (d->domain == NGPRT_ROI_CONTRACT && d->roi_half != 2.0f) return NGPRT_E_INVALID_ARG;
  if (d->occ_res < 2 || d->occ_res > 1024) return NGPRT_E_SHAPE;
  if (!(d->step > 0.0f) || !std::isfinite(d->step)) return NGPRT_E_INVALID_ARG;
  // the box march's skip keeps a margin of one lattice step from occupied
  // voxels; it must dwarf float32 position error
  if (d->domain == NGPRT_ROI_BOX && d->step < d->roi_half * (1.0f / 65536.0f)) return NGPRT_E_INVALID_ARG;
  if (d->max_samples < 1) return NGPRT_E_INVALID_ARG;
  if (!(d->t_threshold >= 0.0f) || !std::isfinite(d->t_threshold)) return NGPRT_E_INVALID_ARG;
  const bool plain_mlp = d->mlp_in == 7 && d->mlp_hidden == 16 && d->mlp_out == 3;
  const bool view_mlp = d->mlp_in == 23 && d->mlp_hidden == 64 && d->mlp_out == 3;
  if (!plain_mlp && !view_mlp) return NGPRT_E_UNSUPPORTED;
  if (d->feature_model != NGPRT_MODEL_HASH && d->feature_model != NGPRT_MODEL_BAKED)
    return NGPRT_E_INVALID_ARG;
  if (d->feature_model == NGPRT_MODEL_BAKED) {
    if (d->n_levels > 4) return NGPRT_E_SHAPE;
    if (d->coarse_res < 1 || d->coarse_res > 2048) return NGPRT_E_SHAPE;
    if (d->aggregation < NGPRT_AGG_SEPARATE_V || d->aggregation > NGPRT_AGG_SUM) return NGPRT_E_INVALID_ARG;
    if (d->aggregation != NGPRT_AGG_SEPARATE_V && d->table_dtype != NGPRT_F32) return NGPRT_E_UNSUPPORTED;
    const int n_const = d->aggregation == NGPRT_AGG_SEPARATE_INV ? 2 * d->n_levels
                        : d->aggregation == NGPRT_AGG_SHARED_INV ? d->n_levels : 0;
    for (int j = 0; j < n_const; ++j)
      if (!std::isfinite(d->gate_params[j])) return NGPRT_E_INVALID_ARG;
  } else if (d->aggregation != NGPRT_AGG_SEPARATE_V) {
    return NGPRT_E_INVALID_ARG;
  }
  if (d->occ_levels != 0) {
    const int F = d->occ_fine_res;
    if (d->occ_levels < 2 || d->occ_levels > 5) return NGPRT_E_SHAPE;
    if (F < 32 || F > 1024 || (F & (F - 1)) != 0) return NGPRT_E_SHAPE;
    if ((F >> (d->occ_levels - 1)) < 32) return NGPRT_E_SHAPE;
    bool found = false;
    for (int j = 0; j < d->occ_levels; ++j) found = found || (F >> j) == d->occ_res;
    if (!found) return NGPRT_E_SHAPE;
    if (d->use_distance != 0 && d->use_distance != 1) return NGPRT_E_INVALID_ARG;
  }
  return NGPRT_OK;
}

void ngprt_destroy(ngprt_ctx* ctx) {
  if (!ctx) return;
  int cur = 0;
  bool switched = hipGetDevice(&cur) == hipSuccess && cur != ctx->device &&
                  hipSetDevice(ctx->device) == hipSuccess;
  (void)hipDeviceSynchronize();
  if (ctx->feat) (void)hipFree(ctx->feat);
  if (ctx->logit) (void)hipFree(ctx->logit);
  if (ctx->scales_dev) (void)hipFree(ctx->scales_dev);
  if (ctx->grid) (void)hipFree(ctx->grid);
  if (ctx->mlp) (void)hipFree(ctx->mlp);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->prop_wb) (void)hipFree(ctx->prop_wb);
  if (ctx->prop_grad) (void)hipFree(ctx->prop_grad);
  if (ctx->prop_net) (void)hipFree(ctx->prop_net);
  if (ctx->prop_tmp) (void)hipFree(ctx->prop_tmp);
  if (ctx->count_ws) (void)hipFree(ctx->count_ws);
  if (ctx->mlp_rec) (void)hipFree(ctx->mlp_rec);
  if (ctx->cidx) (void)hipFree(ctx->cidx);
  if (ctx->catlas) (void)hipFree(ctx->catlas);
  for (int j = 0; j < 5; ++j)
    if (ctx->pyr[j]) (void)hipFree(ctx->pyr[j]);
  if (ctx->pwide) (void)hipFree(ctx->pwide);
  if (switched) (void)hipSetDevice(cur);
  delete ctx;
}

int ngprt_test_fail_alloc(int64_t after) {
  g_fail_alloc_after.store(after < 0 ? -1 : after);
  return NGPRT_OK;
}

int ngprt_create(const ngprt_desc* desc, ngprt_ctx** out) {
  if (!out) return NGPRT_E_INVALID_ARG;
  int rc = ngprt_validate_desc(desc);
  if (rc) return rc;
  ngprt_ctx* ctx = new (std::nothrow) ngprt_ctx();
  if (!ctx) return NGPRT_E_ALLOC;
  ctx->desc = *desc;
  ctx->T = int64_t(1) << desc->log2_table_size;
  for (int l = 0; l < NGPRT_MAX_LEVELS; ++l)
    for (int c = 0; c < 9; ++c) ctx->scales_host[l][c] = 1.0f;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return NGPRT_E_HIP;
  }
  const int64_t L = desc->n_levels;
  const size_t eb = dtype_bytes(desc->table_dtype);
  const int64_t R = desc->occ_res;
  bool ok = dev_malloc((void**)&ctx->feat, size_t(L * ctx->T * 8) * eb) == hipSuccess &&
            dev_malloc((void**)&ctx->logit, size_t(L * ctx->T) * eb) == hipSuccess &&
            dev_malloc((void**)&ctx->scales_dev, sizeof(float) * (NGPRT_MAX_LEVELS * 9 + 1)) == hipSuccess &&
            dev_malloc((void**)&ctx->grid, size_t(R * R * R) * sizeof(uint16_t)) == hipSuccess &&
            dev_malloc((void**)&ctx->mlp, sizeof(float) * mlp_param_count(desc)) == hipSuccess &&
            (!is_view_mlp(desc) ||
             dev_malloc((void**)&ctx->mlp_rec, sizeof(float) * kMlpViewRec) == hipSuccess);
  if (ok)
    ok = hipMemcpy(ctx->scales_dev, &ctx->scales_host[0][0], sizeof(float) * NGPRT_MAX_LEVELS * 9,
                   hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ngprt_destroy(ctx);
    return NGPRT_E_ALLOC;
  }
  // this device's copy of the allocation-free backward's static scratch; a
  // failure here only disables ngprt_render_backward_noalloc (which reports it)
  (void)init_static_scratch(ctx);
  ctx->last_error.clear();
  *out = ctx;
  return NGPRT_OK;
}

int ngprt_load_tables(ngprt_ctx* ctx, const float* dev_tables, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_tables) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_tables is NULL");
  int rc = launch_load_tables(ctx, dev_tables, (hipStream_t)stream);
  if (rc == NGPRT_OK) ctx->tables_loaded = true;
  return rc;
}

int ngprt_load_coarse(ngprt_ctx* ctx, int64_t n_blocks, const int32_t* dev_block_index,
                      const float* dev_atlas, const float* host_default, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  const ngprt_desc& d = ctx->desc;
  if (d.feature_model != NGPRT_MODEL_BAKED)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the context does not use the baked feature model");
  if (n_blocks < 0 || n_blocks > (int64_t(1) << 31) / 512)
    return fail(ctx, NGPRT_E_INVALID_ARG, "n_blocks out of range");
  if (!dev_block_index || !host_default || (n_blocks > 0 && !dev_atlas))
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (d.coarse_res + 1 + 7) / 8;
  const int64_t n_idx = nb * nb * nb;
  // the index grid decides which atlas rows the kernels read: check it here
  std::vector<int32_t> idx(static_cast<size_t>(n_idx));
  if (hipMemcpyAsync(idx.data(), dev_block_index, sizeof(int32_t) * n_idx, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return check_launch(ctx, "block index copy");
  for (int64_t i = 0; i < n_idx; ++i)
    if (idx[size_t(i)] < -1 || idx[size_t(i)] >= n_blocks)
      return fail(ctx, NGPRT_E_INVALID_ARG, "block index entry outside [-1, n_blocks)");
  const int C = coarse_channels(d), Cpad = coarse_row_floats(C);
  ctx->coarse_loaded = false;
  // same block count as the loaded grid (a training step's update): keep the
  // allocations; the index grid's size is fixed by the descriptor
  const bool reuse = ctx->cidx != nullptr && ctx->n_blocks == n_blocks && (n_blocks == 0 || ctx->catlas);
  if (!reuse) {
    if (ctx->cidx) (void)hipFree(ctx->cidx);
    if (ctx->catlas) (void)hipFree(ctx->catlas);
    ctx->cidx = nullptr;
    ctx->catlas = nullptr;
    ctx->n_blocks = -1;
    if (dev_malloc((void**)&ctx->cidx, sizeof(int32_t) * n_idx) != hipSuccess ||
        (n_blocks > 0 &&
         dev_malloc((void**)&ctx->catlas, sizeof(float) * size_t(n_blocks) * 512 * Cpad) != hipSuccess)) {
      (void)hipGetLastError();
      return fail(ctx, NGPRT_E_ALLOC, "coarse grid allocation failed");
    }
  }
  if (hipMemcpyAsync(ctx->cidx, idx.data(), sizeof(int32_t) * n_idx, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return check_launch(ctx, "block index upload");
  ctx->n_blocks = n_blocks;
  for (int j = 0; j < 16; ++j) ctx->cdef[j] = j < C ? host_default[j] : 0.0f;
  if (n_blocks > 0) {
    int rc = launch_pack_atlas(ctx, dev_atlas, n_blocks, st);
    if (rc) return rc;
  }
  // the host copy of the index grid is freed on return: finish the upload first
  if (hipStreamSynchronize(st) != hipSuccess) return check_launch(ctx, "coarse grid upload");
  ctx->coarse_loaded = true;
  return NGPRT_OK;
}

int ngprt_export_tables(ngprt_ctx* ctx, void* dev_codes, float* dev_scales, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_codes) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_codes is NULL");
  if (!ctx->tables_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "tables not loaded");
  return launch_export_tables(ctx, dev_codes, dev_scales, (hipStream_t)stream);
}

int ngprt_load_occupancy(ngprt_ctx* ctx, const uint8_t* dev_occ, const uint8_t* dev_dist, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_occ) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_occ is NULL");
  if (ctx->desc.occ_levels != 0)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the context marches an occupancy pyramid");
  int rc = launch_build_distance(ctx, dev_occ, dev_dist, (hipStream_t)stream);
  if (rc == NGPRT_OK) ctx->occ_loaded = true;
  return rc;
}

int ngprt_load_occupancy_pyramid(ngprt_ctx* ctx, const uint8_t* dev_occ_fine, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (ctx->desc.occ_levels == 0)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the context marches a single occupancy grid");
  if (!dev_occ_fine) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_occ_fine is NULL");
  ctx->occ_loaded = false;
  int rc = launch_build_pyramid(ctx, dev_occ_fine, (hipStream_t)stream);
  if (rc == NGPRT_OK) ctx->occ_loaded = true;
  return rc;
}

int ngprt_export_distance(ngprt_ctx* ctx, uint8_t* dev_dist, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_dist) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_dist is NULL");
  if (!ctx->occ_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "occupancy not loaded");
  return launch_export_distance(ctx, dev_dist, (hipStream_t)stream);
}

int ngprt_load_mlp(ngprt_ctx* ctx, const float* dev_params, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_params) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_params is NULL");
  if (hipMemcpyAsync(ctx->mlp, dev_params, sizeof(float) * mlp_param_count(&ctx->desc),
                     hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
    return check_launch(ctx, "mlp copy");
  if (is_view_mlp(&ctx->desc)) {
    int rc = launch_view_mlp_arrange(ctx, ctx->mlp, (hipStream_t)stream);
    if (rc) return rc;
  }
  ctx->mlp_loaded = true;
  return NGPRT_OK;
}

static int check_ready(ngprt_ctx* ctx) {
  if (!ctx->tables_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "tables not loaded");
  if (ctx->desc.feature_model == NGPRT_MODEL_BAKED && !ctx->coarse_loaded)
    return fail(ctx, NGPRT_E_NOT_LOADED, "coarse grid not loaded");
  if (!ctx->occ_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "occupancy not loaded");
  return NGPRT_OK;
}

}  // extern "C"

namespace ngprt {
// Host checks shared by the hash-model render backward entry points.
int check_backward_args(ngprt_ctx* ctx, const float* o, const float* d, const float* grad_rgb,
                        const float* grad_tables, const float* grad_mlp) {
  if (!o || !d || !grad_rgb || !grad_tables || !grad_mlp) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if (ctx->desc.table_dtype != NGPRT_F32) return fail(ctx, NGPRT_E_DTYPE, "backward needs float32 tables");
  if (ctx->desc.feature_model != NGPRT_MODEL_HASH)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "backward supports the hash feature model only");
  if (is_view_mlp(&ctx->desc))
    return fail(ctx, NGPRT_E_UNSUPPORTED, "backward supports the 7-16-16-3 deferred MLP only");
  int rc = check_ready(ctx);
  if (rc) return rc;
  if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
  return NGPRT_OK;
}
}  // namespace ngprt

extern "C" {

int ngprt_render(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                 const ngprt_outputs* out, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!out || !out->rgb) return fail(ctx, NGPRT_E_INVALID_ARG, "out->rgb is required");
  if (!dev_origins || !dev_dirs) return fail(ctx, NGPRT_E_INVALID_ARG, "ray pointers are NULL");
  int rc = check_ready(ctx);
  if (rc) return rc;
  if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
  if (is_view_mlp(&ctx->desc) && (!out->c_d || !out->feat))
    return fail(ctx, NGPRT_E_INVALID_ARG, "the view-dependent MLP needs the c_d and feat outputs");
  RayOut o{out->rgb,       out->c_d,     out->feat,   out->t_final, out->depth,
           out->n_samples, out->n_reads, out->t_first, out->t_far,   out->t_half, out->dist_loss,
           nullptr};
  const ngprt_proposal_cfg none{0.0f, 0.0f, 0, 0.0f};
  return launch_render(ctx, n_rays, dev_origins, dev_dirs, o, nullptr, false, nullptr, none, nullptr,
                       (hipStream_t)stream);
}

}  // extern "C"

// Shared checks and launch of the two proposal renders.
static int render_with_proposal(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                                const float* dev_proposal, bool use_net, const ngprt_proposal_cfg* cfg,
                                const ngprt_outputs* out, int32_t* dev_fallback, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (!cfg) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL proposal configuration");
  if (!std::isfinite(cfg->margin) || cfg->margin < 0.0f) return fail(ctx, NGPRT_E_INVALID_ARG, "bad margin");
  if (cfg->conf_threshold != cfg->conf_threshold || cfg->far_guard != cfg->far_guard)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NaN confidence threshold or far guard");
  if (cfg->use_near != 0 && cfg->use_near != 1) return fail(ctx, NGPRT_E_INVALID_ARG, "use_near must be 0 or 1");
  if (n_rays == 0) return NGPRT_OK;
  if (!out || !out->rgb) return fail(ctx, NGPRT_E_INVALID_ARG, "out->rgb is required");
  if (!dev_origins || !dev_dirs || (!use_net && !dev_proposal))
    return fail(ctx, NGPRT_E_INVALID_ARG, "ray or proposal pointers are NULL");
  int rc = check_ready(ctx);
  if (rc) return rc;
  if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
  if (use_net && !ctx->prop_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "proposal network not loaded");
  if (is_view_mlp(&ctx->desc) && (!out->c_d || !out->feat))
    return fail(ctx, NGPRT_E_INVALID_ARG, "the view-dependent MLP needs the c_d and feat outputs");
  RayOut o{out->rgb,       out->c_d,     out->feat,   out->t_final, out->depth,
           out->n_samples, out->n_reads, out->t_first, out->t_far,   out->t_half, out->dist_loss,
           use_net ? out->proposal : nullptr};
  return launch_render(ctx, n_rays, dev_origins, dev_dirs, o, use_net ? nullptr : dev_proposal, use_net,
                       o.proposal, *cfg, dev_fallback, (hipStream_t)stream);
}

extern "C" {

int ngprt_render_intervals(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                           const float* dev_proposal, const ngprt_proposal_cfg* cfg, const ngprt_outputs* out,
                           int32_t* dev_fallback, void* stream) {
  return render_with_proposal(ctx, n_rays, dev_origins, dev_dirs, dev_proposal, false, cfg, out, dev_fallback,
                              stream);
}

int ngprt_render_proposal(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                          const ngprt_proposal_cfg* cfg, const ngprt_outputs* out, int32_t* dev_fallback,
                          void* stream) {
  return render_with_proposal(ctx, n_rays, dev_origins, dev_dirs, nullptr, true, cfg, out, dev_fallback,
                              stream);
}

int ngprt_proposal_load(ngprt_ctx* ctx, const float* dev_params, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!dev_params) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  return load_proposal(ctx, dev_params, (hipStream_t)stream);
}

int ngprt_debug_eval_points(ngprt_ctx* ctx, int64_t n, const float* dev_pos, int32_t* dev_idx,
                            float* dev_fused, float* dev_weights, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n < 0");
  if (n == 0) return NGPRT_OK;
  if (!dev_pos) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_pos is NULL");
  if (!ctx->tables_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "tables not loaded");
  if (ctx->desc.feature_model == NGPRT_MODEL_BAKED && !ctx->coarse_loaded)
    return fail(ctx, NGPRT_E_NOT_LOADED, "coarse grid not loaded");
  return launch_eval_points(ctx, n, dev_pos, dev_idx, dev_fused, dev_weights, (hipStream_t)stream);
}

int ngprt_gather_probe(ngprt_ctx* ctx, int64_t n_points, uint32_t seed, int32_t pairs, float* dev_out,
                       void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_points < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_points < 0");
  if (n_points == 0) return NGPRT_OK;
  if (!dev_out) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_out is NULL");
  if (pairs != 0 && pairs != 1) return fail(ctx, NGPRT_E_INVALID_ARG, "pairs must be 0 or 1");
  if (!ctx->tables_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "tables not loaded");
  return launch_gather_probe(ctx, n_points, seed, pairs, dev_out, (hipStream_t)stream);
}

int ngprt_debug_march(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                      int32_t cap, int32_t* dev_sample_k, int32_t* dev_n_samples, int32_t* dev_n_reads,
                      int32_t naive, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0 || cap < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "negative size");
  if (cap > 0 && !dev_sample_k) return fail(ctx, NGPRT_E_INVALID_ARG, "dev_sample_k is NULL");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_origins || !dev_dirs) return fail(ctx, NGPRT_E_INVALID_ARG, "ray pointers are NULL");
  int rc = check_ready(ctx);
  if (rc) return rc;
  return launch_march(ctx, n_rays, dev_origins, dev_dirs, cap, dev_sample_k, dev_n_samples,
                      dev_n_reads, naive, (hipStream_t)stream);
}

int ngprt_render_backward_reg(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                              const float* dev_dirs, const float* dev_grad_rgb, const float* dev_grad_dist,
                              float* dev_grad_tables, float* dev_grad_mlp, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  int rc = check_backward_args(ctx, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_tables, dev_grad_mlp);
  if (rc) return rc;
  return launch_backward(ctx, n_rays, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_dist, nullptr, nullptr,
                         nullptr, dev_grad_tables, nullptr, dev_grad_mlp, (hipStream_t)stream);
}

int ngprt_render_backward_baked(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                                const float* dev_grad_rgb, const float* dev_grad_dist, float* dev_grad_tables,
                                float* dev_grad_atlas, float* dev_grad_mlp, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_origins || !dev_dirs || !dev_grad_rgb || !dev_grad_tables || !dev_grad_mlp)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if (ctx->desc.table_dtype != NGPRT_F32)
    return fail(ctx, NGPRT_E_DTYPE, "backward needs float32 tables");
  if (ctx->desc.feature_model != NGPRT_MODEL_BAKED)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "ngprt_render_backward_baked needs the baked feature model");
  if (ctx->desc.aggregation != NGPRT_AGG_SEPARATE_V)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the baked backward supports Separate-Att (V) only");
  if (is_view_mlp(&ctx->desc))
    return fail(ctx, NGPRT_E_UNSUPPORTED, "backward supports the 7-16-16-3 deferred MLP only");
  int rc = check_ready(ctx);
  if (rc) return rc;
  if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
  if (ctx->n_blocks > 0 && !dev_grad_atlas) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  return launch_backward(ctx, n_rays, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_dist, nullptr, nullptr,
                         nullptr, dev_grad_tables, dev_grad_atlas, dev_grad_mlp, (hipStream_t)stream);
}

int ngprt_view_mlp_backward(ngprt_ctx* ctx, int64_t n_rays, const float* dev_dirs, const float* dev_c_d,
                            const float* dev_feat, const float* dev_grad_rgb, float* dev_grad_cf,
                            float* dev_grad_mlp, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_dirs || !dev_c_d || !dev_feat || !dev_grad_rgb || !dev_grad_cf || !dev_grad_mlp)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if (!is_view_mlp(&ctx->desc))
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the context does not use the view-dependent MLP");
  if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
  return launch_view_mlp_backward(ctx, n_rays, dev_dirs, dev_c_d, dev_feat, dev_grad_rgb, dev_grad_cf,
                                  dev_grad_mlp, (hipStream_t)stream);
}

int ngprt_render_backward_features(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                                   const float* dev_dirs, const float* dev_grad_cf, const float* dev_grad_dist,
                                   float* dev_grad_tables, float* dev_grad_atlas, const float* dev_c_d,
                                   const float* dev_feat, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_origins || !dev_dirs || !dev_grad_cf || !dev_grad_tables)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if ((dev_c_d == nullptr) != (dev_feat == nullptr))
    return fail(ctx, NGPRT_E_INVALID_ARG, "dev_c_d and dev_feat go together");
  if (dev_c_d && dev_grad_dist)
    return fail(ctx, NGPRT_E_INVALID_ARG, "the forward's C_d and F are taken without the regulariser only");
  if (ctx->desc.table_dtype != NGPRT_F32)
    return fail(ctx, NGPRT_E_DTYPE, "backward needs float32 tables");
  const bool baked = ctx->desc.feature_model == NGPRT_MODEL_BAKED;
  if (baked && ctx->desc.aggregation != NGPRT_AGG_SEPARATE_V)
    return fail(ctx, NGPRT_E_UNSUPPORTED, "the baked backward supports Separate-Att (V) only");
  int rc = check_ready(ctx);
  if (rc) return rc;
  if (baked && ctx->n_blocks > 0 && !dev_grad_atlas) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  return launch_backward(ctx, n_rays, dev_origins, dev_dirs, nullptr, dev_grad_dist, dev_grad_cf, dev_c_d,
                         dev_feat, dev_grad_tables, baked ? dev_grad_atlas : nullptr, nullptr, (hipStream_t)stream);
}

int ngprt_set_deterministic_gradients(ngprt_ctx* ctx, int on) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  ctx->det_grad = on != 0;
  return NGPRT_OK;
}

int ngprt_render_backward_fwd(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                              const float* dev_c_d, const float* dev_feat, const float* dev_grad_rgb,
                              float* dev_grad_tables, float* dev_grad_atlas, float* dev_grad_mlp, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_c_d || !dev_feat) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  const bool baked = ctx->desc.feature_model == NGPRT_MODEL_BAKED;
  if (baked) {
    if (!dev_origins || !dev_dirs || !dev_grad_rgb || !dev_grad_tables || !dev_grad_mlp)
      return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
    if (ctx->desc.table_dtype != NGPRT_F32) return fail(ctx, NGPRT_E_DTYPE, "backward needs float32 tables");
    if (ctx->desc.aggregation != NGPRT_AGG_SEPARATE_V)
      return fail(ctx, NGPRT_E_UNSUPPORTED, "the baked backward supports Separate-Att (V) only");
    if (is_view_mlp(&ctx->desc))
      return fail(ctx, NGPRT_E_UNSUPPORTED, "backward supports the 7-16-16-3 deferred MLP only");
    int rc = check_ready(ctx);
    if (rc) return rc;
    if (!ctx->mlp_loaded) return fail(ctx, NGPRT_E_NOT_LOADED, "mlp not loaded");
    if (ctx->n_blocks > 0 && !dev_grad_atlas) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  } else {
    int rc = check_backward_args(ctx, dev_origins, dev_dirs, dev_grad_rgb, dev_grad_tables, dev_grad_mlp);
    if (rc) return rc;
  }
  return launch_backward(ctx, n_rays, dev_origins, dev_dirs, dev_grad_rgb, nullptr, nullptr, dev_c_d, dev_feat,
                         dev_grad_tables, baked ? dev_grad_atlas : nullptr, dev_grad_mlp, (hipStream_t)stream);
}

int ngprt_render_backward(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                          const float* dev_grad_rgb, float* dev_grad_tables, float* dev_grad_mlp,
                          void* stream) {
  return ngprt_render_backward_reg(ctx, n_rays, dev_origins, dev_dirs, dev_grad_rgb, nullptr, dev_grad_tables,
                                   dev_grad_mlp, stream);
}

int ngprt_step_autotune(ngprt_ctx* ctx, int64_t n_rays, const int32_t* dev_n_samples, ngprt_step_tuner* tuner,
                        void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (!tuner || !dev_n_samples) return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if (n_rays < 1) return fail(ctx, NGPRT_E_INVALID_ARG, "empty batch");
  const ngprt_step_tuner& t = *tuner;
  if (!(t.s0 > 0.0f) || !std::isfinite(t.s0) || !std::isfinite(t.n_min) || !(t.kappa >= 0.0f) ||
      !(t.kappa < 1.0f) || !(t.gamma_min > 0.0f) || !(t.gamma_min <= 1.0f) || !(t.gamma > 0.0f) ||
      !(t.gamma <= 1.0f))
    return fail(ctx, NGPRT_E_INVALID_ARG, "bad auto-tuning parameters");
  long long total = 0;
  int rc = sum_counts(ctx, n_rays, dev_n_samples, &total, (hipStream_t)stream);
  if (rc) return rc;
  // Eq. S3, in double precision on the host
  const double mean = double(total) / double(n_rays);
  double g = t.gamma;
  g = mean >= double(t.n_min) ? std::min(1.0, (1.0 + double(t.kappa)) * g)
                              : std::max(double(t.gamma_min), (1.0 - double(t.kappa)) * g);
  const float gf = float(g);
  const float step = float(double(gf) * double(t.s0));
  ngprt_desc d = ctx->desc;
  d.step = step;
  if (ngprt_validate_desc(&d) != NGPRT_OK) return fail(ctx, NGPRT_E_INVALID_ARG, "auto-tuned step is invalid");
  ctx->desc.step = step;
  tuner->gamma = gf;
  tuner->mean_samples = float(mean);
  return NGPRT_OK;
}

int ngprt_set_step(ngprt_ctx* ctx, float step) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  ngprt_desc d = ctx->desc;
  d.step = step;
  if (ngprt_validate_desc(&d) != NGPRT_OK) return fail(ctx, NGPRT_E_INVALID_ARG, "invalid step");
  ctx->desc.step = step;
  return NGPRT_OK;
}

int ngprt_adam_step(int64_t n, float* dev_param, const float* dev_grad, float* dev_m, float* dev_v,
                    int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1) return NGPRT_E_INVALID_ARG;
  if (n == 0) return NGPRT_OK;
  if (!dev_param || !dev_grad || !dev_m || !dev_v) return NGPRT_E_INVALID_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
      !std::isfinite(lr))
    return NGPRT_E_INVALID_ARG;
  return launch_adam(n, dev_param, dev_grad, dev_m, dev_v, step, lr, beta1, beta2, eps,
                     (hipStream_t)stream);
}

int ngprt_proposal_infer(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                         const float* dev_params, float* dev_out, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 0) return fail(ctx, NGPRT_E_INVALID_ARG, "n_rays < 0");
  if (n_rays == 0) return NGPRT_OK;
  if (!dev_origins || !dev_dirs || !dev_params || !dev_out)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  return launch_prop_infer(ctx, n_rays, dev_origins, dev_dirs, dev_params, dev_out, (hipStream_t)stream);
}

int ngprt_proposal_train_step(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                              const float* dev_dirs, const float* dev_labels, int32_t phase, float margin,
                              float* dev_params, float* dev_m, float* dev_v, int32_t step, float lr,
                              float* dev_loss, float* dev_grad, void* stream) {
  if (!ctx) return NGPRT_E_INVALID_ARG;
  if (n_rays < 1) return fail(ctx, NGPRT_E_INVALID_ARG, "empty batch");
  if (!dev_origins || !dev_dirs || !dev_labels || !dev_params)
    return fail(ctx, NGPRT_E_INVALID_ARG, "NULL pointer");
  if (phase != 1 && phase != 2) return fail(ctx, NGPRT_E_INVALID_ARG, "phase must be 1 or 2");
  if ((dev_m == nullptr) != (dev_v == nullptr)) return fail(ctx, NGPRT_E_INVALID_ARG, "m and v go together");
  if (dev_m && step < 1) return fail(ctx, NGPRT_E_INVALID_ARG, "step must be >= 1");
  if (!std::isfinite(lr) || !std::isfinite(margin)) return fail(ctx, NGPRT_E_INVALID_ARG, "bad lr/margin");
  return launch_prop_train(ctx, n_rays, dev_origins, dev_dirs, dev_labels, phase, margin, dev_params, dev_m,
                           dev_v, step, lr, dev_loss, dev_grad, (hipStream_t)stream);
}

}  // extern "C"
