// Internal types shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>

#include "../../include/ngprt.h"

namespace ngprt {

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };
enum { DOM_BOX = 0, DOM_CONTRACT = 1 };
constexpr int kMaxLevels = NGPRT_MAX_LEVELS;
constexpr int kMlpParams = 451;          // deferred MLP 7 -> 16 -> 16 -> 3
constexpr int kMlpViewParams = 5891;     // view-dependent MLP 23 -> 64 -> 64 -> 3
constexpr int kMlpViewRec = 8960;        // its weights arranged for the MFMA sequence
constexpr int kMaxLattice = 1 << 16;   // hard bound on lattice points per ray
constexpr int kMaxPyr = 5;             // occupancy pyramid levels

// channels per coarse vertex of the baked model: f~ (8) and the attention
// parameters stored per vertex (2L separate, L shared, none for constant
// gates or SUM)
inline int coarse_channels(const ngprt_desc& d) {
  return 8 + (d.aggregation == NGPRT_AGG_SEPARATE_V ? 2 * d.n_levels
              : d.aggregation == NGPRT_AGG_SHARED_V ? d.n_levels : 0);
}
// floats per coarse atlas row: C channels rounded up to whole float4 loads
// (8, 12 or 16)
inline int coarse_row_floats(int C) { return (C + 3) / 4 * 4; }

// Scene constants passed by value to kernels (lands in scalar registers).
struct SceneArgs {
  int L;
  int log2T;
  uint32_t mask;
  int N[kMaxLevels];
  float Nf[kMaxLevels];
  float scale[kMaxLevels][9];     // FP8 dequantisation scales (1 otherwise)
  const void* feat;               // [L][T][8] storage dtype
  const void* logit;              // [L][T]    storage dtype
  const uint16_t* grid;           // [R^3]: low byte G, bit 8 = occupied
  int R;
  float Rf;
  float lo;                       // grid covers [lo, -lo]^3
  float inv_ext;                  // 1 / (2 * roi_half)
  float vox;                      // voxel edge (grid-domain units)
  float v_over_step;              // vox / step
  float step;
  float thr;
  int max_samples;
  // baked feature model (model = 1): block-sparse coarse vertex grid
  int model;
  int LC;                         // coarse resolution (vertices 0..LC per axis)
  float LCf;
  int nb;                         // blocks per axis, ceil((LC + 1) / 8)
  int Cpad;                       // floats per atlas row (12 or 16)
  const int32_t* cidx;            // [nb^3] atlas row of each block or -1
  const float* catlas;            // [n_blocks][512][Cpad]
  int64_t n_blocks;               // atlas rows
  float cdef[16];                 // value of every vertex of an empty block
  // aggregation other than Separate-Att (V) (gen = 1): fine level l's gate
  // parameters are coarse channel gidx[l][0 / 1] (density / colour), or
  // the constant gconst[l][0 / 1] where that index is -1 (SUM: +inf, so
  // the sigmoid is exactly 1)
  int gen;
  int gidx[4][2];
  float gconst[4][2];
  // multi-level occupancy (pyr_n > 0): bit grids, level j of resolution pyrR[j]
  int pyr_n;
  int pyr_jg;                     // pyramid level of the distance grid's resolution; its words hold
                                  // in bits 9-11 the coarsest empty level >= pyr_jg (1 + level - pyr_jg,
                                  // 0: all occupied)
  int use_dist;                   // consult the distance grid (Eq. 9) when the exiting level is coarser
  int view_mlp;                   // the deferred MLP is the view-dependent one (a separate pass)
  int pyrR[kMaxPyr];
  const uint32_t* pyr[kMaxPyr];   // [R^3 / 32] words, x fastest, bit x & 31
  // pyramid whose distance grid is one level above the finest (pyr_jg == 1),
  // else NULL: per voxel of the distance grid the word of `grid` in bits
  // 0-15 and, in bit 16 + (x & 1) + 2 (y & 1) + 4 (z & 1), whether the finest
  // level's child (x, y, z) is occupied, so one read decides every level
  const uint32_t* pwide;
};

struct RayOut {
  float* rgb;
  float* c_d;
  float* feat;
  float* t_final;
  float* depth;
  int32_t* n_samples;
  int32_t* n_reads;
  float* t_first;
  float* t_far;
  float* t_half;
  float* dist_loss;
  float* proposal;
};

}  // namespace ngprt

struct ngprt_ctx {
  ngprt_desc desc;
  int device = 0;
  int64_t T = 0;
  void* feat = nullptr;       // [L][T][8]
  void* logit = nullptr;      // [L][T]
  float* scales_dev = nullptr;// [16][9] scales
  float scales_host[NGPRT_MAX_LEVELS][9];
  uint16_t* grid = nullptr;   // [R^3]
  float* mlp = nullptr;       // [451] or, view-dependent MLP, [5891]
  float* mlp_rec = nullptr;   // view-dependent MLP: weights in MFMA order [8960]
  void* ws = nullptr;         // workspace (per-wave gradient partials of backward / proposal)
  size_t ws_bytes = 0;
  void* prop_wb = nullptr;    // proposal weights in bfloat16 [7556]
  void* prop_net = nullptr;   // loaded proposal network: A-operand tiles [32][64] uint2 + biases [132]
  void* prop_tmp = nullptr;   // the same layout for ngprt_proposal_infer's caller-owned weights
  bool prop_loaded = false;
  void* count_ws = nullptr;   // step auto-tuning: per-block partial sums of sample counts + total
  int vmlp_resident = 0;      // view_mlp_kernel workgroups resident together (0: not yet queried)
  bool det_grad = false;      // table gradients by sorted segment sums instead of atomics
  void* prop_grad = nullptr;  // proposal gradient [7556] when the caller wants none
  int32_t* cidx = nullptr;    // baked model: block index grid [nb^3]
  float* catlas = nullptr;    // baked model: atlas [n_blocks][512][Cpad]
  int64_t n_blocks = 0;
  float cdef[16] = {};
  bool coarse_loaded = false;
  uint32_t* pyr[5] = {};      // occupancy pyramid bit grids
  uint32_t* pwide = nullptr;  // [R^3] distance-grid words with the finest level's child bits
  bool pyr_loaded = false;
  bool tables_loaded = false;
  bool occ_loaded = false;
  bool mlp_loaded = false;
  std::string last_error;
};

namespace ngprt {
int fail(ngprt_ctx* ctx, int code, const std::string& msg);
int check_launch(ngprt_ctx* ctx, const char* what);
SceneArgs scene_args(const ngprt_ctx* ctx);

// launchers (defined in the kernel translation units)
int launch_build_distance(ngprt_ctx* ctx, const uint8_t* occ, const uint8_t* dist, hipStream_t s);
int launch_export_distance(ngprt_ctx* ctx, uint8_t* out, hipStream_t s);
int launch_load_tables(ngprt_ctx* ctx, const float* tables, hipStream_t s);
int launch_export_tables(ngprt_ctx* ctx, void* codes, float* scales, hipStream_t s);
// prop: per-ray proposals [n][4] given by the caller, or use_net: the network
// loaded by ngprt_proposal_load runs in the kernel (its outputs to prop_out)
int launch_render(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const RayOut& out,
                  const float* prop, bool use_net, float* prop_out, const ngprt_proposal_cfg& pc,
                  int32_t* fallback, hipStream_t s);
int launch_eval_points(ngprt_ctx* ctx, int64_t n, const float* pos, int32_t* idx, float* fused,
                       float* weights, hipStream_t s);
int launch_march(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, int32_t cap,
                 int32_t* sk, int32_t* ns, int32_t* nr, int naive, hipStream_t s);
// Deterministic table gradients: the backward writes every corner
// contribution (key = level * T + entry, 9 values) to record
// ((off[ray] + sample) * L + level) * 8 + corner instead of adding it.
struct DetRecords {
  const int64_t* off = nullptr;   // per ray: its first sample's index among all samples; NULL: off
  uint32_t* keys = nullptr;
  uint32_t* order = nullptr;      // record index (the sort's payload)
  float* vals = nullptr;          // [records][9]
  int64_t n = 0;                  // records; an index at or beyond is not written
};
// fcd, ffv: the forward's per-ray C_d [n][3] and F [n][4], or NULL (pass 1
// recomputes them); given only without grad_dist
int launch_backward(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                    const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                    float* gtab, float* gatlas, float* gmlp, hipStream_t s);
// workspace of launch_backward_ws: one MLP-gradient partial per wave of 64
// rays plus kSumGroups group sums, every element written before it is read
size_t backward_workspace_bytes(int64_t n);
int launch_backward_ws(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                       const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                       float* gtab, float* gatlas, float* gmlp, float* workspace, hipStream_t s,
                       const DetRecords& det = DetRecords());
// the same with deterministic table gradients (hash model; allocates the
// records, synchronises the stream)
int launch_backward_det(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* grad_rgb,
                        const float* grad_dist, const float* ups, const float* fcd, const float* ffv,
                        float* gtab, float* gmlp, float* workspace, hipStream_t s);
int init_static_scratch(ngprt_ctx* ctx);
// Every device allocation of the library goes through these two, so that a
// test can make one fail (ngprt_test_fail_alloc).
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s);
// sum of n int32 counts on the GPU in a fixed order; synchronises the stream
int sum_counts(ngprt_ctx* ctx, int64_t n, const int32_t* counts, long long* host_total, hipStream_t s);
int check_backward_args(ngprt_ctx* ctx, const float* o, const float* d, const float* grad_rgb,
                        const float* grad_tables, const float* grad_mlp);
int launch_view_mlp_backward(ngprt_ctx* ctx, int64_t n, const float* d, const float* c_d, const float* feat,
                             const float* grad_rgb, float* grad_cf, float* gmlp, hipStream_t s);
int launch_view_mlp_arrange(ngprt_ctx* ctx, const float* params, hipStream_t s);
int launch_view_mlp(ngprt_ctx* ctx, int64_t n, const float* d, const float* c_d, const float* feat,
                    float* rgb, hipStream_t s);
int launch_build_pyramid(ngprt_ctx* ctx, const uint8_t* occ_fine, hipStream_t s);
int launch_pack_atlas(ngprt_ctx* ctx, const float* atlas, int64_t n_blocks, hipStream_t s);
int launch_gather_probe(ngprt_ctx* ctx, int64_t n, uint32_t seed, int pairs, float* out, hipStream_t s);
int launch_adam(int64_t n, float* p, const float* g, float* m, float* v, int32_t step, float lr,
                float b1, float b2, float eps, hipStream_t s);
int launch_prop_arrange(ngprt_ctx* ctx, const float* P, void* dst, hipStream_t s);
int load_proposal(ngprt_ctx* ctx, const float* P, hipStream_t s);
int launch_prop_infer(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* P,
                      float* out, hipStream_t s);
int launch_prop_train(ngprt_ctx* ctx, int64_t n, const float* o, const float* d, const float* labels,
                      int phase, float margin, float* P, float* m, float* v, int32_t step, float lr,
                      float* loss, float* grad_out, hipStream_t s);
}  // namespace ngprt
