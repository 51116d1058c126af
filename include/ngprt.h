/*
 * ngprt.h -- C ABI of the MI355X (gfx950) NGP-RT rendering library.
 *
 * The library renders rays through a baked NGP-RT-style scene (arXiv
 * 2407.10482): it marches each ray with an occupancy grid (or pyramid) and
 * the occupancy distance grid (Sec. 4.3, Eq. 9), looks up every level of
 * multi-level hash tables of explicit deferred features at each occupied
 * sample (Sec. 4.1, Eq. 6; Sec. 3, Eq. 3), fuses the levels with attention
 * (Sec. 4.2, Eq. 7-8: a softmax over per-entry logits, or the paper's
 * sigmoid gates from a baked coarse grid), composites front to back
 * (Sec. 3, Eq. 2 and Eq. 5) and runs one deferred MLP per ray (Eq. 5,
 * optionally view-dependent).  Backward entry points give the gradients of
 * a loss through all of it, for training.
 *
 * Conventions
 *  - Every pointer named dev_* is device memory on the current HIP device.
 *    Host pointers are named host_* or are plain structs.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call that
 *    takes a stream only enqueues work on it and returns; results are valid
 *    once the stream has passed the call.  No call synchronises the device
 *    except ngprt_create / ngprt_destroy and the load functions (which may).
 *  - The library owns the scene: load_* copy (and re-layout / quantise) the
 *    caller's buffers into library memory; the caller may free its buffers
 *    once the stream has passed the call.  Render calls borrow the ray and
 *    output pointers only for the duration of the enqueued work.
 *  - Every function returns NGPRT_OK (0) or a negative NGPRT_E_* code.  No
 *    C++ exception crosses this boundary.  ngprt_last_error() holds a
 *    message for the most recent failure on a context.
 *  - A context is not thread-safe; calls that overlap on one context race.
 *
 * Arithmetic contract
 *  - Integer outputs (hash indices, the distance grid, sample lattice
 *    indices, sample and read counts, quantised table bytes) are exact.
 *  - The chain that decides them (positions, voxel and corner indices,
 *    trilinear weights, interpolated density and logits, the softmax across
 *    levels, the density activation and transmittance) uses IEEE float32
 *    add/sub/mul/div/sqrt without contraction, a fixed summation order and a
 *    library-defined exponential, so it is reproducible off the GPU.
 */
#ifndef NGPRT_H
#define NGPRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NGPRT_MAX_LEVELS 16

enum ngprt_status {
  NGPRT_OK = 0,
  NGPRT_E_INVALID_ARG = -1, /* null pointer, bad enum, negative count */
  NGPRT_E_SHAPE = -2,       /* sizes inconsistent with the descriptor */
  NGPRT_E_DTYPE = -3,       /* unsupported table dtype */
  NGPRT_E_NOT_LOADED = -4,  /* render before tables / occupancy / MLP were loaded */
  NGPRT_E_ALLOC = -5,       /* device allocation failed */
  NGPRT_E_HIP = -6,         /* a HIP runtime call or kernel launch failed */
  NGPRT_E_UNSUPPORTED = -7  /* valid request the library does not implement */
};

enum ngprt_dtype { NGPRT_F32 = 0, NGPRT_BF16 = 1, NGPRT_FP8E4M3 = 2 };

enum ngprt_domain {
  /* Axis-aligned cube ROI [-roi_half, roi_half]^3; straight lattice
   * t_k = t0 + k*step from the ray's entry t0. */
  NGPRT_ROI_BOX = 0,
  /* Unbounded scene contracted into the ball of radius 2
   * (x -> x for |x| <= 1, (2 - 1/|x|) x/|x| otherwise); the grids cover
   * [-2, 2]^3 (roi_half must be 2); lattice of equal contracted arc length
   * starting at t = 0. */
  NGPRT_ROI_CONTRACT = 1
};

enum ngprt_feature_model {
  /* Every level a hash level of 8 feature channels + 1 attention logit;
   * the levels are fused by a softmax over the interpolated logits. */
  NGPRT_MODEL_HASH = 0,
  /* The paper's construction (Sec. 4.1 Eq. 6; Sec. 4.2 Eq. 7-8): a coarse
   * vertex grid of resolution L_C (loaded by ngprt_load_coarse) holds the
   * deferred features f~ and per-level attention parameters (omega_l,
   * beta_l); n_levels (1..4) fine hash levels hold 8-channel features f^_l;
   * f = f~ + [sum_l sigmoid(omega_l) sigma^_l, sum_l sigmoid(beta_l) c^_l,
   * sum_l sigmoid(beta_l) v^_l]. */
  NGPRT_MODEL_BAKED = 1
};

/* How NGPRT_MODEL_BAKED fuses the fine levels (the aggregation variants the
 * paper ablates in Sec. 5.2, Table 3).  g is the sigmoid; s_l = sigma^_l,
 * c_l = [c^_l, v^_l]. */
enum ngprt_aggregation {
  /* Separate-Att (V), the paper's design (Eq. 7-8): omega_l, beta_l stored
   * per coarse vertex; f^ = [sum g(omega_l) s_l, sum g(beta_l) c_l]. */
  NGPRT_AGG_SEPARATE_V = 0,
  /* Shared-Att (V): one a_l per coarse vertex gates both modalities. */
  NGPRT_AGG_SHARED_V = 1,
  /* Separate-Att (Inv): omega_l, beta_l are scene constants
   * (desc.gate_params = [omega_1, beta_1, ..., omega_L, beta_L]). */
  NGPRT_AGG_SEPARATE_INV = 2,
  /* Shared-Att (Inv): a_l scene constants (desc.gate_params = [a_1..a_L]). */
  NGPRT_AGG_SHARED_INV = 3,
  /* SUM (MERF's aggregation): f^ = sum_l f^_l, no gates. */
  NGPRT_AGG_SUM = 4
};

/* Scene descriptor (copied by ngprt_create). */
typedef struct ngprt_desc {
  int32_t n_levels;                          /* L, 1..16 */
  int32_t resolutions[NGPRT_MAX_LEVELS];     /* N_l per level, >= 1 (explicit integers) */
  int32_t log2_table_size;                   /* T = 1 << log2_table_size, 4..24 */
  int32_t table_dtype;                       /* enum ngprt_dtype: storage of the tables */
  int32_t domain;                            /* enum ngprt_domain */
  float roi_half;                            /* grid extent; a power of two */
  int32_t occ_res;                           /* R: occupancy / distance grids are R^3, 2..1024 */
  float step;                                /* lattice step (box: world units; contract: contracted units) */
  int32_t max_samples;                       /* cap on evaluated samples per ray, >= 1 */
  float t_threshold;                         /* stop once T < t_threshold; 0 disables */
  int32_t mlp_in, mlp_hidden, mlp_out;       /* 7, 16, 3: the deferred MLP of C_d, F;
                                              * 23, 64, 3: the view-dependent MLP_psi of
                                              * C_d, F and SH(d) (see ngprt_load_mlp) */
  int32_t feature_model;                     /* enum ngprt_feature_model */
  int32_t coarse_res;                        /* L_C of NGPRT_MODEL_BAKED, 1..2048 (else ignored) */
  int32_t occ_levels;      /* 0: one occupancy grid of occ_res (ngprt_load_occupancy); 2..5: an
                            * occupancy pyramid of occ_levels levels whose finest has
                            * occ_fine_res (ngprt_load_occupancy_pyramid) */
  int32_t occ_fine_res;    /* pyramid: finest resolution, a power of two <= 1024 with
                            * occ_fine_res >> (occ_levels - 1) >= 32; occ_res must be one of
                            * the pyramid's resolutions (the distance grid's) */
  int32_t use_distance;    /* pyramid: 1 = consult the distance grid (Eq. 9), 0 = pyramid only */
  int32_t aggregation;     /* NGPRT_MODEL_BAKED: enum ngprt_aggregation (0 for the hash model);
                            * other than NGPRT_AGG_SEPARATE_V needs float32 tables and has no
                            * backward */
  float gate_params[8];    /* NGPRT_AGG_SEPARATE_INV / _SHARED_INV: the 2L / L attention
                            * parameters before their sigmoid, finite; else ignored */
} ngprt_desc;

typedef struct ngprt_ctx ngprt_ctx;

/* Optional per-ray outputs of ngprt_render.  rgb is required; NULL skips a field. */
typedef struct ngprt_outputs {
  float* rgb;        /* [n][3] sigmoid(C_d + MLP(C_d, F))           (Eq. 5) */
  float* c_d;        /* [n][3] composited diffuse colour C_d          (Eq. 5) */
  float* feat;       /* [n][4] composited specular feature F          (Eq. 5) */
  float* t_final;    /* [n]    transmittance after the last sample    (Eq. 2) */
  float* depth;      /* [n]    sum_i w_i t_i */
  int32_t* n_samples;/* [n]    evaluated (occupied) samples */
  int32_t* n_reads;  /* [n]    occupancy/distance grid reads (marching points) */
  float* t_first;    /* [n]    t of the first evaluated sample (0 if none) */
  float* t_far;      /* [n]    t of the sample after which T < 1e-3 (the last sample's t if
                      *        never; 0 if no sample): the proposal's far-end label */
  float* t_half;     /* [n]    t of the sample after which T < 0.5 (last sample's t if never) */
  float* dist_loss;  /* [n]    distortion regulariser of the ray (supplement Eq. S2) over its
                      *        rendering weights w_i on the lattice intervals
                      *        [k_i step, (k_i + 1) step] (k_i the sample's lattice index):
                      *        sum_ij w_i w_j |m_i - m_j| + step/3 sum_i w_i^2, m_i = (k_i + 1/2) step */
  float* proposal;   /* [n][4] ngprt_render_proposal only: the loaded network's t_near, t_far,
                      *        t_term and sigmoid(confidence logit) for the ray */
} ngprt_outputs;

/* Create a context on the current HIP device.  Validates the descriptor
 * (host only).  *out is set only on success. */
int ngprt_create(const ngprt_desc* desc, ngprt_ctx** out);

/* Free the context and all library-owned device memory (synchronises). */
void ngprt_destroy(ngprt_ctx* ctx);

/* Validate a descriptor without creating anything (host only). */
int ngprt_validate_desc(const ngprt_desc* desc);

/* Load hash tables from float32 [L][T][9] (channels sigma_raw, r, g, b,
 * s0..s3, logit; Sec. 4.1 explicit deferred features plus one attention
 * logit per entry) and store them in desc.table_dtype:
 *  F32 as is; BF16 round-to-nearest-even; FP8E4M3 (OCP E4M3FN) with one
 *  float32 scale per (level, channel), s = amax/448 (1 if amax = 0),
 *  code = RNE-saturate(x / s).  Stored internally as a feature array
 *  [L][T][8] and a logit array [L][T]. */
int ngprt_load_tables(ngprt_ctx* ctx, const float* dev_tables, void* stream);

/* NGPRT_MODEL_BAKED: load the coarse grid (Sec. 4.1: the baked grids F~ and
 * A of resolution L_C, stored together).  Vertices (vx, vy, vz), 0 <= v <=
 * L_C, are grouped in blocks of 8^3; nb = ceil((L_C + 1) / 8).
 *  dev_block_index  int32 [nb][nb][nb] (z, y, x): the block's row in the
 *                   atlas, or -1 for an empty block; every entry must be in
 *                   [-1, n_blocks) (checked on the host: the index grid is
 *                   copied back once; otherwise NGPRT_E_INVALID_ARG).
 *  dev_atlas        float32 [n_blocks][8][8][8][C] (z, y, x inside the
 *                   block), C = 8 + 2L channels [sigma~, r, g, b, s0..s3,
 *                   omega_1, beta_1, ..., omega_L, beta_L] (attention
 *                   parameters before their sigmoid); NULL if n_blocks = 0.
 *                   NGPRT_AGG_SHARED_V: C = 8 + L, [f~, a_1..a_L];
 *                   the constant-gate and SUM aggregations: C = 8, [f~].
 *  host_default     float32 [C]: the value of every vertex of an empty block.
 * The fine levels are loaded by ngprt_load_tables in the same [L][T][9]
 * layout as the hash model, channel 8 unused.  Synchronises the stream.
 * NGPRT_MODEL_HASH contexts return NGPRT_E_UNSUPPORTED. */
int ngprt_load_coarse(ngprt_ctx* ctx, int64_t n_blocks, const int32_t* dev_block_index,
                      const float* dev_atlas, const float* host_default, void* stream);

/* Read back the stored tables as [L][T][9] in the storage dtype
 * (float32 / bf16 bits / e4m3 bytes) and, for FP8, the scales [L][9]
 * (dev_scales may be NULL otherwise). */
int ngprt_export_tables(ngprt_ctx* ctx, void* dev_codes, float* dev_scales, void* stream);

/* Load the occupancy grid (uint8 [R][R][R], x fastest, nonzero = occupied).
 * dev_dist: the occupancy distance grid G (uint8 [R^3]) or NULL to build it
 * on the GPU: G = min(255, floor(box-gap distance in voxels to the nearest
 * occupied voxel)), 0 for occupied voxels and their 26 neighbours, 255 when
 * nothing is occupied (Sec. 4.3). */
int ngprt_load_occupancy(ngprt_ctx* ctx, const uint8_t* dev_occ, const uint8_t* dev_dist,
                         void* stream);

/* Multi-level occupancy (Sec. 4.3: the march that Eq. 9's s_O refers to;
 * supplement "Real-time Rendering" item 1: five levels 512^3 ... 32^3).
 * dev_occ_fine: uint8 [F][F][F] (F = occ_fine_res, x fastest, nonzero =
 * occupied).  Level j (resolution F >> j) marks a voxel occupied when any of
 * its 8 children is; the distance grid G is built from the level of
 * resolution occ_res as in ngprt_load_occupancy.  The march reads the levels
 * coarse to fine at each lattice point not known to be empty; a sample is
 * taken where the finest level is occupied; otherwise the march skips the
 * exiting level's voxel (box: to one lattice step before its exit along the
 * ray; contracted domain: the ball inscribed in it, less voxel/1024) or, when
 * use_distance is set and the exiting level is coarser than G, by the G rule
 * if that skips further.  The sampled lattice points are those of an
 * exhaustive march over the finest level.  Needs occ_levels > 0
 * (NGPRT_E_UNSUPPORTED otherwise); ngprt_load_occupancy then returns
 * NGPRT_E_UNSUPPORTED.  Device memory held: the levels (F^3 / 8 bytes for
 * the finest, an eighth of that for each next), the G grid (2 R^3 bytes) and,
 * when occ_res = F / 2, a 4 R^3-byte copy of G's words that also carries each
 * voxel's 8 finest-level children, so the march decides a lattice point with
 * one read; allocated by the first call, reused by later ones
 * (NGPRT_E_ALLOC if an allocation fails; the context then has no occupancy
 * until a load succeeds). */
int ngprt_load_occupancy_pyramid(ngprt_ctx* ctx, const uint8_t* dev_occ_fine, void* stream);

/* Copy the distance grid in use to dev_dist (uint8 [R^3]). */
int ngprt_export_distance(ngprt_ctx* ctx, uint8_t* dev_dist, void* stream);

/* Load the deferred MLP (Eq. 5): float32 W0[16][7], b0[16], W1[16][16],
 * b1[16], W2[3][16], b2[3] (451 values, row-major, out x in), input
 * [C_d, F].  With mlp_hidden = 64 it is the view-dependent MLP_psi (Eq. 5;
 * supplement "Network Design"): W0[64][23], b0[64], W1[64][64], b1[64],
 * W2[3][64], b2[3] (5891 values), input [C_d, F, SH(d)] with SH(d) the 16
 * real spherical harmonics of degrees 0..3 of the normalised ray direction
 * (orthonormal, no Condon-Shortley phase; order l = 0..3, m = -l..l; zero for
 * a zero or non-finite direction).  That MLP runs as a pass after the march
 * over the C_d and F outputs, so ngprt_render / ngprt_render_proposal then
 * need out->c_d and out->feat (NGPRT_E_INVALID_ARG otherwise). */
int ngprt_load_mlp(ngprt_ctx* ctx, const float* dev_params, void* stream);

/* Render n_rays rays.  dev_origins, dev_dirs: float32 [n][3] (directions
 * need not be unit length; the lattice step is in units of t*|d| only for
 * the contracted domain).  Rays with a non-finite component, a zero
 * direction, or missing the ROI get zero samples and rgb = sigmoid(MLP(0)).
 * n_rays = 0 is a no-op. */
int ngprt_render(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                 const float* dev_dirs, const ngprt_outputs* out, void* stream);

/* How a per-ray sample-interval proposal [t_near, t_far, t_term, conf]
 * restricts the march (an extension; see ngprt_render_proposal). */
typedef struct ngprt_proposal_cfg {
  float conf_threshold; /* rays with conf >= conf_threshold use their proposal */
  float margin;         /* padding of the interval, in t units, finite and >= 0 */
  int32_t use_near;     /* 1: skip the lattice points before t_near - margin; 0: march from the start */
  float far_guard;      /* <= 0: a lattice point beyond t_far + margin ends the ray; > 0: it ends the
                         * ray only when the ray's transmittance is below far_guard (so the colour
                         * weight dropped is below far_guard), otherwise the ray marches on */
} ngprt_proposal_cfg;

/* Render with the learned per-ray sample-interval proposal (an extension;
 * the network is described at ngprt_proposal_infer and loaded by
 * ngprt_proposal_load, NGPRT_E_NOT_LOADED otherwise).  The render kernel
 * runs the network for its rays before marching (no separate pass; the
 * outputs go to out->proposal when given).  A ray whose confidence reaches
 * cfg->conf_threshold marches only the lattice points with t in
 * [t_near - margin, t_far + margin] of the plain render's lattice (the far
 * end subject to cfg->far_guard): with cfg->use_near, in the box domain from
 * lattice index max(0, floor((t_near - margin - t0) / step)), t0 the ROI
 * entry, and in the contracted domain lattice points before t_near - margin
 * are visited without a grid read.  A proposed ray that takes no sample in
 * its interval marches again from its start as the plain march, so its
 * result is the plain render's bit for bit (dev_fallback, int32 [n]
 * NULL-able, marks those rays; out->n_reads counts the reads of both
 * marches).  Other rays march plainly.  A NULL or invalid cfg ->
 * NGPRT_E_INVALID_ARG. */
int ngprt_render_proposal(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                          const float* dev_dirs, const ngprt_proposal_cfg* cfg,
                          const ngprt_outputs* out, int32_t* dev_fallback, void* stream);

/* ngprt_render_proposal with the proposals given per ray instead of the
 * loaded network: dev_proposal, float32 [n][4] = t_near, t_far, t_term,
 * confidence (out->proposal is ignored). */
int ngprt_render_intervals(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                           const float* dev_dirs, const float* dev_proposal,
                           const ngprt_proposal_cfg* cfg, const ngprt_outputs* out,
                           int32_t* dev_fallback, void* stream);

/* Load the proposal network's float32 master weights [7556] (the layout of
 * ngprt_proposal_infer) for ngprt_render_proposal: copied into library
 * memory as bfloat16 (round to nearest even) product operands and float32
 * biases; the caller may free or update its buffer once the stream has
 * passed the call (load again after training steps). */
int ngprt_proposal_load(ngprt_ctx* ctx, const float* dev_params, void* stream);

/* Parity helpers.  Evaluate the lookup + attention chain at n positions in
 * the grid's domain (box: world coordinates; contract: contracted
 * coordinates).  Any output may be NULL: dev_idx int32 [n][L][8] corner
 * table indices, dev_fused float32 [n][8] fused channels, dev_weights
 * float32 [n][L] attention weights. */
int ngprt_debug_eval_points(ngprt_ctx* ctx, int64_t n, const float* dev_pos, int32_t* dev_idx,
                            float* dev_fused, float* dev_weights, void* stream);

/* Gather ceiling probe (measurement aid, not on the render path).  For each
 * of n_points pseudo-random "samples" (stream `seed`), gathers, per level of
 * the loaded tables, 8 feature rows + logits at random entries of that level
 * (pairs = 0: all independent; pairs = 1: 4 random entries e and their
 * neighbours e ^ 1, the placement of a cell's two x-adjacent corners under
 * the spatial hash of the multiresolution hash encoding, Sec. 3 of the
 * paper, when the cell's x index is even), dequantises them like the render
 * path and writes their float32 sum to dev_out [n_points].  Requested bytes
 * per point equal a render sample's: L * 8 * (row + logit) bytes.  Tables
 * must be loaded; NULL dev_out or pairs outside {0, 1} -> INVALID_ARG. */
int ngprt_gather_probe(ngprt_ctx* ctx, int64_t n_points, uint32_t seed, int32_t pairs, float* dev_out,
                       void* stream);

/* March only (no MLP): per ray, the lattice indices of the first `cap`
 * evaluated samples (dev_sample_k int32 [n][cap], -1 padded), the sample
 * count and the grid-read count.  naive != 0 reads every lattice point
 * instead of skipping with the distance grid. */
int ngprt_debug_march(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                      const float* dev_dirs, int32_t cap, int32_t* dev_sample_k,
                      int32_t* dev_n_samples, int32_t* dev_n_reads, int32_t naive, void* stream);

/* Gradients of a loss through ngprt_render (a training extension).
 * dev_grad_rgb: float32 [n][3] dL/drgb.  Accumulates (+=) dL/dtables into
 * dev_grad_tables, float32 [L][T][9] in the layout ngprt_load_tables takes,
 * and dL/dmlp into dev_grad_mlp, float32 [451]; the caller zeroes them.
 * The forward is recomputed per ray (two re-marches, no per-sample state;
 * ngprt_render_backward_fwd takes the forward's C_d and F and needs one);
 * table gradients are summed with float atomics, so their low bits depend
 * on execution order (ngprt_set_deterministic_gradients removes that).  Needs float32 tables (NGPRT_E_DTYPE otherwise) and
 * the hash feature model (NGPRT_E_UNSUPPORTED for NGPRT_MODEL_BAKED).  May
 * grow a library-owned workspace (stream-ordered allocation). */
int ngprt_render_backward(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                          const float* dev_dirs, const float* dev_grad_rgb, float* dev_grad_tables,
                          float* dev_grad_mlp, void* stream);

/* ngprt_render_backward with the distortion regulariser (supplement Eq. S2,
 * the per-ray value ngprt_render writes to out->dist_loss): dev_grad_dist,
 * float32 [n] (NULL = 0), is dL/d(dist_loss) per ray, so a loss
 * L_color + eta * sum_rays dist_loss takes dev_grad_dist = eta.  The
 * regulariser's gradient reaches the tables through the rendering weights
 * (dL/dw_i = g_r (2 sum_j w_j |m_i - m_j| + 2/3 step w_i)). */
int ngprt_render_backward_reg(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                              const float* dev_dirs, const float* dev_grad_rgb, const float* dev_grad_dist,
                              float* dev_grad_tables, float* dev_grad_mlp, void* stream);

/* The backward of ngprt_render_backward (hash model) or
 * ngprt_render_backward_baked (baked model; dev_grad_atlas as there, NULL
 * for the hash model), 7-16-16-3 deferred MLP, without the regulariser,
 * given the forward's per-ray composited features: dev_c_d float32 [n][3]
 * and dev_feat float32 [n][4] as ngprt_render wrote them to out->c_d and
 * out->feat for the same scene, MLP, step and rays (Eq. 5's C_d and F).
 * The backward then skips its first re-march, which recomputes exactly
 * these values, and gives the same gradients (the MLP gradient bit for
 * bit).  NULL dev_c_d or dev_feat -> NGPRT_E_INVALID_ARG; the other
 * conditions are those of the two entry points it stands for. */
int ngprt_render_backward_fwd(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins, const float* dev_dirs,
                              const float* dev_c_d, const float* dev_feat, const float* dev_grad_rgb,
                              float* dev_grad_tables, float* dev_grad_atlas, float* dev_grad_mlp, void* stream);

/* Deterministic table gradients, for gradient checks (off by default).
 * The backward adds float contributions with atomics, in an order that
 * varies from run to run, so a table gradient's last bits vary.  With on
 * != 0, the hash-model backward entry points of this context instead write
 * every corner contribution to a record of its own, sort the records by
 * table entry (stably, so each entry keeps the order ray, sample, level,
 * corner) and add each entry's records in that order: the same gradient
 * bit for bit on every run.  Slower; allocates about 52 bytes per
 * contribution (samples x L x 8 of them, at most NGPRT_DET_MAX_RECORDS per
 * call, else NGPRT_E_SHAPE) and synchronises the stream.  The baked model's
 * backward then returns NGPRT_E_UNSUPPORTED, as does
 * ngprt_render_backward_noalloc (it cannot allocate the records). */
#define NGPRT_DET_MAX_RECORDS 67108864
int ngprt_set_deterministic_gradients(ngprt_ctx* ctx, int on);

/* Test hook for failure handling (not for production use): after `after`
 * more successful device allocations by the library (any context, any
 * thread), the next one fails as if the device were out of memory, and the
 * hook disarms; after < 0 disarms it.  The call that meets the failure
 * returns NGPRT_E_ALLOC (ngprt_create: and no context) and leaves its
 * context usable.  Always NGPRT_OK. */
int ngprt_test_fail_alloc(int64_t after);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight training loops, hosts that forbid allocation): the same
 * computation as ngprt_render_backward_reg (same arguments, conditions and
 * results; the MLP gradient bit for bit), with its workspace in a static
 * device array of NGPRT_NOALLOC_SCRATCH_BYTES that each GPU holds from the
 * first ngprt_create on it until the process ends.  It allocates nothing.
 * n_rays above NGPRT_NOALLOC_MAX_RAYS -> NGPRT_E_SHAPE (nothing enqueued).
 * Every call on one GPU shares that array and the next call overwrites it:
 * calls that overlap on one GPU (other streams, threads or contexts) race,
 * so the caller serialises them.  Needs nothing cleared between calls. */
#define NGPRT_NOALLOC_MAX_RAYS 524288
#define NGPRT_NOALLOC_SCRATCH_BYTES 14893824 /* (MAX_RAYS / 64 + 64) * 451 floats */
int ngprt_render_backward_noalloc(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                                  const float* dev_dirs, const float* dev_grad_rgb,
                                  const float* dev_grad_dist, float* dev_grad_tables,
                                  float* dev_grad_mlp, void* stream);

/* ngprt_render_backward_reg for the baked feature model (Sec. 4.1 Eq. 6,
 * Sec. 4.2 Eq. 7-8): f = f~ + [sum_l g(omega_l) sigma^_l, sum_l g(beta_l)
 * c^_l, sum_l g(beta_l) v^_l], g the sigmoid.  Accumulates (+=)
 * dL/d(fine tables) into dev_grad_tables, float32 [L][T][9] (channel 8 is
 * not written: the baked model has no per-level logit), and dL/d(atlas)
 * into dev_grad_atlas, float32 [n_blocks][8][8][8][8 + 2L] in the layout
 * ngprt_load_coarse takes (NULL allowed when n_blocks = 0); the default
 * vector of empty blocks takes no gradient; dL/dmlp into dev_grad_mlp
 * [451].  The caller zeroes all three; the updated atlas is handed back
 * with ngprt_load_coarse (the library keeps a padded copy).  Atomics make
 * the low bits order-dependent, as for the hash model.  Needs float32
 * tables (NGPRT_E_DTYPE), NGPRT_MODEL_BAKED and the 7-16-16-3 MLP
 * (NGPRT_E_UNSUPPORTED otherwise); same workspace note. */
int ngprt_render_backward_baked(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                                const float* dev_dirs, const float* dev_grad_rgb, const float* dev_grad_dist,
                                float* dev_grad_tables, float* dev_grad_atlas, float* dev_grad_mlp,
                                void* stream);

/* Backward of the view-dependent MLP (Eq. 5; supplement "Network Design"),
 * rgb = sigmoid(C_d + MLP_psi(C_d, F, SH(d))), for contexts with the
 * 23-64-64-3 MLP (NGPRT_E_UNSUPPORTED otherwise).  Inputs per ray: the
 * directions, C_d [n][3] and F [n][4] as ngprt_render wrote them, dL/drgb
 * [n][3].  Writes dL/dC_d and dL/dF to dev_grad_cf, float32 [n][7]
 * (C_d first), and accumulates (+=) dL/dpsi into dev_grad_mlp [5891] (the
 * caller zeroes it; partial sums per 64 rays added in a fixed order).  SH(d)
 * is a constant input.  May grow the library workspace. */
int ngprt_view_mlp_backward(ngprt_ctx* ctx, int64_t n_rays, const float* dev_dirs, const float* dev_c_d,
                            const float* dev_feat, const float* dev_grad_rgb, float* dev_grad_cf,
                            float* dev_grad_mlp, void* stream);

/* The render backward from dL/dC_d and dL/dF per ray (dev_grad_cf, float32
 * [n][7], e.g. from ngprt_view_mlp_backward) instead of dL/drgb: the MLP
 * is not involved.  Accumulates (+=) dL/dtables into dev_grad_tables [L][T][9]
 * and, for NGPRT_MODEL_BAKED, dL/datlas into dev_grad_atlas (layouts and
 * conditions as ngprt_render_backward_reg / ngprt_render_backward_baked;
 * dev_grad_atlas is ignored for the hash model).  dev_grad_dist as in
 * ngprt_render_backward_reg.  dev_c_d [n][3] and dev_feat [n][4]: the
 * forward's composited C_d and F (out->c_d, out->feat of ngprt_render on
 * the same scene and rays), or both NULL; given, the first re-march that
 * recomputes them is skipped (same gradients).  Not with dev_grad_dist
 * (NGPRT_E_INVALID_ARG), nor one of the two alone. */
int ngprt_render_backward_features(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                                   const float* dev_dirs, const float* dev_grad_cf, const float* dev_grad_dist,
                                   float* dev_grad_tables, float* dev_grad_atlas, const float* dev_c_d,
                                   const float* dev_feat, void* stream);

/* Change the lattice step (the paper's marching-step auto-tuning,
 * supplement Eq. S3, scales it between training batches).  Same checks as
 * desc.step (NGPRT_E_INVALID_ARG).  Later calls use the new step. */
int ngprt_set_step(ngprt_ctx* ctx, float step);

/* Marching-step auto-tuning of the paper's training (supplement, "Auto-tuning
 * of Marching Step Size", Eq. S3), applied between training batches. */
typedef struct ngprt_step_tuner {
  float s0;           /* base step (the desc.step the scene was created with), > 0 */
  float n_min;        /* N_min: the mean sample count below which the step shrinks (paper: 3) */
  float kappa;        /* progressive multiplier, in [0, 1) (paper: 0.001) */
  float gamma_min;    /* lower bound of the scaler, in (0, 1] (paper: 0.2217) */
  float gamma;        /* the scaler, in (0, 1]; start at 1; updated by each call */
  float mean_samples; /* output: the batch's mean evaluated samples per ray */
} ngprt_step_tuner;

/* One auto-tuning update after a training batch: N = the mean of
 * dev_n_samples (int32 [n_rays], e.g. out->n_samples of the batch's render,
 * summed on the GPU in a fixed order); gamma <- min(1, (1 + kappa) gamma) if
 * N >= n_min, else max(gamma_min, (1 - kappa) gamma) (in double precision,
 * then rounded to float32); then the context's step becomes gamma * s0
 * rounded once to float32 (as ngprt_set_step; later calls use it).
 * Synchronises the stream (the host needs N).  Invalid parameters, an empty
 * batch or NULL pointers -> NGPRT_E_INVALID_ARG (nothing changed). */
int ngprt_step_autotune(ngprt_ctx* ctx, int64_t n_rays, const int32_t* dev_n_samples,
                        ngprt_step_tuner* tuner, void* stream);

/* One Adam update (Kingma & Ba; the paper's training uses beta1 = 0.9,
 * beta2 = 0.99, eps = 1e-8, supplement "Optimization") over n float32
 * parameters in place: m, v are the moment buffers (caller-owned, zero
 * before step 1), step >= 1 the 1-based step for bias correction. */
int ngprt_adam_step(int64_t n, float* dev_param, const float* dev_grad, float* dev_m, float* dev_v,
                    int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Learned per-ray sample-interval proposal (an extension; the paper names
 * adaptive sampling only as orthogonal related work, Sec. 2).  Network:
 * [o; d] -> Fourier features sin/cos(2^k pi r_j), k = 0..3 (48) -> 64 -> 64
 * -> 4 with ReLU; outputs t_near, t_far, t_term, confidence.  dev_params:
 * float32 master weights [7556] = W1[64][48], b1[64], W2[64][64], b2[64],
 * W3[4][64], b3[4], caller-owned.  Products run on bfloat16 operands with
 * float32 accumulation.  ctx provides workspace only (no scene needed). */

/* dev_out: float32 [n][4] = t_near, t_far, t_term, sigmoid(confidence logit). */
int ngprt_proposal_infer(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                         const float* dev_dirs, const float* dev_params, float* dev_out,
                         void* stream);

/* One training step on a batch of n_rays >= 1 rays.  dev_labels: float32
 * [n][4] = t_near, t_far, t_term, valid (1 for rays with samples, else 0).
 * Loss = (sum over valid rays of the pinball loss of t_near at quantile
 * 0.05 and of t_far at 0.95 plus the squared error of t_term, + for phase 2
 * the cross-entropy of the confidence against "the predicted interval
 * widened by margin contains [t_near, t_far]") / n.  Adds the batch
 * loss to dev_loss[0] (NULL-able); writes the gradient to dev_grad [7556]
 * (NULL-able); when dev_m and dev_v (Adam moments [7556], zero before step
 * 1) are given, applies Adam (beta1 0.9, beta2 0.99, eps 1e-8, step >= 1) to
 * dev_params in place.  Gradients are reduced in a fixed order. */
int ngprt_proposal_train_step(ngprt_ctx* ctx, int64_t n_rays, const float* dev_origins,
                              const float* dev_dirs, const float* dev_labels, int32_t phase,
                              float margin, float* dev_params, float* dev_m, float* dev_v,
                              int32_t step, float lr, float* dev_loss, float* dev_grad, void* stream);

/* Human-readable name of a status code (static storage). */
const char* ngprt_status_string(int status);

/* Message of the last failure on ctx ("" if none; static-lifetime while ctx lives). */
const char* ngprt_last_error(const ngprt_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* NGPRT_H */
