/*
 * dass.h -- C ABI of the MI355X (gfx950) hot path of per-timestep Gaussian-splatting
 * streaming (DASS, arXiv 2411.14847).
 *
 * The problem statement (Sec. 3.1): at timestep t, start from the Gaussians of t-1 and fit
 * them to C synchronised views, by rendering and back-propagating through the tile-based
 * differentiable rasterizer (App. A.1), shifting the dynamic Gaussians (Sec. 3.3), updating
 * with Adam, and appending Gaussians where the error is large (Sec. 3.4).
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller unless stated otherwise;
 *     structs passed by pointer (dass_gaussians, dass_camera, ...) live in HOST memory.
 *   - Layout is structure-of-arrays: a parameter with P components is P planes of
 *     `capacity` floats ("[P][capacity]"), so Gaussian g's component p is at p*capacity+g.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream) and the calls
 *     return before it finishes.  They never synchronise the host and never allocate
 *     (except dass_create / dass_reserve / dass_sync and the debug exports).
 *   - Errors are returned as dass_status, never thrown or aborted.  Arguments are checked
 *     before anything is enqueued (DASS_E_INVALID).  A request larger than the reserved
 *     limits returns DASS_E_CAPACITY at once when the host can tell; device-side overflow of
 *     the tile-key buffer is recorded on the device and returned by the next dass_sync().
 *     HIP launch failures return DASS_E_HIP; dass_last_error() then holds a message.
 *   - Gradient outputs ACCUMULATE (+=); the caller zeroes them.
 *   - One context per stream / host thread; calls on one context must not overlap.
 */
#ifndef DASS_H
#define DASS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dass_ctx_s* dass_ctx;
typedef void* dass_stream; /* hipStream_t */

typedef enum {
  DASS_OK = 0,
  DASS_E_INVALID = 1,     /* bad argument (null pointer, size out of range, ...)   */
  DASS_E_OOM = 2,         /* device allocation failed (create / reserve only)      */
  DASS_E_CAPACITY = 3,    /* request exceeds the reserved limits                   */
  DASS_E_HIP = 4,         /* a HIP call failed                                     */
  DASS_E_UNSUPPORTED = 5  /* valid request the library does not handle             */
} dass_status;

#define DASS_MAX_VIEWS 32  /* views per render call */
#define DASS_MAX_SH_DEGREE 3

/* Gaussians G_t = {G^base, G^var} (Sec. 3.1): rows [0, n_base) are the base set, rows
 * [n_base, n) the densified set.  Parametrisation (App. A.1): position mu, rotation
 * quaternion q = (w,x,y,z) (any non-zero norm; normalised inside), scale s = exp(log_scale),
 * opacity o = sigmoid(opacity_logit), colour from real spherical harmonics of degree
 * sh_degree: plane k*3+c holds basis k (k = l*l + l + m) of channel c, and
 * rgb_c = max(0, sum_k sh[k*3+c] Y_k(normalise(mu - campos)) + 0.5). */
typedef struct {
  int32_t n;          /* live Gaussians, 0 <= n <= capacity                  */
  int32_t capacity;   /* plane stride (floats)                               */
  int32_t n_base;     /* 0 <= n_base <= n                                    */
  int32_t sh_degree;  /* 0..3                                                */
  float* mean;        /* [3][capacity]                                       */
  float* quat;        /* [4][capacity]                                       */
  float* log_scale;   /* [3][capacity]                                       */
  float* opacity_logit; /* [capacity]                                        */
  float* sh;          /* [3*(sh_degree+1)^2][capacity]                       */
} dass_gaussians;

/* Pinhole camera: x_cam = R x_world + t (R row-major), camera frame x right, y down,
 * z forward; pixel (u,v) = (fx x/z + cx, fy y/z + cy), pixel centres at integer
 * coordinates; campos = camera centre in world space (for the view direction of the colour). */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float campos[3];
  int32_t width, height;
} dass_camera;

/* One rendered view: rgb [3][height][width], t_final (final transmittance) [height][width],
 * n_contrib [height][width] = number of entries of the pixel's tile list up to and
 * including the last one blended. */
typedef struct {
  float* rgb;
  float* t_final;
  int32_t* n_contrib;
} dass_image;

/* Gradients with the layout of dass_gaussians (capacity stride).  Any pointer may be NULL
 * to skip that parameter.  Accumulated (+=). */
typedef struct {
  float* mean;
  float* quat;
  float* log_scale;
  float* opacity_logit;
  float* sh;
} dass_grads;

/* Render options.  tile_w, tile_h in {16, 32, 64} pixels (a NULL opts means 16x16): the
 * tile is the key bin of the binning and sort; the blend splits it into 16x16 sub-tiles.  The
 * images are the same for every tile size; n_contrib and the keys depend on it. */
#define DASS_FLAG_COUNT_PAIRS 1u /* render_fwd also counts evaluated / blended (pixel, entry)
                                    pairs (read with dass_debug_pair_counts); slower */
#define DASS_FLAG_SUBTILE8 2u    /* blend each tile as 8x8 sub-tiles, one pixel per lane (four
                                    times the waves: for small images with long lists); same
                                    lists and order as 16x16 sub-tiles, pixel offsets rounded
                                    relative to the smaller sub-tile's origin */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t batch;  /* list entries the blend stages in LDS at a time: 64, 128 or 256 (0 means
                     128); only the speed depends on it */
  uint32_t flags; /* DASS_FLAG_* bits */
} dass_opts;

/* Sizes the context reserves device memory for. */
typedef struct {
  int32_t max_gaussians; /* capacity of the scenes rendered (< 2^28)            */
  int32_t max_views;     /* views per render call (<= DASS_MAX_VIEWS)            */
  int64_t max_keys;      /* tile keys per render call, summed over its views;
                            at most 0xFFFF0000 (keys are indexed with 32 bits)   */
  int64_t max_tiles;     /* tiles per render call, summed over its views (< 2^31) */
} dass_limits;

/* ---- context ---------------------------------------------------------------------------- */

/* Creates a context on HIP device `device` and reserves `limits`.  Returns DASS_E_HIP if no
 * device is available, DASS_E_OOM if the reservation fails. */
dass_status dass_create(dass_ctx* out, int32_t device, const dass_limits* limits);

/* Grows (never shrinks) the reservation.  Synchronises the context's device. */
dass_status dass_reserve(dass_ctx ctx, const dass_limits* limits);

/* Frees everything the context owns.  NULL is allowed. */
void dass_destroy(dass_ctx ctx);

/* Message for the last failing call on this context (valid until the next call). */
const char* dass_last_error(dass_ctx ctx);

/* Waits for `stream` and returns DASS_E_CAPACITY if a render since the previous sync ran out
 * of tile-key space (its outputs are then invalid), DASS_E_HIP on an asynchronous HIP
 * error, DASS_OK otherwise.  Clears the recorded device error. */
dass_status dass_sync(dass_ctx ctx, dass_stream stream);

/* ---- hot path --------------------------------------------------------------------------- */

/* Forward of the tile-based rasterizer (App. A.1) for n_views cameras in one pass:
 * projection of each Gaussian (Sigma = R S S^T R^T; Sigma_2D = J W Sigma W^T J^T + 0.3 I;
 * cull at camera depth <= 0.2; radius ceil(3 sqrt(lambda_max(Sigma_2D)))), tile keys
 * (tile << 32 | float32 depth bits) for every tile of the Gaussian's rectangle, a stable
 * sort by key, per-tile ranges, and the front-to-back blend of each pixel
 * C = sum_i c_i a_i prod_{j<i}(1-a_j) + T_final * bg with a_i = min(0.99, o_i G_i(pixel)),
 * entries with a_i < 1/255 skipped, and the walk stopped before an entry that would take
 * the transmittance below 1e-4.  out[v] receives view v.  The context keeps the sorted
 * tile lists for the matching render_bwd.
 * Errors: DASS_E_INVALID (null pointers, n > capacity, sh_degree > 3, n_views outside
 * [1, min(max_views, DASS_MAX_VIEWS)], width/height <= 0, a tile edge not in {16, 32, 64});
 * DASS_E_CAPACITY (n > max_gaussians, total tiles > max_tiles; key overflow via dass_sync). */
dass_status render_fwd(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams,
                       int32_t n_views, const float bg[3], dass_image* out,
                       const dass_opts* opts, dass_stream stream);

/* Reverse-mode adjoint of the matching render_fwd (same ctx, g, cams, bg; no render on the
 * context in between).  dl_drgb: host array of n_views device pointers, each [3][H][W].
 * Accumulates dL/d(parameter) into `grads`, and for every Gaussian visible in a view adds the
 * L2 norm of dL/d(pixel-space mean) of that view to gradnorm_sum[g] and 1 to grad_count[g]
 * (the historical view-space positional gradient of Sec. 3.4; either may be NULL).  The
 * transmittance of each entry is recovered from T_final walking the list backwards; no
 * per-pixel lists are stored.  Derivatives through an active clamp (alpha = 0.99, colour
 * = 0, Jacobian clamp) are zero.  Float atomics make the sums order-nondeterministic.
 * opts must give the tile size of the matching render_fwd (DASS_E_INVALID otherwise). */
dass_status render_bwd(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams,
                       int32_t n_views, const float bg[3], const dass_image* fwd_out,
                       const float* const* dl_drgb, dass_grads* grads, float* gradnorm_sum,
                       int32_t* grad_count, const dass_opts* opts, dass_stream stream);

#define DASS_FWD 0
#define DASS_ADJOINT 1

/* Dynamics-aware shift (Sec. 3.3): for the dynamic Gaussians dyn_idx[j] (distinct indices
 * in [0, in->n)), mu' = mu + dpos[:,j] and q' = normalise(q) (x) normalise(drot[:,j])
 * (Hamilton product, (w,x,y,z)); every other Gaussian keeps mu and q.
 * DASS_FWD: writes out->mean and out->quat for rows [0, in->n) (out may not alias in; its
 *   other planes are not touched -- point them at in's).  d_out, d_dpos, d_drot unused.
 * DASS_ADJOINT: d_dpos[:,j] += d_out->mean[:,dyn_idx[j]], d_drot[:,j] += the adjoint of the
 *   product and both normalisations applied to d_out->quat[:,dyn_idx[j]].  out unused.
 * dpos [3][n_dyn], drot [4][n_dyn], d_dpos [3][n_dyn], d_drot [4][n_dyn]. */
dass_status shift_apply(dass_ctx ctx, int32_t mode, const int32_t* dyn_idx, int32_t n_dyn,
                        const float* dpos, const float* drot, const dass_gaussians* in,
                        dass_gaussians* out, const dass_grads* d_out, float* d_dpos,
                        float* d_drot, dass_stream stream);

/* One parameter group of adam_step: n contiguous floats (param, grad, m, v). */
typedef struct {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t n;
  float lr;
} dass_adam_group;

/* Adam with bias correction (step is 1-based), all groups in one pass:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps).
 * `groups` is a host array.  Errors: DASS_E_INVALID for n_groups < 1, step < 1, null
 * pointers in a group with n > 0, or negative n. */
dass_status adam_step(dass_ctx ctx, const dass_adam_group* groups, int32_t n_groups, float beta1,
                      float beta2, float eps, int32_t step, dass_stream stream);

/* adam_step with the 1-based step count in device memory: *d_step is incremented by one on the
 * device and the incremented value is used for the bias correction.  For launch sequences
 * captured once and replayed (a HIP graph), where a host-side step would be frozen. */
dass_status adam_step_device_count(dass_ctx ctx, const dass_adam_group* groups, int32_t n_groups,
                                   float beta1, float beta2, float eps, int32_t* d_step,
                                   dass_stream stream);

/* Error-guided densification (Sec. 3.4, Alg. 1, Eq. 4).  For every base Gaussian n in
 * [0, g->n_base): its Alg. 1 pixel in each view (full projection, Round(z) = floor(z+0.5),
 * x from x_norm and W, y from y_norm and H; points behind a camera or off the image are not
 * projected); S_err = Gaussians whose pixel has err > gamma_err in some view; with
 * gbar = gradnorm_sum/grad_count (0 if the count is 0), the set
 * S = {gbar > tau_pos} u (S_err n {gbar > tau_err}) is ranked by its largest error at its
 * pixels (descending), ties by index.  Child j in [0, K) copies parent S[j mod |S|], with
 * K = 0 if S is empty, else min(k_max, capacity - n); the child's mean moves by
 * R diag(s) z with z three standard normals from SplitMix64(seed) draws 4j..4j+3 through
 * Box-Muller, and its log-scale drops by ln 1.6.  Children are written to rows [n, n+K).
 * K is written to the device scalar *n_appended; the caller reads it and advances g->n.
 * err_maps: host array of n_views device pointers [H][W]; gradnorm_sum, grad_count [n_base]. */
dass_status densify_append(dass_ctx ctx, dass_gaussians* g, const float* const* err_maps,
                           const dass_camera* cams, int32_t n_views, const float* gradnorm_sum,
                           const int32_t* grad_count, float gamma_err, float tau_pos,
                           float tau_err, int32_t k_max, uint64_t seed, int32_t* n_appended,
                           dass_stream stream);

/* L1 term of the fidelity loss (Eqs. 2/3 with lambda = 0) and the error map of Sec. 3.4:
 * with V = n_views and each view's render/target [3][H][W],
 * L = (1/V) sum_v mean_{c,p} |render - target|; dl_drgb = sign(render - target)/(3 H W V)
 * (written, not accumulated); err[v] [H][W] = mean over channels of |render - target|;
 * *loss (device float) += L.  Host arrays of n_views device pointers; err may be NULL. */
dass_status dass_l1_loss_grad(dass_ctx ctx, const dass_camera* cams, int32_t n_views,
                              const float* const* render, const float* const* target,
                              float* const* dl_drgb, float* const* err, float* loss,
                              dass_stream stream);

/* render_fwd fused with dass_l1_loss_grad: the same render (out[v].t_final, n_contrib, and
 * out[v].rgb unless it is NULL) with the blend's epilogue forming the L1 term against
 * target[v]: dl_drgb[v] and err[v] (err may be NULL) bit-identical to dass_l1_loss_grad on
 * the rendered image, and *loss (device float, may be NULL) += L summed in a different order
 * (equal up to float rounding).  Saves writing and re-reading the image in a training step.
 * Errors as render_fwd, plus DASS_E_INVALID for a NULL target or dl_drgb array or entry. */
dass_status dass_render_fwd_l1(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams,
                               int32_t n_views, const float bg[3], dass_image* out,
                               const float* const* target, float* const* dl_drgb, float* const* err,
                               float* loss, const dass_opts* opts, dass_stream stream);

/* The fidelity loss of Eq. (3): L = (1/V) sum_v [(1 - lambda) L1_v + lambda D-SSIM_v] with
 * L1_v = mean over channels and pixels of |render - target| and D-SSIM_v = 1 - SSIM_v, SSIM_v
 * the mean over channels and pixels of the single-scale SSIM map (11x11 Gaussian window,
 * sigma 1.5, normalised; window sums with zero padding; C1 = 0.01^2, C2 = 0.03^2 for images in
 * [0, 1]).  Writes dl_drgb[v] = dL/drender (not accumulated) and err[v] [H][W] = mean over
 * channels of |render - target| (Sec. 3.4; err may be NULL); *loss (device float, may be
 * NULL) += L.  lambda in [0, 1]; lambda = 0 is dass_l1_loss_grad (scratch may then be NULL).
 * scratch: host array of n_views device pointers to 9 H W floats each, caller-owned and
 * overwritten.  Host arrays of n_views device pointers otherwise as dass_l1_loss_grad.
 * Errors: DASS_E_INVALID (lambda outside [0, 1], NULL arrays or entries, bad sizes). */
dass_status dass_fidelity_loss_grad(dass_ctx ctx, const dass_camera* cams, int32_t n_views,
                                    const float* const* render, const float* const* target,
                                    float lambda, float* const* dl_drgb, float* const* err,
                                    float* loss, float* const* scratch, dass_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dass_fidelity_loss_grad with the D-SSIM maps kept
 * in the library's own static scratch instead of caller scratch.  Same arguments, results
 * and errors otherwise (bit-identical outputs for the same inputs).  The scratch holds
 * 9 * DASS_NOALLOC_MAX_PIXELS floats (72 MiB) per GPU, reserved when the library's code is
 * loaded on that GPU and held until the process ends; its address is looked up once per GPU
 * when a context is created there.  The views' pixels (sum of width * height) must not exceed
 * DASS_NOALLOC_MAX_PIXELS: DASS_E_INVALID otherwise, before anything is enqueued.  Calls no
 * allocator.  Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * maps: calls that overlap on one GPU (different streams, or threads without ordering) race;
 * calls ordered on one stream do not. */
#define DASS_NOALLOC_MAX_PIXELS (1 << 21)
dass_status dass_fidelity_loss_grad_noalloc(dass_ctx ctx, const dass_camera* cams, int32_t n_views,
                                            const float* const* render, const float* const* target,
                                            float lambda, float* const* dl_drgb, float* const* err,
                                            float* loss, dass_stream stream);

/* ---- hash-encoded deformation fields (Sec. 3.3; sizes in App. B) ------------------------ */

/* A deformation field H_dyn or H_st: the multi-resolution hash encoding of a position followed
 * by an MLP with one ReLU hidden layer, giving the shift offsets of Sec. 3.3.  For a query at
 * mu: p = clamp((mu - aabb_min) / (aabb_max - aabb_min), 0, 1) per axis; at level l, with
 * x = p N_l, the cell c0 = min(floor(x), N_l - 1) and frac = x - c0 (p, x and c0 in float64), the
 * encoding's F features
 * are the trilinear blend of the rows of the 8 corners c0 + d (d in {0,1}^3, weight
 * prod(d ? frac : 1 - frac)); a corner's row is c_x + (N_l+1)(c_y + (N_l+1) c_z) when
 * (N_l+1)^3 <= T, else (c_x xor c_y 2654435761 xor c_z 805459861) mod T (32-bit unsigned).
 * The L levels' features, level-major, form enc (L*F); h = relu(w1 enc + b1);
 * out = w2 h + b2; dpos = out[0:3], drot = (1, 0, 0, 0) + out[3:7] (a zero output layer is the
 * identity shift; shift_apply normalises drot). */
#define DASS_HASH_MAX_LEVELS 16
typedef struct {
  int32_t levels;      /* L in [1, 16]                                              */
  int32_t features;    /* F in {1, 2, 4, 8}, L * F <= 64                             */
  int32_t log2_table;  /* T = 2^log2_table rows per level, log2_table in [4, 24]     */
  int32_t hidden;      /* hidden units: 32 or 64                                     */
  int32_t res[DASS_HASH_MAX_LEVELS]; /* N_l in [1, 2^20] for l < L (others unread)  */
  float aabb_min[3], aabb_max[3];    /* the box mapped onto [0, 1]^3 (max > min)    */
  float* table;        /* [L][T][F] device                                           */
  float* w1;           /* [hidden][L*F] device                                       */
  float* b1;           /* [hidden] device                                            */
  float* w2;           /* [7][hidden] device                                         */
  float* b2;           /* [7] device                                                 */
} dass_hash_field;

/* Gradients with the shapes of a dass_hash_field's arrays (device; NULL skips one).
 * Accumulated (+=). */
typedef struct {
  float* table;
  float* w1;
  float* b1;
  float* w2;
  float* b2;
} dass_hash_field_grads;

/* Queries the field at m Gaussians: query j reads row idx[j] of mean [3][stride] (idx NULL:
 * row j) and writes dpos [3][ld] and drot [4][ld] column j (ld >= m).  A row outside [0, n)
 * gets the identity shift (dpos 0, drot (1, 0, 0, 0)).  The outputs feed shift_apply.
 * Errors: DASS_E_INVALID for a field outside the limits above, NULL pointers, m < 0, n < 0,
 * stride < n, ld < m, or idx NULL with m > n. */
dass_status dass_hash_field_fwd(dass_ctx ctx, const dass_hash_field* field, const float* mean,
                                int64_t stride, int32_t n, const int32_t* idx, int32_t m,
                                float* dpos, float* drot, int64_t ld, dass_stream stream);

/* Reverse-mode adjoint of dass_hash_field_fwd with the same arguments: given d_dpos [3][ld] and
 * d_drot [4][ld] (dL/d of the outputs), accumulates dL/d(table, w1, b1, w2, b2) into `grads`.
 * Queries outside [0, n) add nothing.  The weight gradients are summed per workgroup and then
 * over workgroups in a fixed order; table gradients use float atomics (order-nondeterministic).
 * Errors as dass_hash_field_fwd, plus DASS_E_INVALID for a NULL grads and DASS_E_CAPACITY for
 * m > max_gaussians (the per-query workspace reserved by the context). */
dass_status dass_hash_field_bwd(dass_ctx ctx, const dass_hash_field* field, const float* mean,
                                int64_t stride, int32_t n, const int32_t* idx, int32_t m,
                                const float* d_dpos, const float* d_drot, int64_t ld,
                                const dass_hash_field_grads* grads, dass_stream stream);

/* ---- selective inheritance and pruning of G^var (Sec. 3.2, App. B, Sec. 3.4) ------------- */

/* Selective inheritance: each G^var Gaussian (row n_base + j, j < n - n_base) has a learnable
 * m[j]; the mask M_j = Quant(sigmoid(m_j)) (1 exactly when m_j >= 0) multiplies the rendered
 * opacity and scale, o_r = M o and s_r = M s.  Writes the planes to render with, in the scene's
 * parametrisation and capacity stride: logit_eff [capacity] and log_scale_eff [3][capacity] get
 * rows [0, n) of the scene's opacity logits and log-scales, with -inf (opacity and scale 0) for
 * masked G^var rows.  Render a dass_gaussians whose opacity_logit / log_scale point at them.
 * Errors: DASS_E_INVALID (scene checks as render_fwd, NULL outputs, outputs aliasing the
 * scene's planes, m NULL with G^var non-empty). */
dass_status dass_inherit_apply(dass_ctx ctx, const dass_gaussians* g, const float* m,
                               float* logit_eff, float* log_scale_eff, dass_stream stream);

/* Gradient of the inheritance values with the straight-through estimator (App. B): the forward
 * used M, the backward treats it as sigmoid(m).  Given the render's gradients with respect to
 * the effective planes (d_logit_eff [capacity], d_log_scale_eff [3][capacity], e.g. render_bwd
 * into a dass_grads), accumulates into dm [n - n_base]
 *   dm_j += (dL/dM_j + lambda_inher) sigmoid'(m_j),
 * dL/dM_j = d_logit_eff / (1 - o) + sum_d d_log_scale_eff,d for unmasked rows (o = sigmoid of the
 * scene's logit), 0 for masked ones (they are not drawn); *loss (device float, may be NULL)
 * += lambda_inher sum_j sigmoid(m_j), the mask loss of Eq. (2).
 * Errors: DASS_E_INVALID (NULL arrays with G^var non-empty, lambda_inher negative or not
 * finite). */
dass_status dass_inherit_adjoint(dass_ctx ctx, const dass_gaussians* g, const float* m,
                                 const float* d_logit_eff, const float* d_log_scale_eff,
                                 float lambda_inher, float* dm, float* loss, dass_stream stream);

/* Removes G^var rows in place, keeping the order of the rest: row n_base + j stays when
 * (m == NULL or m[j] >= 0, the inheritance mask) and (min_opacity <= 0 or its opacity
 * sigmoid(logit) >= min_opacity, the low-opacity pruning of Sec. 3.4).  Every parameter plane is
 * moved; rows [0, n_base) are untouched.  The kept count is written to the device int *n_kept;
 * the caller reads it and sets g->n = n_base + *n_kept (rows beyond are left unspecified).
 * Errors: DASS_E_INVALID (scene checks, NULL n_kept, min_opacity >= 1), DASS_E_CAPACITY (more
 * G^var rows than max_gaussians). */
dass_status dass_compact_var(dass_ctx ctx, dass_gaussians* g, const float* m, float min_opacity,
                             int32_t* n_kept, dass_stream stream);

/* ---- identity features and the dynamics mask (Sec. 3.3) ------------------------------------ */

#define DASS_MAX_FEATURES 16 /* identity-feature channels (Gaussian Grouping uses 16) */
#define DASS_MAX_OBJECTS 256

/* Renders per-Gaussian identity features with the lists of the last render_fwd on this context
 * (same g, cams, opts; no render in between): out[v] [channels][H][W] receives
 * F_c(p) = sum_i e_{i,c} alpha_i T_i, with the colour blend's alpha and transmittance (same
 * culling, skip and stop) and no background.  features [channels][g->capacity] (row g = the
 * Gaussian's vector e_g), channels in [1, 16].  This is the render M of Gaussian Grouping's
 * identity encodings that DASS queries for object IDs (Sec. 3.3).
 * Errors: DASS_E_INVALID (as render_bwd, bad channels, NULL arrays). */
dass_status dass_render_features(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams,
                                 int32_t n_views, const float* features, int32_t channels,
                                 float* const* out, const dass_opts* opts, dass_stream stream);

/* Per-Gaussian dynamics mask (Sec. 3.3): a pixel of view v is dynamic when flow[v] (its
 * optical-flow magnitude, [H][W]) exceeds gamma_op; the objects of the dynamic pixels,
 * argmax_k (cls_w[k] . F(p) + cls_b[k]) of the rendered features feat_imgs[v] [channels][H][W]
 * (first index on ties), are the dynamic objects; Gaussian g in [0, n) is dynamic when the same
 * classification of its feature features[:, g] ([channels][stride]) is a dynamic object.
 * Writes the dynamic Gaussians in increasing order to dyn_idx [n] (device) and their count to
 * the device int *n_dyn (the caller reads it); dyn_objects [n_objects] (device, may be NULL)
 * receives 1 for each dynamic object, else 0.  cls_w [n_objects][channels], cls_b [n_objects]
 * (device).  Views' sizes come from cams (their other fields are unused).
 * Errors: DASS_E_INVALID (channels outside [1, 16], n_objects outside [1, 256], NULL arrays,
 * n > stride, NaN gamma_op), DASS_E_CAPACITY (n > max_gaussians). */
dass_status dass_dynamic_mask(dass_ctx ctx, const dass_camera* cams, int32_t n_views,
                              const float* const* feat_imgs, const float* const* flow,
                              float gamma_op, const float* cls_w, const float* cls_b,
                              int32_t n_objects, int32_t channels, const float* features,
                              int64_t stride, int32_t n, int32_t* dyn_idx, int32_t* n_dyn,
                              uint32_t* dyn_objects, dass_stream stream);

/* ---- stage timers --------------------------------------------------------------------- */

/* Stages timed with HIP events on the stream of each call while profiling is on. */
typedef enum {
  DASS_STAGE_PROJECT = 0,     /* per-Gaussian projection, all views                 */
  DASS_STAGE_DEPTH_SORT = 1,  /* per-view depth order                                */
  DASS_STAGE_BINNING = 2,     /* records into depth order, scan, tile-key emission   */
  DASS_STAGE_KEY_SORT = 3,    /* stable sort of tile keys                            */
  DASS_STAGE_RANGES = 4,      /* per-tile ranges                                     */
  DASS_STAGE_BLEND_FWD = 5,   /* front-to-back blend                                 */
  DASS_STAGE_BLEND_BWD = 6,   /* adjoint of the blend                                */
  DASS_STAGE_PROJECT_BWD = 7, /* adjoint of the projection                           */
  DASS_STAGE_SHIFT = 8,       /* shift_apply (either mode)                           */
  DASS_STAGE_ADAM = 9,        /* adam_step                                           */
  DASS_STAGE_L1 = 10,         /* dass_l1_loss_grad, dass_fidelity_loss_grad          */
  DASS_STAGE_DENSIFY = 11,    /* densify_append                                      */
  DASS_STAGE_FIELD = 12,      /* dass_hash_field_fwd / dass_hash_field_bwd             */
  DASS_STAGE_INHERIT = 13,    /* dass_inherit_apply / _adjoint, dass_compact_var       */
  DASS_NUM_STAGES = 14
} dass_stage;

/* Starts recording: up to max_records intervals per stage (allocates the events). */
dass_status dass_profile_begin(dass_ctx ctx, int32_t max_records);

/* Stops recording, waits for the device, and writes per stage the summed duration in
 * milliseconds and the number of intervals (host arrays of DASS_NUM_STAGES; either may be NULL). */
dass_status dass_profile_end(dass_ctx ctx, double* total_ms, int32_t* records);

/* ---- debug exports (synchronise; for parity tests) ------------------------------------- */

/* Pair counts of the last render_fwd run with DASS_FLAG_COUNT_PAIRS: evaluated = (pixel, list
 * entry) pairs whose alpha was computed, blended = pairs composited (host outputs). */
dass_status dass_debug_pair_counts(dass_ctx ctx, uint64_t* evaluated, uint64_t* blended);


/* Sorted tile keys of view `view` of the last render_fwd: copies up to `max` keys
 * ((tile << 32) | float32 depth bits, tile = ty*tiles_x + tx) and values (Gaussian index) into
 * the device buffers, writes the view's ranges [tiles][2] (int64, offsets within the view's
 * key list; (0,0) for an empty tile) into the device buffer `ranges`, and the key count into
 * *count (host).  DASS_E_CAPACITY if the view has more than `max` keys. */
dass_status dass_debug_keys(dass_ctx ctx, int32_t view, uint64_t* keys, uint32_t* vals,
                            int64_t max, int64_t* ranges, int64_t* count);

/* Tile-size autotuner.  For each of the n_candidates options (tile_w, tile_h, batch and flags, e.g.
 * DASS_FLAG_SUBTILE8) runs render_fwd + render_bwd of this workload once to warm up, then
 * `reps` times between two HIP events on `stream`, and writes the mean milliseconds per
 * fwd+bwd into ms[c] (host array; -1 for a candidate whose tiles or keys exceed the
 * context's budgets) and into *best (host) the index of the first candidate, in the given
 * order of preference, whose time is within 1% of the fastest.  out, dl_drgb and grads
 * are as for render_fwd / render_bwd; grads is accumulated into (scratch for the caller).
 * Synchronises the stream (not for graph capture) and leaves no state for render_bwd.
 * DASS_E_CAPACITY if no candidate fits. */
dass_status dass_autotune_tile(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams,
                               int32_t n_views, const float bg[3], dass_image* out,
                               const float* const* dl_drgb, dass_grads* grads,
                               const dass_opts* candidates, int32_t n_candidates, int32_t reps,
                               int32_t* best, float* ms, dass_stream stream);

/* Per-Gaussian projection of g into one camera as render_fwd computes it, [n][16] doubles
 * (device): u, v, A, B, C (conic), opacity, r, g, b, depth, radius, x0, y0, x1, y1 (tile
 * rectangle for the tile size of opts, NULL = 16x16), visible (integers converted to
 * double).  Synchronises the device. */
dass_status dass_debug_projection(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cam,
                                  const dass_opts* opts, double* out);

#ifdef __cplusplus
}
#endif

#endif /* DASS_H */
