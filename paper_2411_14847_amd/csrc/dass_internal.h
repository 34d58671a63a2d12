// Internal declarations shared by the HIP translation units of libdass (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dass.h"

namespace dass {

// Blend thresholds (fp32 values; the kernels compare in fp32).
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr int kBlendBatch = 128;  // default list entries the blend stages in LDS at a time
// Projection constants (fp32 values widened; the projection runs in fp64).
constexpr double kDilation = (double)0.3f;
constexpr double kNearZ = (double)0.2f;
constexpr double kClip = (double)1.3f;

constexpr int kTile = 16;          // edge of the pixel block one wave blends (a sub-tile)
constexpr int kTilePix = kTile * kTile;
// Tile edges a render call may use (multiples of the sub-tile): a tile of tw x th pixels is one
// key bin; the blend gives each of its (tw/16)(th/16) sub-tiles its own wave.
constexpr int kMaxTileEdge = 64;
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, workgroups dealt round-robin

// Device error bits (ctx->d_err)
constexpr uint32_t kErrKeyOverflow = 1u;
constexpr uint32_t kErrListTooLong = 2u;  // a tile list longer than the blend's position bits

// Camera as the kernels see it (one per view, passed by value).
struct CamK {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float campos[3];
  int W, H, TX, TY;
  int tw, th;     // tile size in pixels
  int tile_base;      // first global tile index of this view
  uint32_t key_base;  // view << CamsK::local_bits: the view's part of a tile key
};
// Tile keys are (view << local_bits) | tile within the view, local_bits wide enough for every
// view's tiles: keys are emitted in view order, so a stable sort of the low local_bits alone
// groups each (view, tile) into one run.
struct CamsK {
  CamK c[DASS_MAX_VIEWS];
  int local_bits;
};

struct SceneK {
  const float* mean;
  const float* quat;
  const float* log_scale;
  const float* logit;
  const float* sh;
  int n, stride, deg;
};

// Per-view output pointers for the blend kernels.
struct ViewIO {
  float* rgb;         // may be NULL in the forward with the fused L1 term (image not kept)
  float* t_final;
  int32_t* n_contrib;
  const float* dl;    // upstream gradient (backward only)
  const float* target;  // fused L1 term (forward only): target image, dL/drgb out, error map out
  float* dl_out;
  float* err;           // may be NULL
  float l1_scale;       // 1 / (3 H W n_views)
  int W, H, TX, tile_base;
};
struct ViewsIO {
  ViewIO v[DASS_MAX_VIEWS];
  int tw, th;  // tile size in pixels
  int sub;     // sub-tile edge (16: four pixels per lane, one per 8x8 quadrant; 8: one pixel)
  int sx, sn;  // sub-tiles per tile row, per tile
  int batch;   // list entries the blend stages in LDS at a time (64, 128 or 256)
  uint32_t* err;  // device error bits (the forward reports a tile list too long to blend)
};
constexpr int kLossSlots = 4096;
constexpr int kFeatMaxC = 16;  // identity-feature channels per render
struct FeatIO {
  float* out[DASS_MAX_VIEWS];  // [C][H][W] per view
  const float* feat;           // [C][stride]
  float* feat16;               // [n][kFeatMaxC] Gaussian-major copy (workspace)
  int64_t stride;
  int C;
  int n;                       // Gaussians of the render (record index = view * n + Gaussian)
};  // partial sums of the fused L1 loss (spread to avoid contention)

// The projected record of one (view, Gaussian), as the blend consumes it (48 bytes).
//   r0 = (u_hi, v_hi, u_lo, v_lo)   pixel-space mean as float hi + lo (fp64-accurate)
//   r1 = (A, B, C, opacity)         inverse of the dilated 2D covariance
//   r2 = (r, g, b, depth)
struct Rec {
  float4 r0, r1, r2;
};

// ---- workspace -------------------------------------------------------------------------
// ---- hash-encoded deformation fields (field.hip) ----------------------------------------
constexpr int kFieldMaxLevels = 16;
constexpr int kFieldMaxBlocks = 768;  // workgroups of the field backward (one partial row each)
struct FieldK {
  const float* table;  // [L][2^log2T][F]
  const float* w1;     // [hidden][L*F]
  const float* b1;     // [hidden]
  const float* w2;     // [7][hidden]
  const float* b2;     // [7]
  int res[kFieldMaxLevels];
  uint32_t dense;      // bit l: level l indexed densely ((N_l + 1)^3 <= T), else hashed
  int L, log2T;
  double lo[3], ext[3];  // box minimum and extent (max - min, exact in float64)
};
struct QueryK {
  const float* mean;  // [3][stride]
  int64_t stride;
  int n;              // rows [0, n) are valid queries
  const int32_t* idx; // [m] rows, or NULL for rows [0, m)
  int m;
  int64_t ld;         // column stride of the offsets / their gradients
};
struct FieldGradsK {
  float* table;
  float* w1;
  float* b1;
  float* w2;
  float* b2;
};
constexpr int64_t kFieldPartialFloats = int64_t(1) << 24;  // per-query-part table-gradient slices (64 MB)
struct SliceMap {
  int begin[kFieldMaxLevels];              // first slice of each level
  int64_t level_floats[kFieldMaxLevels];   // floats of the level's table that can be touched
  int n_slices, n_qparts, features;
};
// Per-query rows of the field backward, feature-major over the m queries of the call ([R][m]).
struct FieldRows {
  float* dpre;  // [hidden] dL/d(pre-activation)
  float* act;   // [hidden] activation
  float* enc;   // [L F] encoding
  float* denc;  // [L F] dL/d(encoding)
  float* dout;  // [7] upstream gradient (zeros for rows outside [0, n))
  double* pn;   // [3] normalised position
};
constexpr int kFieldRowFloats = 64 + 64 + 64 + 64 + 8;  // floats per query reserved for the rows above
struct FieldScratch {
  FieldRows rows;
  float* part;   // [kFieldMaxBlocks][field_part_stride] weight-gradient partials
  float* tpart;  // [kFieldPartialFloats] table-gradient slices of the query parts
};
__host__ __device__ constexpr int field_part_stride(int hidden, int lf) { return hidden * lf + 8 * hidden + 7; }
void launch_field_fwd(const FieldK& f, int F, int hidden, const QueryK& q, float* dpos, float* drot,
                      hipStream_t st);
void launch_field_bwd(const FieldK& f, int F, int hidden, const QueryK& q, const float* d_dpos,
                      const float* d_drot, const FieldGradsK& g, const FieldScratch& ws, hipStream_t st);

// ---- selective inheritance and G^var compaction (inherit.hip) --------------------------
constexpr int kMaxPlanes = 64;
struct CompactPlanes {
  float* plane[kMaxPlanes];  // every parameter plane of the scene (row r at plane[p][r])
  int count;
};
void launch_inherit_apply(const SceneK& s, int nb, const float* m, float* lg_out, float* ls_out, hipStream_t st);
void launch_inherit_adjoint(const SceneK& s, int nb, const float* m, const float* g_logit, const float* g_ls,
                            float lam, float* dm, float* loss, hipStream_t st);
void launch_compact_var(const CompactPlanes& P, const float* logit, int nb, int nv, const float* m, float min_logit,
                        uint32_t* keep, uint64_t* dest, uint64_t* scan_tmp, float* stage, int64_t sstride,
                        int32_t* n_kept, hipStream_t st);

// ---- dynamics mask from identity features (dynmask.hip) ---------------------------------
constexpr int kMaxObjects = 256;
struct DynMaskArgs {
  const float* feat_img[DASS_MAX_VIEWS];  // [C][H][W]
  const float* flow[DASS_MAX_VIEWS];      // [H][W]
  int64_t hw[DASS_MAX_VIEWS];
  int nv;
  float gamma_op;
  const float* w;  // [K][C]
  const float* b;  // [K]
  int K, C;
  const float* feat;  // [C][stride]
  int64_t stride;
  int n;
};
void launch_dynamic_mask(const DynMaskArgs& a, uint32_t* dyn_obj, uint32_t* keep, uint64_t* dest, uint64_t* scan_tmp,
                         int32_t* dyn_idx, int32_t* n_dyn, hipStream_t st);

struct Workspace {
  int64_t cap_vn = 0;     // max views * max gaussians
  int64_t cap_keys = 0;
  int64_t cap_tiles = 0;
  int sort_blocks = 0;
  // per (view, gaussian), view-major, unsorted
  Rec* rec_u = nullptr;
  uint2* rect_u = nullptr;         // (x0 | y0 << 16, x1 | y1 << 16)
  uint64_t* dkey[2] = {nullptr, nullptr};
  uint32_t* dval[2] = {nullptr, nullptr};
  // per sorted position p (view-major, depth order)
  uint2* rect_s = nullptr;
  uint32_t* tt_s = nullptr;        // tiles touched, sorted order
  uint64_t* off_s = nullptr;       // exclusive prefix of tiles touched, [cap_vn + 1]
  uint32_t* gid_s = nullptr;       // gid of sorted position p
  // tile keys carry the record index v * n + g as their value
  float* g2d = nullptr;            // [cap_vn][9], row v * n + g: blend-backward sums (moments of
                                   // dL/d(exponent) over the offsets, d opacity, d rgb)
  uint8_t* vis = nullptr;          // [cap_vn], row v * n + g: bit 3 visible, bit c colour channel c
                                   // above its clamp at 0 (the colour adjoint's only record reads)
  // keys
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint2* ranges = nullptr;         // [cap_tiles]
  // scratch
  uint32_t* hist = nullptr;        // sort histograms
  uint64_t* scan_tmp = nullptr;    // scan block sums
  uint32_t* counters = nullptr;    // [0] = key count (clamped), [1] = densify |S|, [2] = depth-sort count
  unsigned long long* pairs = nullptr;  // [0] evaluated, [1] blended (pair counting only)
  float* loss_slots = nullptr;          // [kLossSlots] partial sums of the fused L1 loss
  float* field_part = nullptr;          // [kFieldMaxBlocks][field_part_stride] weight-gradient partials
  float* field_rows = nullptr;          // [kFieldRowFloats][cap_g] the field backward's per-query rows
  float* g64 = nullptr;                 // [64][cap_g] the compaction's staging copy and the feature render's
                                        // Gaussian-major rows (inside field_rows)
  uint32_t* keep = nullptr;             // [cap_g] compaction keep flags
  uint64_t* keep_scan = nullptr;        // [cap_g + 1] their exclusive prefix
  uint32_t* dyn_obj = nullptr;          // [kMaxObjects] dynamic-object flags
  double* field_pn = nullptr;           // [3][cap_g] normalised query positions
  float* field_tpart = nullptr;         // [kFieldPartialFloats] table-gradient slices of query parts
  int64_t cap_g = 0;                    // queries per field call (max_gaussians)
  uint32_t* err = nullptr;         // device error bits
};

// ---- kernels launched by the host layer ------------------------------------------------
// project.hip
void launch_preprocess(const SceneK& s, const CamsK& cams, int nv, Workspace& ws, hipStream_t st);
void launch_preprocess_bwd(const SceneK& s, const CamsK& cams, int nv, const Workspace& ws,
                           const dass_grads& grads, float* gradnorm, int32_t* gcount, hipStream_t st);
void launch_debug_projection(const SceneK& s, const CamsK& cams, int view, double* out, hipStream_t st);

// sort.hip
// Exclusive scan of n uint32 values into uint64 out[0..n], out[n] = total.
void scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t st);
size_t scan_tmp_elems(int64_t n);
// LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit); the element count is read
// from device memory (*d_count) and must not exceed max_count.  Keys and values ping-pong
// between buffer 0 and 1; returns the index of the buffer holding the result.
int radix_sort_u64(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* d_count, int64_t max_count,
                   int begin_bit, int end_bit, uint32_t* hist, int blocks, hipStream_t st);
int radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* d_count, int64_t max_count,
                   int begin_bit, int end_bit, uint32_t* hist, int blocks, hipStream_t st,
                   int digit_cap = 11);
int sort_blocks_for(int64_t max_count);

// raster.hip
void launch_gather_sorted(int n, int64_t vn, const uint32_t* sorted_gid, Workspace& ws, hipStream_t st);
// emits keys into ws.keys[0]/ws.vals[0] and writes the clamped key count to ws.counters[0]
void launch_emit_keys(int n, int64_t vn, const CamsK& cams, Workspace& ws, hipStream_t st);
void launch_ranges(const uint32_t* keys, int64_t total_tiles, const CamsK& cams, int nv, Workspace& ws, hipStream_t st);
void launch_blend_fwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3],
                      const Workspace& ws, const uint32_t* vals, bool count_pairs, bool l1, hipStream_t st);
// Adds the loss partial sums and `add` to *loss (fixed order) and clears the sums.
void launch_loss_finish(float* slots, float* loss, float add, hipStream_t st);
// accumulates the per-(view, Gaussian) 2D gradients into ws.g2d[(v * n + g) * 9 + k]
void launch_blend_bwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3],
                      const Workspace& ws, const uint32_t* vals, int n, hipStream_t st);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// identity features of the last render's lists (same weights as its colour blend)
void launch_blend_feat(const ViewsIO& io, int nv, int64_t total_tiles, const FeatIO& fo, const Workspace& ws,
                       const uint32_t* vals, hipStream_t st);
void launch_debug_keys(int view, int n, const Workspace& ws, const uint32_t* keys_sorted, const uint32_t* vals_sorted,
                       uint32_t lo, uint32_t cnt, const CamK& cam, uint64_t* kout, uint32_t* vout, hipStream_t st);

// update.hip
void launch_shift_fwd(const SceneK& in, float* out_mean, float* out_quat, const int32_t* dyn_idx,
                      int n_dyn, const float* dpos, const float* drot, hipStream_t st);
void launch_shift_adj(const SceneK& in, const float* dmean, const float* dquat, const int32_t* dyn_idx,
                      int n_dyn, const float* drot, float* d_dpos, float* d_drot, hipStream_t st);

struct AdamGroupK {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  int64_t block_begin;  // first block index of this group
  float lr;
};
constexpr int kAdamMaxGroups = 24;
struct AdamArgs {
  AdamGroupK g[kAdamMaxGroups];
  int n_groups;
  float b1, b2, eps, bc1, bc2;
  const int32_t* d_step;  // if set, the bias corrections come from this device step count
};
void launch_adam(const AdamArgs& a, int64_t total_blocks, hipStream_t st);
void launch_step_increment(int32_t* d_step, hipStream_t st);

struct L1View {
  const float* render;
  const float* target;
  float* dl;
  float* err;
  int64_t hw;
  int64_t block_begin;
};
struct L1Args {
  L1View v[DASS_MAX_VIEWS];
  int nv;
  float scale;  // 1 / (3 H W V) per view is computed per view; scale = 1/V
};
void launch_l1(const L1Args& a, int64_t total_blocks, float* loss, hipStream_t st);

// D-SSIM term of the fidelity loss (loss.hip): one workgroup per ssim_tile_edge()^2 pixel tile.
struct SsimView {
  const float* render;  // [3][H][W]
  const float* target;  // [3][H][W]
  float* dl;            // [3][H][W] written
  float* err;           // [H][W] or NULL
  float* scratch;       // [3 channels][3 maps][H][W]
  int W, H, TX;         // TX = tiles per row
  int64_t block_begin;
};
struct SsimArgs {
  SsimView v[DASS_MAX_VIEWS];
  float gS[DASS_MAX_VIEWS];        // dL/dSSIM(pixel, channel) = -lambda / (3 H W V)
  float l1_scale[DASS_MAX_VIEWS];  // (1 - lambda) / (3 H W V)
  float w[11];                     // normalised Gaussian window, sigma 1.5
  int nv;
};
int64_t ssim_tiles(int W, int H);
int ssim_tile_edge();
// Forward (SSIM map, its derivatives into scratch, loss partials) then backward (dL/drgb, error
// map, L1 partials); the partials go to loss_slots.
void launch_ssim(const SsimArgs& a, int64_t total_blocks, float* loss_slots, hipStream_t st);

struct DensifyArgs {
  const float* err[DASS_MAX_VIEWS];
  CamK cams[DASS_MAX_VIEWS];
  int nv;
  float gamma_err, tau_pos, tau_err;
};
void launch_densify_select(const SceneK& s, const DensifyArgs& a, const float* gsum, const int32_t* gcnt, int n_base,
                           uint32_t* keep, uint64_t* pos, uint64_t* scan_tmp, uint32_t* score_key, uint32_t* sel_keys,
                           uint32_t* sel_vals, uint32_t* d_count, hipStream_t st);
void launch_densify_spawn(float* mean, float* quat, float* log_scale, float* logit, float* sh, int n_planes_sh,
                          int stride, int n, int capacity, const uint32_t* sel_idx, const uint32_t* d_count,
                          int k_max, uint64_t seed, int32_t* n_appended, hipStream_t st);

// error checking helper
inline const char* hip_err_str(hipError_t e) { return hipGetErrorString(e); }

}  // namespace dass
