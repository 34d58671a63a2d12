// Host layer of libdass: context and workspace, argument checks, and the launch sequences of
// the exported entry points.  No entry point on the hot path allocates or synchronises.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dass_internal.h"

namespace dass {
int adam_per_block();
int l1_per_block();
}  // namespace dass

using namespace dass;

struct Profiler {
  bool on = false;
  int max = 0;
  std::vector<hipEvent_t> ev[DASS_NUM_STAGES];  // 2 per record (start, end)
  int used[DASS_NUM_STAGES] = {};
};

struct dass_ctx_s {
  int device = 0;
  float* static_scratch = nullptr;  // this device's copy of the allocation-free call's scratch
  Profiler prof;
  dass_limits lim{};
  Workspace ws;
  std::vector<void*> allocs;
  std::string last_error;
  // state kept by render_fwd for the matching render_bwd
  bool have_fwd = false;
  int fwd_n = 0, fwd_nv = 0, fwd_stride = 0;
  int64_t fwd_tiles = 0;
  int fwd_tw = kTile, fwd_th = kTile, fwd_sub = kTile;
  int fwd_key_buf = 0;
  CamsK fwd_cams{};
  float fwd_bg[3] = {0.f, 0.f, 0.f};
};

namespace {

dass_status fail(dass_ctx ctx, dass_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail(ctx, DASS_E_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Records the start / end of a stage interval on `st` while profiling is on.
void stage_begin(dass_ctx ctx, int stage, hipStream_t st) {
  Profiler& p = ctx->prof;
  if (!p.on || p.used[stage] >= p.max) return;
  (void)hipEventRecord(p.ev[stage][2 * p.used[stage]], st);
}
void stage_end(dass_ctx ctx, int stage, hipStream_t st) {
  Profiler& p = ctx->prof;
  if (!p.on || p.used[stage] >= p.max) return;
  (void)hipEventRecord(p.ev[stage][2 * p.used[stage] + 1], st);
  p.used[stage]++;
}

void profile_free(dass_ctx ctx) {
  Profiler& p = ctx->prof;
  for (int s = 0; s < DASS_NUM_STAGES; s++) {
    for (hipEvent_t e : p.ev[s]) (void)hipEventDestroy(e);
    p.ev[s].clear();
    p.used[s] = 0;
  }
  p.on = false;
  p.max = 0;
}

dass_status check_launch(dass_ctx ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, DASS_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return DASS_OK;
}

int bit_width(uint64_t x) {
  int b = 0;
  while (x) {
    b++;
    x >>= 1;
  }
  return b;
}

template <typename T>
dass_status dev_alloc(dass_ctx ctx, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 256;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, DASS_E_OOM, "hipMalloc of %zu bytes failed", bytes);
  }
  ctx->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return DASS_OK;
}

void free_all(dass_ctx ctx) {
  for (void* p : ctx->allocs) (void)hipFree(p);
  ctx->allocs.clear();
  ctx->ws = Workspace{};
}

dass_status check_limits(dass_ctx ctx, const dass_limits* l) {
  if (!l) return fail(ctx, DASS_E_INVALID, "limits is NULL");
  if (l->max_gaussians < 0 || l->max_views < 1 || l->max_views > DASS_MAX_VIEWS || l->max_keys < 0 ||
      l->max_tiles < 0)
    return fail(ctx, DASS_E_INVALID, "limits out of range");
  // 32-bit key positions; the margin keeps strided loops over [0, count) from wrapping
  if (l->max_keys > 0xFFFF0000ll || l->max_tiles > 0x7FFFFFFFll)
    return fail(ctx, DASS_E_INVALID, "max_keys must be <= 0xFFFF0000 and max_tiles < 2^31");
  if ((int64_t)l->max_views * l->max_gaussians > 0xFFFFFFFFll)
    return fail(ctx, DASS_E_INVALID, "max_views * max_gaussians must be < 2^32");
  // the blend carries list positions (< max_gaussians) in 28 bits
  if (l->max_gaussians >= (1 << 28)) return fail(ctx, DASS_E_INVALID, "max_gaussians must be < 2^28");
  return DASS_OK;
}

dass_status allocate(dass_ctx ctx, const dass_limits& l) {
  free_all(ctx);
  Workspace& w = ctx->ws;
  w.cap_vn = (int64_t)l.max_views * l.max_gaussians;
  w.cap_keys = l.max_keys;
  w.cap_tiles = l.max_tiles;
  const int64_t vn = w.cap_vn > 0 ? w.cap_vn : 1;
  dass_status s;
#define ALLOC(ptr, cnt) \
  if ((s = dev_alloc(ctx, &(ptr), (size_t)(cnt))) != DASS_OK) return s;
  ALLOC(w.rec_u, vn);
  ALLOC(w.rect_u, vn);
  ALLOC(w.dkey[0], vn);
  ALLOC(w.dkey[1], vn);
  ALLOC(w.dval[0], vn);
  ALLOC(w.dval[1], vn);
  ALLOC(w.rect_s, vn);
  ALLOC(w.tt_s, vn);
  ALLOC(w.off_s, vn + 1);
  ALLOC(w.g2d, vn * 9);
  ALLOC(w.vis, vn);
  ALLOC(w.keys[0], w.cap_keys > 0 ? w.cap_keys : 1);
  ALLOC(w.keys[1], w.cap_keys > 0 ? w.cap_keys : 1);
  ALLOC(w.vals[0], w.cap_keys > 0 ? w.cap_keys : 1);
  ALLOC(w.vals[1], w.cap_keys > 0 ? w.cap_keys : 1);
  ALLOC(w.ranges, w.cap_tiles > 0 ? w.cap_tiles : 1);
  ALLOC(w.hist, 2048 * 1024 + 2048);  // [radix][max sort blocks] counts + radix digit totals
  ALLOC(w.scan_tmp, scan_tmp_elems(vn));
  ALLOC(w.counters, 16);
  ALLOC(w.pairs, 2);
  ALLOC(w.loss_slots, kLossSlots);
  ALLOC(w.field_part, (size_t)kFieldMaxBlocks * field_part_stride(64, 64));
  w.cap_g = l.max_gaussians > 0 ? l.max_gaussians : 1;
  ALLOC(w.field_rows, (size_t)kFieldRowFloats * w.cap_g);
  w.g64 = w.field_rows;
  ALLOC(w.keep, w.cap_g);
  ALLOC(w.keep_scan, w.cap_g + 1);
  ALLOC(w.dyn_obj, kMaxObjects);
  ALLOC(w.field_pn, (size_t)3 * w.cap_g);
  ALLOC(w.field_tpart, (size_t)kFieldPartialFloats);
  ALLOC(w.err, 1);
#undef ALLOC
  w.gid_s = w.dval[0];
  HIP_TRY(ctx, hipMemset(w.counters, 0, 16 * sizeof(uint32_t)));
  HIP_TRY(ctx, hipMemset(w.err, 0, sizeof(uint32_t)));
  HIP_TRY(ctx, hipMemset(w.pairs, 0, 2 * sizeof(unsigned long long)));
  HIP_TRY(ctx, hipMemset(w.loss_slots, 0, kLossSlots * sizeof(float)));  // kept at zero by the loss finish
  HIP_TRY(ctx, hipDeviceSynchronize());
  ctx->lim = l;
  ctx->have_fwd = false;
  return DASS_OK;
}

dass_status check_scene(dass_ctx ctx, const dass_gaussians* g) {
  if (!g) return fail(ctx, DASS_E_INVALID, "gaussians is NULL");
  if (g->n < 0 || g->capacity < 0 || g->n > g->capacity || g->n_base < 0 || g->n_base > g->n)
    return fail(ctx, DASS_E_INVALID, "need 0 <= n_base <= n <= capacity (n=%d, n_base=%d, capacity=%d)", g->n,
                g->n_base, g->capacity);
  if (g->sh_degree < 0 || g->sh_degree > DASS_MAX_SH_DEGREE)
    return fail(ctx, DASS_E_INVALID, "sh_degree %d outside [0,3]", g->sh_degree);
  if (g->n > 0 && (!g->mean || !g->quat || !g->log_scale || !g->opacity_logit || !g->sh))
    return fail(ctx, DASS_E_INVALID, "a parameter plane is NULL");
  return DASS_OK;
}

dass_status make_cams(dass_ctx ctx, const dass_camera* cams, int nv, int tw, int th, CamsK& out,
                      int64_t& total_tiles) {
  if (!cams) return fail(ctx, DASS_E_INVALID, "cams is NULL");
  if (nv < 1 || nv > DASS_MAX_VIEWS || nv > ctx->lim.max_views)
    return fail(ctx, nv > ctx->lim.max_views && nv <= DASS_MAX_VIEWS ? DASS_E_CAPACITY : DASS_E_INVALID,
                "n_views %d outside [1, %d]", nv, std::min(DASS_MAX_VIEWS, ctx->lim.max_views));
  total_tiles = 0;
  std::memset(&out, 0, sizeof(out));
  for (int v = 0; v < nv; v++) {
    const dass_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 65535 * kTile || c.height > 65535 * kTile)
      return fail(ctx, DASS_E_INVALID, "view %d: bad size %dx%d", v, c.width, c.height);
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(ctx, DASS_E_INVALID, "view %d: focal lengths must be > 0", v);
    CamK& k = out.c[v];
    std::memcpy(k.R, c.R, sizeof(k.R));
    std::memcpy(k.t, c.t, sizeof(k.t));
    k.fx = c.fx;
    k.fy = c.fy;
    k.cx = c.cx;
    k.cy = c.cy;
    std::memcpy(k.campos, c.campos, sizeof(k.campos));
    k.W = c.width;
    k.H = c.height;
    k.TX = (c.width + tw - 1) / tw;
    k.TY = (c.height + th - 1) / th;
    k.tw = tw;
    k.th = th;
    k.tile_base = (int)total_tiles;
    total_tiles += (int64_t)k.TX * k.TY;
  }
  if (total_tiles > ctx->ws.cap_tiles)
    return fail(ctx, DASS_E_CAPACITY, "%lld tiles exceed max_tiles %lld", (long long)total_tiles,
                (long long)ctx->ws.cap_tiles);
  int64_t max_view_tiles = 1;
  for (int v = 0; v < nv; v++) max_view_tiles = std::max(max_view_tiles, (int64_t)out.c[v].TX * out.c[v].TY);
  out.local_bits = bit_width((uint64_t)(max_view_tiles - 1));
  if (out.local_bits > 31 || out.local_bits + bit_width((uint64_t)(nv - 1)) > 32)
    return fail(ctx, DASS_E_CAPACITY, "%lld tiles per view do not fit a 32-bit tile key", (long long)max_view_tiles);
  for (int v = 0; v < nv; v++) out.c[v].key_base = (uint32_t)v << out.local_bits;
  return DASS_OK;
}

bool tile_edge_ok(int e) { return e == 16 || e == 32 || e == 64; }

// Validates the options and returns the tile size (16x16 when o is NULL) and sub-tile edge.
dass_status check_opts(dass_ctx ctx, const dass_opts* o, int& tw, int& th, int& sub, int& batch) {
  tw = th = kTile;
  sub = kTile;
  batch = kBlendBatch;
  if (!o) return DASS_OK;
  if (!tile_edge_ok(o->tile_w) || !tile_edge_ok(o->tile_h))
    return fail(ctx, DASS_E_INVALID, "tile %dx%d unsupported (edges 16, 32 or 64)", o->tile_w, o->tile_h);
  if (o->flags & ~(DASS_FLAG_COUNT_PAIRS | DASS_FLAG_SUBTILE8))
    return fail(ctx, DASS_E_INVALID, "unknown option flags");
  if (o->batch != 0 && o->batch != 64 && o->batch != 128 && o->batch != 256)
    return fail(ctx, DASS_E_INVALID, "blend batch %d unsupported (0, 64, 128 or 256)", o->batch);
  tw = o->tile_w;
  th = o->tile_h;
  sub = (o->flags & DASS_FLAG_SUBTILE8) ? 8 : kTile;
  batch = o->batch ? o->batch : kBlendBatch;
  return DASS_OK;
}

void set_tiling(ViewsIO& io, int tw, int th, int sub, int batch) {
  io.tw = tw;
  io.th = th;
  io.sub = sub;
  io.batch = batch;
  io.sx = tw / sub;
  io.sn = (tw / sub) * (th / sub);
}

SceneK scene_of(const dass_gaussians* g) {
  SceneK s;
  s.mean = g->mean;
  s.quat = g->quat;
  s.log_scale = g->log_scale;
  s.logit = g->opacity_logit;
  s.sh = g->sh;
  s.n = g->n;
  s.stride = g->capacity;
  s.deg = g->sh_degree;
  return s;
}

// Scratch of the allocation-free loss call (dass_fidelity_loss_grad_noalloc): the D-SSIM
// derivative maps, 9 floats per pixel of the call's views.  Every device the library runs on
// holds its own copy until the process ends.  In host code the array's name is not a device
// address: kernels and copies get the address looked up per device by static_scratch_of.
constexpr int64_t kStaticScratchFloats = 9ll * DASS_NOALLOC_MAX_PIXELS;
__device__ __align__(256) float scratch[kStaticScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device (the device must be the
// current one).
dass_status static_scratch_of(dass_ctx ctx, int device, float** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices)
    return fail(ctx, DASS_E_UNSUPPORTED, "device %d: the static scratch table holds %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(ctx, DASS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return DASS_OK;
}

}  // namespace

extern "C" {

dass_status dass_create(dass_ctx* out, int32_t device, const dass_limits* limits) {
  if (!out) return DASS_E_INVALID;
  *out = nullptr;
  dass_ctx ctx = new (std::nothrow) dass_ctx_s();
  if (!ctx) return DASS_E_OOM;
  dass_status s = check_limits(ctx, limits);
  if (s != DASS_OK) {
    delete ctx;
    return s;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    delete ctx;
    return DASS_E_HIP;
  }
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return DASS_E_HIP;
  }
  s = allocate(ctx, *limits);
  if (s == DASS_OK) s = static_scratch_of(ctx, device, &ctx->static_scratch);
  if (s != DASS_OK) {
    free_all(ctx);
    delete ctx;
    return s;
  }
  *out = ctx;
  return DASS_OK;
}

dass_status dass_reserve(dass_ctx ctx, const dass_limits* limits) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s = check_limits(ctx, limits);
  if (s != DASS_OK) return s;
  dass_limits l = ctx->lim;
  l.max_gaussians = std::max(l.max_gaussians, limits->max_gaussians);
  l.max_views = std::max(l.max_views, limits->max_views);
  l.max_keys = std::max(l.max_keys, limits->max_keys);
  l.max_tiles = std::max(l.max_tiles, limits->max_tiles);
  if (l.max_gaussians == ctx->lim.max_gaussians && l.max_views == ctx->lim.max_views &&
      l.max_keys == ctx->lim.max_keys && l.max_tiles == ctx->lim.max_tiles)
    return DASS_OK;
  s = check_limits(ctx, &l);
  if (s != DASS_OK) return s;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipDeviceSynchronize());
  return allocate(ctx, l);
}

void dass_destroy(dass_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  profile_free(ctx);
  free_all(ctx);
  delete ctx;
}

const char* dass_last_error(dass_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

dass_status dass_sync(dass_ctx ctx, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // stream-ordered only: a legacy-stream copy here would also wait for (and, while another
  // thread captures a graph, conflict with) every other blocking stream of the device
  hipStream_t st = (hipStream_t)stream;
  uint32_t err = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&err, ctx->ws.err, sizeof(err), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (err) {
    launch_fill_u32(ctx->ws.err, 0u, 1, st);
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (err & kErrKeyOverflow) return fail(ctx, DASS_E_CAPACITY, "tile-key buffer overflow (raise max_keys)");
    if (err & kErrListTooLong)
      return fail(ctx, DASS_E_CAPACITY, "a tile list exceeds 2^27 entries (use smaller tiles)");
  }
  return DASS_OK;
}

// The fused L1 term of render_fwd_l1 (NULL for a plain render_fwd).
struct L1Out {
  const float* const* target;
  float* const* dl_drgb;
  float* const* err;
  float* loss;
};

dass_status render_fwd_impl(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                            const float bg[3], dass_image* out, const L1Out* l1, const dass_opts* opts,
                            dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  int tw, th, sub, batch;
  if ((s = check_opts(ctx, opts, tw, th, sub, batch)) != DASS_OK) return s;
  if (!bg || !out) return fail(ctx, DASS_E_INVALID, "bg or out is NULL");
  CamsK ck;
  int64_t total_tiles = 0;
  if ((s = make_cams(ctx, cams, n_views, tw, th, ck, total_tiles)) != DASS_OK) return s;
  if (g->n > ctx->lim.max_gaussians)
    return fail(ctx, DASS_E_CAPACITY, "n=%d exceeds max_gaussians %d", g->n, ctx->lim.max_gaussians);
  ViewsIO io;
  std::memset(&io, 0, sizeof(io));
  set_tiling(io, tw, th, sub, batch);
  if (l1 && (!l1->target || !l1->dl_drgb)) return fail(ctx, DASS_E_INVALID, "targets or dl_drgb is NULL");
  for (int v = 0; v < n_views; v++) {
    if ((!out[v].rgb && !l1) || !out[v].t_final || !out[v].n_contrib)
      return fail(ctx, DASS_E_INVALID, "out[%d] has a NULL buffer", v);
    io.v[v].rgb = out[v].rgb;
    io.v[v].t_final = out[v].t_final;
    io.v[v].n_contrib = out[v].n_contrib;
    io.v[v].dl = nullptr;
    if (l1) {
      if (!l1->target[v] || !l1->dl_drgb[v]) return fail(ctx, DASS_E_INVALID, "view %d: NULL target or dl_drgb", v);
      io.v[v].target = l1->target[v];
      io.v[v].dl_out = l1->dl_drgb[v];
      io.v[v].err = l1->err ? l1->err[v] : nullptr;
      // as dass_l1_loss_grad: (1/V) / (3 H W)
      io.v[v].l1_scale = (1.0f / (float)n_views) / (3.0f * (float)((int64_t)ck.c[v].W * ck.c[v].H));
    }
    io.v[v].W = ck.c[v].W;
    io.v[v].H = ck.c[v].H;
    io.v[v].TX = ck.c[v].TX;
    io.v[v].tile_base = ck.c[v].tile_base;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  const SceneK sc = scene_of(g);
  const int64_t vn = (int64_t)n_views * g->n;
  const bool count_pairs = opts && (opts->flags & DASS_FLAG_COUNT_PAIRS);
  // 1. projection
  stage_begin(ctx, DASS_STAGE_PROJECT, st);
  launch_preprocess(sc, ck, n_views, ws, st);
  stage_end(ctx, DASS_STAGE_PROJECT, st);
  // 2. per-view depth order: sort (view << 31 | depth bits, index)
  stage_begin(ctx, DASS_STAGE_DEPTH_SORT, st);
  launch_fill_u32(ws.counters + 2, (uint32_t)vn, 1, st);
  const int dcur = radix_sort_u64(ws.dkey, ws.dval, ws.counters + 2, vn, 0, 31 + bit_width((uint64_t)(n_views - 1)),
                                  ws.hist, sort_blocks_for(vn), st);
  ws.gid_s = ws.dval[dcur];
  stage_end(ctx, DASS_STAGE_DEPTH_SORT, st);
  // 3. records into depth order; tile keys in that order; stable sort on the tile id
  stage_begin(ctx, DASS_STAGE_BINNING, st);
  launch_gather_sorted(g->n, vn, ws.gid_s, ws, st);
  launch_emit_keys(g->n, vn, ck, ws, st);
  stage_end(ctx, DASS_STAGE_BINNING, st);
  stage_begin(ctx, DASS_STAGE_KEY_SORT, st);
  // keys arrive in view order, so the tile within the view is the only part left to sort.  An
  // 11-bit digit costs the scatter twice a 10-bit one's per-batch digit work: over the keys of a
  // multi-view call two narrower passes are faster, over one view's keys the single pass is
  const int kcur = radix_sort_u32(ws.keys, ws.vals, ws.counters, ws.cap_keys, 0, ck.local_bits, ws.hist,
                                  sort_blocks_for(ws.cap_keys), st, n_views > 1 ? 10 : 11);
  stage_end(ctx, DASS_STAGE_KEY_SORT, st);
  stage_begin(ctx, DASS_STAGE_RANGES, st);
  launch_ranges(ws.keys[kcur], total_tiles, ck, n_views, ws, st);
  stage_end(ctx, DASS_STAGE_RANGES, st);
  // 4. blend
  if (count_pairs) launch_fill_u32(reinterpret_cast<uint32_t*>(ws.pairs), 0u, 4, st);
  stage_begin(ctx, DASS_STAGE_BLEND_FWD, st);
  launch_blend_fwd(io, n_views, total_tiles, bg, ws, ws.vals[kcur], count_pairs, l1 != nullptr, st);
  stage_end(ctx, DASS_STAGE_BLEND_FWD, st);
  if (l1) {
    stage_begin(ctx, DASS_STAGE_L1, st);
    launch_loss_finish(ws.loss_slots, l1->loss, 0.f, st);
    stage_end(ctx, DASS_STAGE_L1, st);
  }
  if ((s = check_launch(ctx, "render_fwd")) != DASS_OK) return s;
  ctx->have_fwd = true;
  ctx->fwd_n = g->n;
  ctx->fwd_nv = n_views;
  ctx->fwd_stride = g->capacity;
  ctx->fwd_tiles = total_tiles;
  ctx->fwd_tw = tw;
  ctx->fwd_th = th;
  ctx->fwd_sub = sub;
  ctx->fwd_key_buf = kcur;
  ctx->fwd_cams = ck;
  for (int c = 0; c < 3; c++) ctx->fwd_bg[c] = bg[c];
  return DASS_OK;
}

dass_status render_fwd(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                       const float bg[3], dass_image* out, const dass_opts* opts, dass_stream stream) {
  return render_fwd_impl(ctx, g, cams, n_views, bg, out, nullptr, opts, stream);
}

dass_status dass_render_fwd_l1(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                               const float bg[3], dass_image* out, const float* const* target,
                               float* const* dl_drgb, float* const* err, float* loss, const dass_opts* opts,
                               dass_stream stream) {
  const L1Out l1{target, dl_drgb, err, loss};
  return render_fwd_impl(ctx, g, cams, n_views, bg, out, &l1, opts, stream);
}

// True if a call over (g, cameras, tiling) reads the lists and records of the last render_fwd on
// this context: same scene size and stride, the same cameras (every field of the kernels' camera
// records, so poses, intrinsics and image sizes) and the same tile size.  The sub-tile size is
// free: the walk's results do not depend on it.
static bool matches_fwd(const dass_ctx ctx, const dass_gaussians* g, int n_views, int64_t total_tiles, int tw, int th,
                        const CamsK& ck) {
  if (!ctx->have_fwd || ctx->fwd_n != g->n || ctx->fwd_nv != n_views || ctx->fwd_tiles != total_tiles ||
      ctx->fwd_stride != g->capacity || ctx->fwd_tw != tw || ctx->fwd_th != th)
    return false;
  static_assert(sizeof(CamK) == 27 * 4, "CamK holds 4-byte fields only (no padding), compared bytewise");
  return std::memcmp(ctx->fwd_cams.c, ck.c, sizeof(CamK) * (size_t)n_views) == 0;
}

dass_status render_bwd(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                       const float bg[3], const dass_image* fwd_out, const float* const* dl_drgb, dass_grads* grads,
                       float* gradnorm_sum, int32_t* grad_count, const dass_opts* opts, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  int tw, th, sub, batch;
  if ((s = check_opts(ctx, opts, tw, th, sub, batch)) != DASS_OK) return s;
  if (!bg || !fwd_out || !dl_drgb || !grads) return fail(ctx, DASS_E_INVALID, "NULL argument");
  CamsK ck;
  int64_t total_tiles = 0;
  if ((s = make_cams(ctx, cams, n_views, tw, th, ck, total_tiles)) != DASS_OK) return s;
  if (!matches_fwd(ctx, g, n_views, total_tiles, tw, th, ck))
    return fail(ctx, DASS_E_INVALID, "render_bwd does not match the last render_fwd on this context "
                                     "(scene size, cameras or tile size)");
  // alpha is recomputed from pixel offsets relative to the sub-tile's origin, rounded as the
  // forward's (whose blend decisions n_contrib records) only at the same sub-tile size
  if (sub != ctx->fwd_sub)
    return fail(ctx, DASS_E_INVALID, "render_bwd: sub-tile size %d differs from the last render_fwd's %d", sub,
                ctx->fwd_sub);
  for (int c = 0; c < 3; c++)
    if (bg[c] != ctx->fwd_bg[c])
      return fail(ctx, DASS_E_INVALID, "render_bwd: background differs from the last render_fwd's");
  ViewsIO io;
  std::memset(&io, 0, sizeof(io));
  set_tiling(io, tw, th, sub, batch);
  for (int v = 0; v < n_views; v++) {
    if (!fwd_out[v].t_final || !fwd_out[v].n_contrib || !dl_drgb[v])
      return fail(ctx, DASS_E_INVALID, "view %d: NULL t_final, n_contrib or dl_drgb", v);
    io.v[v].rgb = nullptr;
    io.v[v].t_final = fwd_out[v].t_final;
    io.v[v].n_contrib = fwd_out[v].n_contrib;
    io.v[v].dl = dl_drgb[v];
    io.v[v].W = ck.c[v].W;
    io.v[v].H = ck.c[v].H;
    io.v[v].TX = ck.c[v].TX;
    io.v[v].tile_base = ck.c[v].tile_base;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  const int64_t vn = (int64_t)n_views * g->n;
  launch_fill_u32(reinterpret_cast<uint32_t*>(ws.g2d), 0u, vn * 9, st);
  stage_begin(ctx, DASS_STAGE_BLEND_BWD, st);
  launch_blend_bwd(io, n_views, total_tiles, bg, ws, ws.vals[ctx->fwd_key_buf], g->n, st);
  stage_end(ctx, DASS_STAGE_BLEND_BWD, st);
  stage_begin(ctx, DASS_STAGE_PROJECT_BWD, st);
  launch_preprocess_bwd(scene_of(g), ck, n_views, ws, *grads, gradnorm_sum, grad_count, st);
  stage_end(ctx, DASS_STAGE_PROJECT_BWD, st);
  return check_launch(ctx, "render_bwd");
}

dass_status shift_apply(dass_ctx ctx, int32_t mode, const int32_t* dyn_idx, int32_t n_dyn, const float* dpos,
                        const float* drot, const dass_gaussians* in, dass_gaussians* out, const dass_grads* d_out,
                        float* d_dpos, float* d_drot, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, in)) != DASS_OK) return s;
  if (n_dyn < 0 || n_dyn > in->n) return fail(ctx, DASS_E_INVALID, "n_dyn %d outside [0, n]", n_dyn);
  if (n_dyn > 0 && (!dyn_idx || !drot)) return fail(ctx, DASS_E_INVALID, "dyn_idx or drot is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const SceneK sc = scene_of(in);
  if (mode == DASS_FWD) {
    if (!out || !out->mean || !out->quat) return fail(ctx, DASS_E_INVALID, "out->mean/quat is NULL");
    if (out->capacity != in->capacity) return fail(ctx, DASS_E_INVALID, "out and in capacities differ");
    if (out->mean == in->mean || out->quat == in->quat) return fail(ctx, DASS_E_INVALID, "out may not alias in");
    if (n_dyn > 0 && !dpos) return fail(ctx, DASS_E_INVALID, "dpos is NULL");
    stage_begin(ctx, DASS_STAGE_SHIFT, st);
    launch_shift_fwd(sc, out->mean, out->quat, dyn_idx, n_dyn, dpos, drot, st);
    stage_end(ctx, DASS_STAGE_SHIFT, st);
  } else if (mode == DASS_ADJOINT) {
    if (!d_out) return fail(ctx, DASS_E_INVALID, "d_out is NULL");
    if (n_dyn > 0 && ((d_out->mean && !d_dpos) || (d_out->quat && !d_drot)))
      return fail(ctx, DASS_E_INVALID, "d_dpos or d_drot is NULL");
    stage_begin(ctx, DASS_STAGE_SHIFT, st);
    launch_shift_adj(sc, d_out->mean, d_out->quat, dyn_idx, n_dyn, drot, d_dpos, d_drot, st);
    stage_end(ctx, DASS_STAGE_SHIFT, st);
  } else {
    return fail(ctx, DASS_E_INVALID, "mode must be DASS_FWD or DASS_ADJOINT");
  }
  return check_launch(ctx, "shift_apply");
}

static dass_status field_args(dass_ctx ctx, const dass_hash_field* f, const float* mean, int64_t stride, int32_t n,
                              const int32_t* idx, int32_t m, int64_t ld, FieldK& fk, QueryK& qk) {
  if (!f) return fail(ctx, DASS_E_INVALID, "field is NULL");
  const int L = f->levels, F = f->features;
  if (L < 1 || L > DASS_HASH_MAX_LEVELS) return fail(ctx, DASS_E_INVALID, "levels %d outside [1, 16]", L);
  if (F != 1 && F != 2 && F != 4 && F != 8) return fail(ctx, DASS_E_INVALID, "features %d not 1, 2, 4 or 8", F);
  if (L * F > 64) return fail(ctx, DASS_E_INVALID, "levels * features = %d > 64", L * F);
  if (f->log2_table < 4 || f->log2_table > 24)
    return fail(ctx, DASS_E_INVALID, "log2_table %d outside [4, 24]", f->log2_table);
  if (f->hidden != 32 && f->hidden != 64) return fail(ctx, DASS_E_INVALID, "hidden %d not 32 or 64", f->hidden);
  if (!f->table || !f->w1 || !f->b1 || !f->w2 || !f->b2) return fail(ctx, DASS_E_INVALID, "a field array is NULL");
  fk = FieldK{};
  fk.table = f->table;
  fk.w1 = f->w1;
  fk.b1 = f->b1;
  fk.w2 = f->w2;
  fk.b2 = f->b2;
  fk.L = L;
  fk.log2T = f->log2_table;
  const int64_t T = int64_t(1) << f->log2_table;
  for (int l = 0; l < L; l++) {
    const int64_t N = f->res[l];
    if (N < 1 || N > (1 << 20)) return fail(ctx, DASS_E_INVALID, "res[%d] = %lld outside [1, 2^20]", l, (long long)N);
    fk.res[l] = (int)N;
    if ((N + 1) * (N + 1) * (N + 1) <= T) fk.dense |= 1u << l;
  }
  for (int d = 0; d < 3; d++) {
    const float lo = f->aabb_min[d], hi = f->aabb_max[d];
    if (!(std::isfinite(lo) && std::isfinite(hi) && hi > lo))
      return fail(ctx, DASS_E_INVALID, "aabb axis %d: need finite min < max", d);
    fk.lo[d] = lo;
    fk.ext[d] = (double)hi - (double)lo;
  }
  if (m < 0 || n < 0) return fail(ctx, DASS_E_INVALID, "m %d or n %d negative", m, n);
  if (stride < n) return fail(ctx, DASS_E_INVALID, "stride < n");
  if (ld < m) return fail(ctx, DASS_E_INVALID, "ld < m");
  if (!idx && m > n) return fail(ctx, DASS_E_INVALID, "idx NULL needs m <= n");
  if (m > 0 && !mean) return fail(ctx, DASS_E_INVALID, "mean is NULL");
  qk = QueryK{mean, stride, n, idx, m, ld};
  return DASS_OK;
}

dass_status dass_hash_field_fwd(dass_ctx ctx, const dass_hash_field* field, const float* mean, int64_t stride,
                                int32_t n, const int32_t* idx, int32_t m, float* dpos, float* drot, int64_t ld,
                                dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  FieldK fk;
  QueryK qk;
  dass_status s;
  if ((s = field_args(ctx, field, mean, stride, n, idx, m, ld, fk, qk)) != DASS_OK) return s;
  if (m > 0 && (!dpos || !drot)) return fail(ctx, DASS_E_INVALID, "dpos or drot is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  stage_begin(ctx, DASS_STAGE_FIELD, st);
  launch_field_fwd(fk, field->features, field->hidden, qk, dpos, drot, st);
  stage_end(ctx, DASS_STAGE_FIELD, st);
  return check_launch(ctx, "dass_hash_field_fwd");
}

dass_status dass_hash_field_bwd(dass_ctx ctx, const dass_hash_field* field, const float* mean, int64_t stride,
                                int32_t n, const int32_t* idx, int32_t m, const float* d_dpos, const float* d_drot,
                                int64_t ld, const dass_hash_field_grads* grads, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  FieldK fk;
  QueryK qk;
  dass_status s;
  if ((s = field_args(ctx, field, mean, stride, n, idx, m, ld, fk, qk)) != DASS_OK) return s;
  if (!grads) return fail(ctx, DASS_E_INVALID, "grads is NULL");
  if (m > ctx->ws.cap_g)
    return fail(ctx, DASS_E_CAPACITY, "m %d > max_gaussians %lld (the backward's per-query workspace)", m,
                (long long)ctx->ws.cap_g);
  if (m > 0 && (!d_dpos || !d_drot)) return fail(ctx, DASS_E_INVALID, "d_dpos or d_drot is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const FieldGradsK gk{grads->table, grads->w1, grads->b1, grads->w2, grads->b2};
  stage_begin(ctx, DASS_STAGE_FIELD, st);
  const int64_t mm = m;
  FieldScratch fs{};
  float* r = ctx->ws.field_rows;
  fs.rows.dpre = r;
  fs.rows.act = r + 64 * mm;
  fs.rows.enc = r + 128 * mm;
  fs.rows.denc = r + 192 * mm;
  fs.rows.dout = r + 256 * mm;
  fs.rows.pn = ctx->ws.field_pn;
  fs.part = ctx->ws.field_part;
  fs.tpart = ctx->ws.field_tpart;
  launch_field_bwd(fk, field->features, field->hidden, qk, d_dpos, d_drot, gk, fs, st);
  stage_end(ctx, DASS_STAGE_FIELD, st);
  return check_launch(ctx, "dass_hash_field_bwd");
}

dass_status dass_inherit_apply(dass_ctx ctx, const dass_gaussians* g, const float* m, float* logit_eff,
                               float* log_scale_eff, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  if (g->n > 0 && (!logit_eff || !log_scale_eff)) return fail(ctx, DASS_E_INVALID, "an output plane is NULL");
  if (g->n > g->n_base && !m) return fail(ctx, DASS_E_INVALID, "m is NULL");
  if (logit_eff == g->opacity_logit || log_scale_eff == g->log_scale)
    return fail(ctx, DASS_E_INVALID, "outputs may not alias the scene's planes");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  stage_begin(ctx, DASS_STAGE_INHERIT, st);
  launch_inherit_apply(scene_of(g), g->n_base, m, logit_eff, log_scale_eff, st);
  stage_end(ctx, DASS_STAGE_INHERIT, st);
  return check_launch(ctx, "dass_inherit_apply");
}

dass_status dass_inherit_adjoint(dass_ctx ctx, const dass_gaussians* g, const float* m, const float* d_logit_eff,
                                 const float* d_log_scale_eff, float lambda_inher, float* dm, float* loss,
                                 dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  if (!std::isfinite(lambda_inher) || lambda_inher < 0.f)
    return fail(ctx, DASS_E_INVALID, "lambda_inher must be finite and >= 0");
  if (g->n > g->n_base && (!m || !d_logit_eff || !d_log_scale_eff || !dm))
    return fail(ctx, DASS_E_INVALID, "m, the effective-plane gradients or dm is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  stage_begin(ctx, DASS_STAGE_INHERIT, st);
  launch_inherit_adjoint(scene_of(g), g->n_base, m, d_logit_eff, d_log_scale_eff, lambda_inher, dm, loss, st);
  stage_end(ctx, DASS_STAGE_INHERIT, st);
  return check_launch(ctx, "dass_inherit_adjoint");
}

dass_status dass_compact_var(dass_ctx ctx, dass_gaussians* g, const float* m, float min_opacity, int32_t* n_kept,
                             dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  if (!n_kept) return fail(ctx, DASS_E_INVALID, "n_kept is NULL");
  if (!(min_opacity < 1.f) || std::isnan(min_opacity)) return fail(ctx, DASS_E_INVALID, "min_opacity must be < 1");
  const int nb = g->n_base, nv = g->n - g->n_base;
  if (nv > ctx->ws.cap_g) return fail(ctx, DASS_E_CAPACITY, "G^var rows %d > max_gaussians", nv);
  // keep when logit >= log(min_opacity / (1 - min_opacity)), decided exactly for float logits:
  // the smallest float not below the float64 threshold
  float min_logit = -INFINITY;
  if (min_opacity > 0.f) {
    const double thr = std::log((double)min_opacity / (1.0 - (double)min_opacity));
    min_logit = (float)thr;
    if ((double)min_logit < thr) min_logit = std::nextafter(min_logit, INFINITY);
  }
  CompactPlanes P{};
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  auto add = [&](float* base, int planes) {
    for (int p = 0; p < planes; p++) P.plane[P.count++] = base + (int64_t)p * g->capacity;
  };
  add(g->mean, 3);
  add(g->quat, 4);
  add(g->log_scale, 3);
  add(g->opacity_logit, 1);
  add(g->sh, 3 * K);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  stage_begin(ctx, DASS_STAGE_INHERIT, st);
  launch_compact_var(P, g->opacity_logit, nb, nv, m, min_logit, ws.keep, ws.keep_scan, ws.scan_tmp, ws.g64,
                     ws.cap_g, n_kept, st);
  stage_end(ctx, DASS_STAGE_INHERIT, st);
  return check_launch(ctx, "dass_compact_var");
}

dass_status dass_render_features(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                                 const float* features, int32_t channels, float* const* out, const dass_opts* opts,
                                 dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  int tw, th, sub, batch;
  if ((s = check_opts(ctx, opts, tw, th, sub, batch)) != DASS_OK) return s;
  if (channels < 1 || channels > kFeatMaxC) return fail(ctx, DASS_E_INVALID, "channels %d outside [1, 16]", channels);
  if (!out || (g->n > 0 && !features)) return fail(ctx, DASS_E_INVALID, "NULL features or out");
  CamsK ck;
  int64_t total_tiles = 0;
  if ((s = make_cams(ctx, cams, n_views, tw, th, ck, total_tiles)) != DASS_OK) return s;
  if (!matches_fwd(ctx, g, n_views, total_tiles, tw, th, ck))
    return fail(ctx, DASS_E_INVALID, "dass_render_features does not match the last render_fwd on this context "
                                     "(scene size, cameras or tile size)");
  ViewsIO io;
  std::memset(&io, 0, sizeof(io));
  set_tiling(io, tw, th, sub, batch);
  FeatIO fo{};
  for (int v = 0; v < n_views; v++) {
    if (!out[v]) return fail(ctx, DASS_E_INVALID, "view %d: NULL output", v);
    fo.out[v] = out[v];
    io.v[v].W = ck.c[v].W;
    io.v[v].H = ck.c[v].H;
    io.v[v].TX = ck.c[v].TX;
    io.v[v].tile_base = ck.c[v].tile_base;
  }
  fo.feat = features;
  fo.feat16 = ctx->ws.g64;  // [64][cap_g] floats hold [cap_g][16]
  fo.stride = g->capacity;
  fo.C = channels;
  fo.n = g->n;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  stage_begin(ctx, DASS_STAGE_BLEND_FWD, st);
  launch_blend_feat(io, n_views, total_tiles, fo, ctx->ws, ctx->ws.vals[ctx->fwd_key_buf], st);
  stage_end(ctx, DASS_STAGE_BLEND_FWD, st);
  return check_launch(ctx, "dass_render_features");
}

dass_status dass_dynamic_mask(dass_ctx ctx, const dass_camera* cams, int32_t n_views, const float* const* feat_imgs,
                              const float* const* flow, float gamma_op, const float* cls_w, const float* cls_b,
                              int32_t n_objects, int32_t channels, const float* features, int64_t stride, int32_t n,
                              int32_t* dyn_idx, int32_t* n_dyn, uint32_t* dyn_objects, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!cams || n_views < 0 || n_views > DASS_MAX_VIEWS)
    return fail(ctx, DASS_E_INVALID, "cams NULL or n_views outside [0, %d]", DASS_MAX_VIEWS);
  if (channels < 1 || channels > kFeatMaxC) return fail(ctx, DASS_E_INVALID, "channels %d outside [1, 16]", channels);
  if (n_objects < 1 || n_objects > kMaxObjects)
    return fail(ctx, DASS_E_INVALID, "n_objects %d outside [1, %d]", n_objects, kMaxObjects);
  if (!cls_w || !cls_b || !n_dyn || (n > 0 && (!features || !dyn_idx)))
    return fail(ctx, DASS_E_INVALID, "NULL classifier, features, dyn_idx or n_dyn");
  if (n < 0 || stride < n) return fail(ctx, DASS_E_INVALID, "need 0 <= n <= stride");
  if (n > ctx->ws.cap_g) return fail(ctx, DASS_E_CAPACITY, "n %d > max_gaussians", n);
  if (std::isnan(gamma_op)) return fail(ctx, DASS_E_INVALID, "gamma_op is NaN");
  DynMaskArgs a{};
  for (int v = 0; v < n_views; v++) {
    if (cams[v].width <= 0 || cams[v].height <= 0) return fail(ctx, DASS_E_INVALID, "view %d: bad size", v);
    if (!feat_imgs || !flow || !feat_imgs[v] || !flow[v])
      return fail(ctx, DASS_E_INVALID, "view %d: NULL feature image or flow", v);
    a.feat_img[v] = feat_imgs[v];
    a.flow[v] = flow[v];
    a.hw[v] = (int64_t)cams[v].width * cams[v].height;
  }
  a.nv = n_views;
  a.gamma_op = gamma_op;
  a.w = cls_w;
  a.b = cls_b;
  a.K = n_objects;
  a.C = channels;
  a.feat = features;
  a.stride = stride;
  a.n = n;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  launch_dynamic_mask(a, dyn_objects ? dyn_objects : ws.dyn_obj, ws.keep, ws.keep_scan, ws.scan_tmp, dyn_idx, n_dyn,
                      st);
  return check_launch(ctx, "dass_dynamic_mask");
}

static dass_status adam_impl(dass_ctx ctx, const dass_adam_group* groups, int32_t n_groups, float beta1, float beta2,
                             float eps, int32_t step, int32_t* d_step, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!groups || n_groups < 1 || (!d_step && step < 1))
    return fail(ctx, DASS_E_INVALID, "need groups, n_groups >= 1, step >= 1");
  for (int i = 0; i < n_groups; i++) {
    const dass_adam_group& G = groups[i];
    if (G.n < 0) return fail(ctx, DASS_E_INVALID, "group %d: n < 0", i);
    if (G.n > 0 && (!G.param || !G.grad || !G.m || !G.v)) return fail(ctx, DASS_E_INVALID, "group %d: NULL", i);
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int per = adam_per_block();
  const float bc1 = d_step ? 1.f : (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = d_step ? 1.f : (float)(1.0 - std::pow((double)beta2, (double)step));
  stage_begin(ctx, DASS_STAGE_ADAM, st);
  if (d_step) launch_step_increment(d_step, st);
  for (int base = 0; base < n_groups; base += kAdamMaxGroups) {
    AdamArgs a;
    std::memset(&a, 0, sizeof(a));
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.bc1 = bc1;
    a.bc2 = bc2;
    a.d_step = d_step;
    int64_t blocks = 0;
    int k = 0;
    for (int i = base; i < n_groups && i < base + kAdamMaxGroups; i++) {
      const dass_adam_group& G = groups[i];
      if (G.n == 0) continue;
      a.g[k].p = G.param;
      a.g[k].g = G.grad;
      a.g[k].m = G.m;
      a.g[k].v = G.v;
      a.g[k].n = G.n;
      a.g[k].lr = G.lr;
      a.g[k].block_begin = blocks;
      blocks += (G.n + per - 1) / per;
      k++;
    }
    a.n_groups = k;
    if (k > 0) launch_adam(a, blocks, st);
  }
  stage_end(ctx, DASS_STAGE_ADAM, st);
  return check_launch(ctx, "adam_step");
}

dass_status adam_step(dass_ctx ctx, const dass_adam_group* groups, int32_t n_groups, float beta1, float beta2,
                      float eps, int32_t step, dass_stream stream) {
  return adam_impl(ctx, groups, n_groups, beta1, beta2, eps, step, nullptr, stream);
}

dass_status adam_step_device_count(dass_ctx ctx, const dass_adam_group* groups, int32_t n_groups, float beta1,
                                   float beta2, float eps, int32_t* d_step, dass_stream stream) {
  if (!d_step) return fail(ctx, DASS_E_INVALID, "d_step is NULL");
  return adam_impl(ctx, groups, n_groups, beta1, beta2, eps, 0, d_step, stream);
}

dass_status dass_l1_loss_grad(dass_ctx ctx, const dass_camera* cams, int32_t n_views, const float* const* render,
                              const float* const* target, float* const* dl_drgb, float* const* err, float* loss,
                              dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!cams || !render || !target || !dl_drgb || n_views < 1 || n_views > DASS_MAX_VIEWS)
    return fail(ctx, DASS_E_INVALID, "bad arguments");
  L1Args a;
  std::memset(&a, 0, sizeof(a));
  a.nv = n_views;
  a.scale = 1.0f / (float)n_views;
  int64_t blocks = 0;
  const int per = l1_per_block();
  for (int v = 0; v < n_views; v++) {
    if (!render[v] || !target[v] || !dl_drgb[v]) return fail(ctx, DASS_E_INVALID, "view %d: NULL buffer", v);
    if (cams[v].width <= 0 || cams[v].height <= 0) return fail(ctx, DASS_E_INVALID, "view %d: bad size", v);
    a.v[v].render = render[v];
    a.v[v].target = target[v];
    a.v[v].dl = dl_drgb[v];
    a.v[v].err = err ? err[v] : nullptr;
    a.v[v].hw = (int64_t)cams[v].width * cams[v].height;
    a.v[v].block_begin = blocks;
    blocks += (a.v[v].hw + per - 1) / per;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  stage_begin(ctx, DASS_STAGE_L1, (hipStream_t)stream);
  launch_l1(a, blocks, loss, (hipStream_t)stream);
  stage_end(ctx, DASS_STAGE_L1, (hipStream_t)stream);
  return check_launch(ctx, "dass_l1_loss_grad");
}

}  // extern "C"

namespace {

// Arguments of the two D-SSIM passes for n_views views (the window, per-view scales and tiles);
// the views' derivative maps (9 H W floats each) are scratch[v].  Returns an error message or
// NULL.
const char* ssim_args(const dass_camera* cams, int32_t n_views, const float* const* render,
                      const float* const* target, float lambda, float* const* dl_drgb, float* const* err,
                      float* const* scratch, SsimArgs& a, int64_t& blocks) {
  std::memset(&a, 0, sizeof(a));
  a.nv = n_views;
  {
    double g[11], sum = 0.0;
    for (int k = 0; k < 11; k++) sum += (g[k] = std::exp(-((k - 5.0) * (k - 5.0)) / (2.0 * 1.5 * 1.5)));
    for (int k = 0; k < 11; k++) a.w[k] = (float)(g[k] / sum);
  }
  blocks = 0;
  for (int v = 0; v < n_views; v++) {
    if (!render[v] || !target[v] || !dl_drgb[v] || !scratch[v]) return "NULL buffer";
    if (cams[v].width <= 0 || cams[v].height <= 0) return "bad size";
    SsimView& V = a.v[v];
    V.render = render[v];
    V.target = target[v];
    V.dl = dl_drgb[v];
    V.err = err ? err[v] : nullptr;
    V.scratch = scratch[v];
    V.W = cams[v].width;
    V.H = cams[v].height;
    V.TX = (V.W + ssim_tile_edge() - 1) / ssim_tile_edge();
    V.block_begin = blocks;
    blocks += ssim_tiles(V.W, V.H);
    const double n = 3.0 * (double)V.W * (double)V.H * (double)n_views;
    a.gS[v] = (float)(-(double)lambda / n);
    a.l1_scale[v] = (float)((1.0 - (double)lambda) / n);
  }
  return nullptr;
}

}  // namespace

extern "C" {

dass_status dass_fidelity_loss_grad(dass_ctx ctx, const dass_camera* cams, int32_t n_views, const float* const* render,
                                   const float* const* target, float lambda, float* const* dl_drgb,
                                   float* const* err, float* loss, float* const* scratch, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!(lambda >= 0.f && lambda <= 1.f)) return fail(ctx, DASS_E_INVALID, "lambda %g outside [0, 1]", lambda);
  if (lambda == 0.f)  // the L1 term alone
    return dass_l1_loss_grad(ctx, cams, n_views, render, target, dl_drgb, err, loss, stream);
  if (!cams || !render || !target || !dl_drgb || !scratch || n_views < 1 || n_views > DASS_MAX_VIEWS)
    return fail(ctx, DASS_E_INVALID, "bad arguments");
  SsimArgs a;
  int64_t blocks = 0;
  if (const char* why = ssim_args(cams, n_views, render, target, lambda, dl_drgb, err, scratch, a, blocks))
    return fail(ctx, DASS_E_INVALID, "%s", why);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  stage_begin(ctx, DASS_STAGE_L1, st);
  launch_ssim(a, blocks, ctx->ws.loss_slots, st);
  launch_loss_finish(ctx->ws.loss_slots, loss, lambda, st);  // + lambda: the 1 of 1 - SSIM, over views
  stage_end(ctx, DASS_STAGE_L1, st);
  return check_launch(ctx, "dass_fidelity_loss_grad");
}

dass_status dass_fidelity_loss_grad_noalloc(dass_ctx ctx, const dass_camera* cams, int32_t n_views,
                                           const float* const* render, const float* const* target, float lambda,
                                           float* const* dl_drgb, float* const* err, float* loss,
                                           dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!cams || n_views < 1 || n_views > DASS_MAX_VIEWS) return fail(ctx, DASS_E_INVALID, "bad arguments");
  int64_t pixels = 0;
  for (int v = 0; v < n_views; v++) {
    if (cams[v].width <= 0 || cams[v].height <= 0) return fail(ctx, DASS_E_INVALID, "view %d: bad size", v);
    pixels += (int64_t)cams[v].width * cams[v].height;
  }
  if (pixels > DASS_NOALLOC_MAX_PIXELS)
    return fail(ctx, DASS_E_INVALID, "%lld pixels over the views; the allocation-free call takes at most %d",
                (long long)pixels, DASS_NOALLOC_MAX_PIXELS);
  if (!ctx->static_scratch) return fail(ctx, DASS_E_HIP, "no static scratch on device %d", ctx->device);
  // each view's 9 H W maps carved in view order from this device's static scratch
  float* views[DASS_MAX_VIEWS];
  int64_t off = 0;
  for (int v = 0; v < n_views; v++) {
    views[v] = ctx->static_scratch + off;
    off += 9ll * cams[v].width * cams[v].height;
  }
  return dass_fidelity_loss_grad(ctx, cams, n_views, render, target, lambda, dl_drgb, err, loss, views, stream);
}

dass_status densify_append(dass_ctx ctx, dass_gaussians* g, const float* const* err_maps, const dass_camera* cams,
                           int32_t n_views, const float* gradnorm_sum, const int32_t* grad_count, float gamma_err,
                           float tau_pos, float tau_err, int32_t k_max, uint64_t seed, int32_t* n_appended,
                           dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  if (!err_maps || !cams || !n_appended || k_max < 0 || n_views < 1 || n_views > DASS_MAX_VIEWS)
    return fail(ctx, DASS_E_INVALID, "bad arguments");
  if (g->n_base > 0 && (!gradnorm_sum || !grad_count))
    return fail(ctx, DASS_E_INVALID, "gradnorm_sum / grad_count is NULL");
  if (g->n_base > ctx->ws.cap_vn || g->n_base > ctx->ws.cap_g)
    return fail(ctx, DASS_E_CAPACITY, "n_base exceeds the reserved workspace");
  DensifyArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nv = n_views;
  a.gamma_err = gamma_err;
  a.tau_pos = tau_pos;
  a.tau_err = tau_err;
  for (int v = 0; v < n_views; v++) {
    if (!err_maps[v]) return fail(ctx, DASS_E_INVALID, "err_maps[%d] is NULL", v);
    const dass_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0) return fail(ctx, DASS_E_INVALID, "view %d: bad size", v);
    a.err[v] = err_maps[v];
    CamK& k = a.cams[v];
    std::memcpy(k.R, c.R, sizeof(k.R));
    std::memcpy(k.t, c.t, sizeof(k.t));
    k.fx = c.fx;
    k.fy = c.fy;
    k.cx = c.cx;
    k.cy = c.cy;
    k.W = c.width;
    k.H = c.height;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  const SceneK sc = scene_of(g);
  stage_begin(ctx, DASS_STAGE_DENSIFY, st);
  launch_fill_u32(ws.counters + 1, 0u, 1, st);
  // members packed in index order into u32 keys (the depth-sort buffers, free here), the score key
  // staged in the second buffer; a stable 32-bit sort ranks by score, ties by index
  uint32_t* k32[2] = {reinterpret_cast<uint32_t*>(ws.dkey[0]), reinterpret_cast<uint32_t*>(ws.dkey[1])};
  launch_densify_select(sc, a, gradnorm_sum, grad_count, g->n_base, ws.keep, ws.keep_scan, ws.scan_tmp, k32[1], k32[0],
                        ws.dval[0], ws.counters + 1, st);
  const int cur = radix_sort_u32(k32, ws.dval, ws.counters + 1, g->n_base, 0, 32, ws.hist, sort_blocks_for(g->n_base),
                                 st);
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  launch_densify_spawn(g->mean, g->quat, g->log_scale, g->opacity_logit, g->sh, 3 * K, g->capacity, g->n,
                       g->capacity, ws.dval[cur], ws.counters + 1, k_max, seed, n_appended, st);
  stage_end(ctx, DASS_STAGE_DENSIFY, st);
  ctx->have_fwd = false;  // the depth-order buffers were reused
  return check_launch(ctx, "densify_append");
}

dass_status dass_debug_keys(dass_ctx ctx, int32_t view, uint64_t* keys, uint32_t* vals, int64_t max, int64_t* ranges,
                            int64_t* count) {
  if (!ctx || !count || !ranges) return DASS_E_INVALID;
  if (!ctx->have_fwd || view < 0 || view >= ctx->fwd_nv) return fail(ctx, DASS_E_INVALID, "no such view");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipDeviceSynchronize());
  const CamK& c = ctx->fwd_cams.c[view];
  const int nt = c.TX * c.TY;
  std::vector<uint2> r(nt);
  HIP_TRY(ctx, hipMemcpy(r.data(), ctx->ws.ranges + c.tile_base, nt * sizeof(uint2), hipMemcpyDeviceToHost));
  // the view's tiles are runs of the sorted keys (runs of all views interleave); concatenated in
  // tile order they are the view's key list
  std::vector<int64_t> rel(2 * (size_t)nt, 0);
  int64_t cnt = 0;
  for (int t = 0; t < nt; t++)
    if (r[t].y > r[t].x) {
      rel[2 * t] = cnt;
      cnt += r[t].y - r[t].x;
      rel[2 * t + 1] = cnt;
    }
  *count = cnt;
  if (cnt > max) return fail(ctx, DASS_E_CAPACITY, "view has %lld keys", (long long)cnt);
  if (cnt > 0 && (!keys || !vals)) return DASS_E_INVALID;
  HIP_TRY(ctx, hipMemcpy(ranges, rel.data(), rel.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  for (int t = 0; t < nt; t++)
    if (r[t].y > r[t].x)
      launch_debug_keys(view, ctx->fwd_n, ctx->ws, ctx->ws.keys[ctx->fwd_key_buf], ctx->ws.vals[ctx->fwd_key_buf],
                        r[t].x, r[t].y - r[t].x, c, keys + rel[2 * t], vals + rel[2 * t], nullptr);
  HIP_TRY(ctx, hipDeviceSynchronize());
  return check_launch(ctx, "dass_debug_keys");
}

dass_status dass_debug_projection(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cam,
                                  const dass_opts* opts, double* out) {
  if (!ctx) return DASS_E_INVALID;
  dass_status s;
  if ((s = check_scene(ctx, g)) != DASS_OK) return s;
  if (!out) return fail(ctx, DASS_E_INVALID, "out is NULL");
  int tw, th, sub, batch;
  if ((s = check_opts(ctx, opts, tw, th, sub, batch)) != DASS_OK) return s;
  (void)sub;
  CamsK ck;
  int64_t total = 0;
  const int64_t keep = ctx->ws.cap_tiles;
  ctx->ws.cap_tiles = INT64_MAX;  // the tile budget does not apply to this export
  s = make_cams(ctx, cam, 1, tw, th, ck, total);
  ctx->ws.cap_tiles = keep;
  if (s != DASS_OK) return s;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  launch_debug_projection(scene_of(g), ck, 0, out, nullptr);
  HIP_TRY(ctx, hipDeviceSynchronize());
  return check_launch(ctx, "dass_debug_projection");
}

dass_status dass_profile_begin(dass_ctx ctx, int32_t max_records) {
  if (!ctx || max_records < 1) return DASS_E_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  profile_free(ctx);
  Profiler& p = ctx->prof;
  for (int s = 0; s < DASS_NUM_STAGES; s++) {
    p.ev[s].resize(2 * (size_t)max_records);
    for (auto& e : p.ev[s]) HIP_TRY(ctx, hipEventCreate(&e));
  }
  p.max = max_records;
  p.on = true;
  return DASS_OK;
}

dass_status dass_profile_end(dass_ctx ctx, double* total_ms, int32_t* records) {
  if (!ctx) return DASS_E_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Profiler& p = ctx->prof;
  HIP_TRY(ctx, hipDeviceSynchronize());
  for (int s = 0; s < DASS_NUM_STAGES; s++) {
    double acc = 0.0;
    for (int i = 0; i < p.used[s]; i++) {
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, p.ev[s][2 * i], p.ev[s][2 * i + 1]));
      acc += ms;
    }
    if (total_ms) total_ms[s] = acc;
    if (records) records[s] = p.used[s];
  }
  profile_free(ctx);
  return DASS_OK;
}

dass_status dass_debug_pair_counts(dass_ctx ctx, uint64_t* evaluated, uint64_t* blended) {
  if (!ctx || !evaluated || !blended) return DASS_E_INVALID;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipDeviceSynchronize());
  unsigned long long h[2];
  HIP_TRY(ctx, hipMemcpy(h, ctx->ws.pairs, sizeof(h), hipMemcpyDeviceToHost));
  *evaluated = h[0];
  *blended = h[1];
  return DASS_OK;
}

dass_status dass_autotune_tile(dass_ctx ctx, const dass_gaussians* g, const dass_camera* cams, int32_t n_views,
                               const float bg[3], dass_image* out, const float* const* dl_drgb, dass_grads* grads,
                               const dass_opts* candidates, int32_t n_candidates, int32_t reps, int32_t* best,
                               float* ms, dass_stream stream) {
  if (!ctx) return DASS_E_INVALID;
  if (!candidates || n_candidates < 1 || reps < 1 || !best || !ms)
    return fail(ctx, DASS_E_INVALID, "autotune: bad candidate list, reps or output pointers");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dass_status s = DASS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s = fail(ctx, DASS_E_HIP, "autotune: hipEventCreate failed");
  }
  *best = -1;
  float best_ms = 0.f;
  for (int c = 0; c < n_candidates && s == DASS_OK; c++) {
    ms[c] = -1.f;  // stays negative for a candidate that does not fit the context's budgets
    const dass_opts* o = &candidates[c];
    auto one = [&]() -> dass_status {
      dass_status r = render_fwd(ctx, g, cams, n_views, bg, out, o, stream);
      if (r == DASS_OK) r = render_bwd(ctx, g, cams, n_views, bg, out, dl_drgb, grads, nullptr, nullptr, o, stream);
      return r;
    };
    dass_status r = one();  // warm-up; also finds a tile or key budget this tile size exceeds
    if (r == DASS_OK) r = dass_sync(ctx, stream);
    if (r == DASS_E_CAPACITY) continue;
    if (r != DASS_OK) {
      s = r;
      break;
    }
    if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) {
      s = fail(ctx, DASS_E_HIP, "autotune: hipEventRecord failed");
      break;
    }
    for (int i = 0; i < reps && r == DASS_OK; i++) r = one();
    if (r == DASS_OK && hipEventRecord(e1, (hipStream_t)stream) != hipSuccess)
      r = fail(ctx, DASS_E_HIP, "autotune: hipEventRecord failed");
    if (r == DASS_OK) r = dass_sync(ctx, stream);
    if (r != DASS_OK) {
      s = r;
      break;
    }
    float t = 0.f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      s = fail(ctx, DASS_E_HIP, "autotune: hipEventElapsedTime failed");
      break;
    }
    ms[c] = t / (float)reps;
    if (*best < 0 || ms[c] < best_ms) {
      *best = c;
      best_ms = ms[c];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // the first candidate (in the caller's order of preference) within 1% of the fastest, so that
  // timing noise between near-equal sizes does not flip the choice from run to run (at 2% a
  // tile size whose key sort takes a second pass was chosen while 1.6% behind the fastest)
  if (s == DASS_OK && *best >= 0) {
    for (int c = 0; c < n_candidates; c++)
      if (ms[c] >= 0.f && ms[c] <= 1.01f * best_ms) {
        *best = c;
        break;
      }
  }
  ctx->have_fwd = false;  // the kept state belongs to the last candidate: render again before render_bwd
  if (s == DASS_OK && *best < 0) s = fail(ctx, DASS_E_CAPACITY, "autotune: no candidate fits the context's budgets");
  return s;
}

}  // extern "C"
