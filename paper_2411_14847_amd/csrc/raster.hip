// Tile binning and the front-to-back blend with its adjoint (App. A.1).
//
// Binning.  After the per-view depth sort of (view, depth bits, index), the projected records
// are permuted into that order, so a Gaussian's sorted position p already encodes its view
// and depth rank.  Keys are then just global tile ids (view tile base + ty*TX + tx), emitted
// in p order and sorted stably on the tile bits only; the stable order inside a tile is the
// depth order.  Ranges are the [first, last+1) of each tile id.
//
// Blend.  One 256-thread workgroup per 16x16 tile; each wave owns an 8x8 quadrant.  The tile's
// list is consumed in batches of 256 entries staged in LDS; every lane walks its pixel front
// to back, and the workgroup stops as soon as every pixel has hit the transmittance stop.
// The backward recomputes each entry's alpha per batch, recovers the transmittance by dividing
// out (1 - alpha) from T_final while walking backwards, sums each Gaussian's 9 gradient terms
// over the wave and issues one vector atomic per (Gaussian, wave).
#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kBatchB = 256;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ int xcd_logical(int bid, int per) {
  // consecutive workgroups land on different XCDs; give each XCD a contiguous tile range
  return (bid % kNumXcd) * per + bid / kNumXcd;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n; j += stride) p[j] = v;
}

__global__ __launch_bounds__(256) void k_gather_sorted(int n, int64_t vn, const uint32_t* __restrict__ sorted_gid,
                                                       const Rec* __restrict__ rec_u, const uint32_t* __restrict__ tt_u,
                                                       const uint2* __restrict__ rect_u, Rec* __restrict__ rec_s,
                                                       uint32_t* __restrict__ tt_s, uint2* __restrict__ rect_s,
                                                       uint32_t* __restrict__ inv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= vn) return;
  const int64_t v = p / n;
  const int64_t i = v * n + sorted_gid[p];
  rec_s[p] = rec_u[i];
  tt_s[p] = tt_u[i];
  rect_s[p] = rect_u[i];
  inv[i] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_emit_keys(int n, int64_t vn, CamsK cams, const uint32_t* __restrict__ tt_s,
                                                   const uint2* __restrict__ rect_s, const uint64_t* __restrict__ off,
                                                   int64_t cap, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= vn) return;
  const uint32_t tt = tt_s[p];
  if (tt == 0) return;
  const int v = (int)(p / n);
  const CamK& c = cams.c[v];
  const uint2 r = rect_s[p];
  const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
  uint64_t k = off[p];
  if (k + tt > (uint64_t)cap) atomicOr(err, kErrKeyOverflow);
  for (int ty = y0; ty < y1; ty++)
    for (int tx = x0; tx < x1; tx++, k++)
      if (k < (uint64_t)cap) {
        keys[k] = (uint32_t)(c.tile_base + ty * c.TX + tx);
        vals[k] = (uint32_t)p;
      }
}

__global__ void k_clamp_count(const uint64_t* __restrict__ total, int64_t cap, uint32_t* __restrict__ count) {
  const uint64_t t = *total;
  *count = (uint32_t)(t < (uint64_t)cap ? t : (uint64_t)cap);
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ d_count,
                                                uint2* __restrict__ ranges) {
  const uint32_t count = *d_count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint32_t t = keys[i];
    if (i == 0 || keys[i - 1] != t) ranges[t].x = (uint32_t)i;
    if (i == count - 1 || keys[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
  }
}

__device__ __forceinline__ int view_of(const ViewsIO& io, int nv, int b) {
  int v = 0;
  while (v + 1 < nv && b >= io.v[v + 1].tile_base) v++;
  return v;
}

template <bool COUNT>
__global__ __launch_bounds__(kTilePix) void k_blend_fwd(ViewsIO io, int nv, int total_tiles, int per, float bg0,
                                                        float bg1, float bg2, const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ vals,
                                                        const Rec* __restrict__ rec_s,
                                                        unsigned long long* __restrict__ pairs) {
  __shared__ float2 s_xy[kBatchB];
  __shared__ float4 s_co[kBatchB];
  __shared__ float4 s_rgb[kBatchB];
  const int b = xcd_logical(blockIdx.x, per);
  if (b >= total_tiles) return;
  const int v = view_of(io, nv, b);
  const ViewIO& V = io.v[v];
  const int t = b - V.tile_base;
  const int tx = t % V.TX, ty = t / V.TX;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
  const int px = tx * kTile + lx, py = ty * kTile + ly;
  const bool inside = px < V.W && py < V.H;
  const float fx0 = (float)(tx * kTile), fy0 = (float)(ty * kTile);
  const float flx = (float)lx, fly = (float)ly;
  const uint2 r = ranges[b];
  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  int last = 0;
  bool done = !inside;
  uint32_t n_eval = 0, n_blend = 0;
  for (uint32_t start = r.x; start < r.y; start += kBatchB) {
    const int n_in = (int)min((uint32_t)kBatchB, r.y - start);
    if (tid < n_in) {
      const uint32_t p = vals[start + tid];
      const Rec R = rec_s[p];
      s_xy[tid] = make_float2((R.r0.x - fx0) + R.r0.z, (R.r0.y - fy0) + R.r0.w);
      s_co[tid] = make_float4(-0.5f * kLog2e * R.r1.x, -kLog2e * R.r1.y, -0.5f * kLog2e * R.r1.z, R.r1.w);
      s_rgb[tid] = make_float4(R.r2.x, R.r2.y, R.r2.z, 0.f);
    }
    __syncthreads();
    if (!done) {
      const int base = (int)(start - r.x);
      for (int j = 0; j < n_in; j++) {
        const float2 xy = s_xy[j];
        const float4 co = s_co[j];
        const float dx = xy.x - flx, dy = xy.y - fly;
        const float pw = co.x * dx * dx + co.z * dy * dy + co.y * dx * dy;
        if (COUNT) n_eval++;
        if (pw > 0.f) continue;
        const float a = fminf(kAlphaMax, co.w * __builtin_amdgcn_exp2f(pw));
        if (a < kAlphaMin) continue;
        const float Tn = T * (1.f - a);
        if (Tn < kTStop) {
          done = true;
          break;
        }
        if (COUNT) n_blend++;
        const float4 c = s_rgb[j];
        const float w = a * T;
        c0 += c.x * w;
        c1 += c.y * w;
        c2 += c.z * w;
        T = Tn;
        last = base + j + 1;
      }
    }
    if (__syncthreads_count(done) == kTilePix) break;
  }
  if (inside) {
    const int64_t hw = (int64_t)V.W * V.H;
    const int64_t pix = (int64_t)py * V.W + px;
    V.rgb[pix] = c0 + T * bg0;
    V.rgb[hw + pix] = c1 + T * bg1;
    V.rgb[2 * hw + pix] = c2 + T * bg2;
    V.t_final[pix] = T;
    V.n_contrib[pix] = last;
  }
  if (COUNT) {
    atomicAdd(&pairs[0], (unsigned long long)n_eval);
    atomicAdd(&pairs[1], (unsigned long long)n_blend);
  }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ __launch_bounds__(kTilePix) void k_blend_bwd(ViewsIO io, int nv, int total_tiles, int per, float bg0,
                                                        float bg1, float bg2, const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ vals,
                                                        const Rec* __restrict__ rec_s, float* __restrict__ g2d) {
  __shared__ float2 s_xy[kBatchB];
  __shared__ float4 s_co[kBatchB];   // log2-scaled conic + opacity (as the forward)
  __shared__ float4 s_cn[kBatchB];   // conic A, B, C
  __shared__ float4 s_rgb[kBatchB];
  __shared__ uint32_t s_p[kBatchB];
  __shared__ int s_max;
  const int b = xcd_logical(blockIdx.x, per);
  if (b >= total_tiles) return;
  const int v = view_of(io, nv, b);
  const ViewIO& V = io.v[v];
  const int t = b - V.tile_base;
  const int tx = t % V.TX, ty = t / V.TX;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
  const int px = tx * kTile + lx, py = ty * kTile + ly;
  const bool inside = px < V.W && py < V.H;
  const float fx0 = (float)(tx * kTile), fy0 = (float)(ty * kTile);
  const float flx = (float)lx, fly = (float)ly;
  const uint2 r = ranges[b];
  const int64_t hw = (int64_t)V.W * V.H;
  const int64_t pix = (int64_t)py * V.W + px;
  float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f;
  int last = 0;
  if (inside) {
    T = V.t_final[pix];
    last = V.n_contrib[pix];
    dC0 = V.dl[pix];
    dC1 = V.dl[hw + pix];
    dC2 = V.dl[2 * hw + pix];
  }
  float B0 = bg0, B1 = bg1, B2 = bg2;  // colour behind the current entry
  if (tid == 0) s_max = 0;
  __syncthreads();
  atomicMax(&s_max, last);
  __syncthreads();
  const int max_last = min(s_max, (int)(r.y - r.x));  // n_contrib never exceeds the list length
  if (max_last <= 0) return;
  const int nbatch = (max_last + kBatchB - 1) / kBatchB;
  for (int bi = nbatch - 1; bi >= 0; bi--) {
    const uint32_t start = r.x + (uint32_t)bi * kBatchB;
    const int n_in = min(kBatchB, max_last - bi * kBatchB);
    __syncthreads();
    if (tid < n_in) {
      const uint32_t p = vals[start + tid];
      const Rec R = rec_s[p];
      s_xy[tid] = make_float2((R.r0.x - fx0) + R.r0.z, (R.r0.y - fy0) + R.r0.w);
      s_co[tid] = make_float4(-0.5f * kLog2e * R.r1.x, -kLog2e * R.r1.y, -0.5f * kLog2e * R.r1.z, R.r1.w);
      s_cn[tid] = make_float4(R.r1.x, R.r1.y, R.r1.z, 0.f);
      s_rgb[tid] = make_float4(R.r2.x, R.r2.y, R.r2.z, 0.f);
      s_p[tid] = p;
    }
    __syncthreads();
    for (int j = n_in - 1; j >= 0; j--) {
      const int idx = bi * kBatchB + j;
      const float2 xy = s_xy[j];
      const float4 co = s_co[j];
      const float dx = xy.x - flx, dy = xy.y - fly;
      const float pw = co.x * dx * dx + co.z * dy * dy + co.y * dx * dy;
      const float G = __builtin_amdgcn_exp2f(pw);
      const float araw = co.w * G;
      const float a = fminf(kAlphaMax, araw);
      const bool valid = (idx < last) && (pw <= 0.f) && (a >= kAlphaMin);
      float g[9];
      if (valid) {
        T = T / (1.f - a);
        const float4 c = s_rgb[j];
        const float w = a * T;
        g[6] = w * dC0;
        g[7] = w * dC1;
        g[8] = w * dC2;
        const float da = T * ((c.x - B0) * dC0 + (c.y - B1) * dC1 + (c.z - B2) * dC2);
        B0 = a * c.x + (1.f - a) * B0;
        B1 = a * c.y + (1.f - a) * B1;
        B2 = a * c.z + (1.f - a) * B2;
        const bool clamped = araw >= kAlphaMax;
        const float dP = clamped ? 0.f : da * a;
        g[5] = clamped ? 0.f : da * G;
        const float4 cn = s_cn[j];
        g[0] = dP * (-cn.x * dx - cn.y * dy);
        g[1] = dP * (-cn.z * dy - cn.y * dx);
        g[2] = -0.5f * dP * dx * dx;
        g[3] = -dP * dx * dy;
        g[4] = -0.5f * dP * dy * dy;
      } else {
#pragma unroll
        for (int k = 0; k < 9; k++) g[k] = 0.f;
      }
      if (__ballot(valid) != 0) {
#pragma unroll
        for (int k = 0; k < 9; k++) g[k] = wave_sum(g[k]);
        float mine = g[0];
#pragma unroll
        for (int k = 1; k < 9; k++) mine = (lane == k) ? g[k] : mine;
        if (lane < 9) atomicAdd(&g2d[(int64_t)s_p[j] * 9 + lane], mine);
      }
    }
  }
}

__global__ void k_debug_keys(int view_tile_base, const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                             const Rec* __restrict__ rec_s, const uint32_t* __restrict__ gid_s, uint32_t lo,
                             uint32_t cnt, uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t k = keys[lo + i];
  const uint32_t p = vals[lo + i];
  kout[i] = ((uint64_t)(k - (uint32_t)view_tile_base) << 32) | (uint64_t)__float_as_uint(rec_s[p].r2.w);
  vout[i] = gid_s[p];
}

__global__ void k_debug_ranges(const uint2* __restrict__ ranges, int tile_base, int n_tiles, uint32_t lo,
                               int64_t* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint2 r = ranges[tile_base + t];
  const bool empty = r.y <= r.x;
  out[2 * t] = empty ? 0 : (int64_t)(r.x - lo);
  out[2 * t + 1] = empty ? 0 : (int64_t)(r.y - lo);
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_u32<<<(unsigned)blocks, 256, 0, st>>>(p, v, n);
}

void launch_gather_sorted(int n, int64_t vn, const uint32_t* sorted_gid, Workspace& ws, hipStream_t st) {
  if (vn == 0) return;
  k_gather_sorted<<<(unsigned)((vn + 255) / 256), 256, 0, st>>>(n, vn, sorted_gid, ws.rec_u, ws.tt_u, ws.rect_u,
                                                                 ws.rec_s, ws.tt_s, ws.rect_s, ws.inv);
}

void launch_emit_keys(int n, int64_t vn, const CamsK& cams, Workspace& ws, hipStream_t st) {
  scan_u32_to_u64(ws.tt_s, ws.off_s, vn, ws.scan_tmp, st);
  if (vn > 0)
    k_emit_keys<<<(unsigned)((vn + 255) / 256), 256, 0, st>>>(n, vn, cams, ws.tt_s, ws.rect_s, ws.off_s, ws.cap_keys,
                                                               ws.keys[0], ws.vals[0], ws.err);
  k_clamp_count<<<1, 1, 0, st>>>(ws.off_s + vn, ws.cap_keys, ws.counters);
}

void launch_ranges(const uint32_t* keys, int64_t total_tiles, Workspace& ws, hipStream_t st) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(ws.ranges), 0u, 2 * total_tiles, st);
  int64_t blocks = (ws.cap_keys + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  k_ranges<<<(unsigned)blocks, 256, 0, st>>>(keys, ws.counters, ws.ranges);
}

static inline int per_xcd(int64_t total_tiles) { return (int)((total_tiles + kNumXcd - 1) / kNumXcd); }

void launch_blend_fwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3], const Workspace& ws,
                      const uint32_t* vals, bool count_pairs, hipStream_t st) {
  if (total_tiles == 0) return;
  const int per = per_xcd(total_tiles);
  if (count_pairs)
    k_blend_fwd<true><<<per * kNumXcd, kTilePix, 0, st>>>(io, nv, (int)total_tiles, per, bg[0], bg[1], bg[2],
                                                           ws.ranges, vals, ws.rec_s, ws.pairs);
  else
    k_blend_fwd<false><<<per * kNumXcd, kTilePix, 0, st>>>(io, nv, (int)total_tiles, per, bg[0], bg[1], bg[2],
                                                            ws.ranges, vals, ws.rec_s, nullptr);
}

void launch_blend_bwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3], const Workspace& ws,
                      const uint32_t* vals, hipStream_t st) {
  if (total_tiles == 0) return;
  const int per = per_xcd(total_tiles);
  k_blend_bwd<<<per * kNumXcd, kTilePix, 0, st>>>(io, nv, (int)total_tiles, per, bg[0], bg[1], bg[2], ws.ranges, vals,
                                                   ws.rec_s, ws.g2d);
}

void launch_debug_keys(int view, int n, const Workspace& ws, const uint32_t* keys_sorted, const uint32_t* vals_sorted,
                       uint32_t lo, uint32_t cnt, const CamK& cam, uint64_t* kout, uint32_t* vout, int64_t* rout,
                       hipStream_t st) {
  (void)view;
  (void)n;
  if (cnt > 0)
    k_debug_keys<<<(cnt + 255) / 256, 256, 0, st>>>(cam.tile_base, keys_sorted, vals_sorted, ws.rec_s, ws.gid_s, lo,
                                                     cnt, kout, vout);
  const int nt = cam.TX * cam.TY;
  k_debug_ranges<<<(nt + 255) / 256, 256, 0, st>>>(ws.ranges, cam.tile_base, nt, lo, rout);
}

}  // namespace dass
