// Tile binning and the front-to-back blend with its adjoint (App. A.1).
//
// Binning.  After the per-view depth sort of (view, depth bits, index), the tile counts and
// rectangles are gathered into that order.  Keys are then just global tile ids (view tile base
// + ty*TX + tx), emitted in (view, depth) order with the record index (view * n + Gaussian) as
// value and sorted stably on the tile bits only; the stable order inside a tile is the depth
// order.  Ranges are the [first, last+1) of each tile id.
//
// Blend.  One wave per sub-tile of a tile (16x16 with four pixels per lane, one in each 8x8
// quadrant, or 8x8 with one pixel per lane, for small images where the lists are walked by few
// waves).  The tile's list is consumed in batches of 64, 128 or 256 entries (a per-call option),
// each culled against the quadrants of the wave's sub-tile and compacted into LDS; every lane walks its pixels front
// to back, skipping the quadrants an entry misses, and the wave stops as soon as every pixel
// has hit the transmittance stop.
// The backward recomputes each entry's alpha per batch, recovers the transmittance by dividing
// out (1 - alpha) from T_final while walking backwards, sums each Gaussian's 9 gradient terms
// over the wave and issues one vector atomic per (Gaussian, wave).
#include "dass_internal.h"

namespace dass {
namespace {

// B: list entries staged in LDS per batch (64, 128 or 256; a per-call option)
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

// Tile rectangle and tiles touched (the rectangle's area) of each (view, Gaussian) in (view,
// depth) order, for the scan and the key emission: one gathered 8-byte rectangle per position;
// the records themselves stay where the projection wrote them.
__global__ __launch_bounds__(256) void k_gather_sorted(int n, int64_t vn, const uint32_t* __restrict__ sorted_gid,
                                                       const uint2* __restrict__ rect_u, uint32_t* __restrict__ tt_s,
                                                       uint2* __restrict__ rect_s) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= vn) return;
  const int64_t v = p / n;
  const uint2 r = rect_u[v * n + sorted_gid[p]];
  tt_s[p] = ((r.y & 0xFFFFu) - (r.x & 0xFFFFu)) * ((r.y >> 16) - (r.x >> 16));
  rect_s[p] = r;
}

// Each wave takes 64 consecutive sorted positions (Gaussian-views) and writes all their keys
// (value: the record index of the Gaussian-view) with the keys spread evenly over the lanes: lane l writes keys l, l + 64, ... of the wave's
// run, finding the owning Gaussian by a binary search over the run's end offsets in LDS.  The
// stores of a wave are consecutive, whatever the tile counts.
__global__ __launch_bounds__(256) void k_emit_keys(int n, int64_t vn, CamsK cams, const uint32_t* __restrict__ tt_s,
                                                   const uint2* __restrict__ rect_s, const uint32_t* __restrict__ sorted_gid,
                                                   const uint64_t* __restrict__ off, int64_t cap,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ err) {
  __shared__ uint32_t s_end[4][64];   // end of each Gaussian's keys, relative to the wave's first key
  __shared__ uint4 s_g[4][64];        // key of the rectangle's first tile, TX, width, 1/width
  __shared__ uint32_t s_rec[4][64];   // record index (view * n + Gaussian) = the keys' value
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;  // first position of this wave
  if (p0 >= vn) return;  // uniform over the wave
  const int64_t pm = p0 + lane;
  const bool valid = pm < vn;
  uint32_t my_tt = 0;
  uint64_t my_off = 0;
  if (valid) {
    my_tt = tt_s[pm];
    my_off = off[pm];
    if (my_off + my_tt > (uint64_t)cap) atomicOr(err, kErrKeyOverflow);
    const uint2 r = rect_s[pm];
    const int v = (int)(pm / n);
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF;
    const int w = max(x1 - x0, 1);
    const int TX = cams.c[v].TX;
    s_g[wave][lane] = make_uint4(cams.c[v].key_base + (uint32_t)(y0 * TX + x0), (uint32_t)TX, (uint32_t)w,
                                 __float_as_uint(1.0f / (float)w));
    s_rec[wave][lane] = (uint32_t)((int64_t)v * n + sorted_gid[pm]);
  }
  const uint64_t first = __shfl(my_off, 0, 64);
  const uint32_t end = valid ? (uint32_t)(my_off - first) + my_tt : 0xFFFFFFFFu;  // non-decreasing over lanes
  s_end[wave][lane] = end;
  const int last = (int)min((int64_t)63, vn - 1 - p0);
  const uint32_t total = __shfl(end, last, 64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint32_t k = lane; k < total; k += 64) {
    int src = 0;  // number of Gaussians whose keys end at or before k
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (s_end[wave][src + step - 1] <= k) src += step;
    const uint32_t i = k - (src ? s_end[wave][src - 1] : 0u);  // key index within the Gaussian
    const uint4 gg = s_g[wave][src];
    // i / width by a float reciprocal, corrected to the exact quotient (i < 2^24)
    uint32_t q = (uint32_t)((float)i * __uint_as_float(gg.w));
    int32_t r = (int32_t)(i - q * gg.z);
    if (r < 0) {
      q--;
      r += (int32_t)gg.z;
    } else if (r >= (int32_t)gg.z) {
      q++;
      r -= (int32_t)gg.z;
    }
    const uint64_t kk = first + k;
    if (kk < (uint64_t)cap) {
      keys[kk] = gg.x + q * gg.y + (uint32_t)r;
      vals[kk] = s_rec[wave][src];
    }
  }
}

__global__ void k_clamp_count(const uint64_t* __restrict__ total, int64_t cap, uint32_t* __restrict__ count) {
  const uint64_t t = *total;
  *count = (uint32_t)(t < (uint64_t)cap ? t : (uint64_t)cap);
}

// Global tile index of a key: the view's first tile plus the tile within the view.
struct KeyTiles {
  int tile_base[DASS_MAX_VIEWS];
  int local_bits, nv;
  uint32_t total_tiles;
};

// Per-tile ranges of the sorted keys: four consecutive keys per thread (one 16-byte load) and
// their two neighbours; a key that differs from its predecessor starts a range, one that differs
// from its successor ends it.  Ranges are stored by global tile index.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ d_count,
                                                const KeyTiles kt, uint2* __restrict__ ranges) {
  const int64_t count = *d_count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i0 < count; i0 += stride) {
    uint32_t k[6];  // keys i0 - 1 .. i0 + 4 (entries outside [0, count) unused)
    if (i0 + 4 <= count) {
      const uint4 v = *reinterpret_cast<const uint4*>(keys + i0);
      k[1] = v.x;
      k[2] = v.y;
      k[3] = v.z;
      k[4] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; j++) k[1 + j] = i0 + j < count ? keys[i0 + j] : 0u;
    }
    k[0] = i0 > 0 ? keys[i0 - 1] : 0u;
    k[5] = i0 + 4 < count ? keys[i0 + 4] : 0u;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = i0 + j;
      if (i >= count) break;
      const uint32_t key = k[1 + j];
      const bool starts = i == 0 || k[j] != key, ends = i == count - 1 || k[2 + j] != key;
      if (!starts && !ends) continue;
      const uint32_t v = key >> kt.local_bits;
      if (v >= (uint32_t)kt.nv) continue;  // not reached: every key below the count was emitted
      const uint32_t t = (uint32_t)kt.tile_base[v] + (key & ((1u << kt.local_bits) - 1u));
      if (t >= kt.total_tiles) continue;
      if (starts) ranges[t].x = (uint32_t)i;
      if (ends) ranges[t].y = (uint32_t)(i + 1);
    }
  }
}

__device__ __forceinline__ int view_of(const ViewsIO& io, int nv, int b) {
  int v = 0;
  while (v + 1 < nv && b >= io.v[v + 1].tile_base) v++;
  return v;
}

// ---- blend ------------------------------------------------------------------------------------
// One wave per sub-tile (16x16 or 8x8 pixels).  The sub-tile is cut into 8x8 quadrants and
// lane (qx, qy) of the 8x8 lane grid owns pixel (qx, qy) of every quadrant.  Batches of up to
// 128 list entries are loaded by the wave, culled per quadrant and compacted into LDS in list
// order; an entry leaves a quadrant only if the minimum of its quadratic form over the
// quadrant's pixel rectangle exceeds the alpha >= 1/255 level by a margin, i.e. when every pixel
// of that quadrant would skip it anyway, and leaves the list when no quadrant keeps it.  The list
// position of every kept entry is carried along (low 27 bits, the quadrant mask in the top four),
// so n_contrib still counts positions in the full list; the walk skips a quadrant an entry misses
// with a uniform branch.
// An entry's alpha never exceeds its opacity, so only an entry with opacity >= 0.99 can meet the
// alpha clamp; the backward marks those (kClampBit) and tests the clamp for its zero derivative
// on them alone.  For any other entry the clamp is inactive in the definition's arithmetic (the
// opacity times a falloff <= 1 is below 0.99), and an alpha that float32 rounds to 0.99 there
// keeps its derivative.
constexpr int kLanes = 64;
constexpr int kPosBits = 27;  // list positions carried with the clamp bit and the quadrant mask
constexpr int kPosMask = (1 << kPosBits) - 1;
constexpr uint32_t kClampBit = 1u << kPosBits;
constexpr int kQmShift = 28;
constexpr float kNever = 2.0f;  // alpha threshold of a stopped pixel: above every alpha (<= 0.99)

__device__ __forceinline__ uint64_t lane_lt_mask(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// Minimum of q(d) = A dx^2 + 2B dx dy + C dy^2, d = pixel - mean, over the pixel-centre
// rectangle [x0, x1] x [y0, y1] (mean at (mx, my)); ia, ic = 1/A, 1/C (0 if not positive).  For
// a convex q the minimiser is the mean when it lies inside; otherwise it lies on the edge that
// faces the mean in x (when mx is outside [x0, x1]) or on the one that faces it in y: the
// vertical segment at the rectangle's x nearest mx and the horizontal segment at its y nearest my
// hold it in every case, and on each segment the line minimiser is clamped to the segment.
__device__ __forceinline__ float rect_min_q(float mx, float my, float A, float B, float C, float ia, float ic,
                                            float x0, float x1, float y0, float y1) {
  // (med3 of a value and an ordered pair clamps it to the pair's interval)
  float dx = __builtin_amdgcn_fmed3f(mx, x0, x1) - mx;
  float dy = __builtin_amdgcn_fmed3f(-B * dx * ic, y0 - my, y1 - my);
  const float qv = A * dx * dx + 2.f * B * dx * dy + C * dy * dy;
  dy = __builtin_amdgcn_fmed3f(my, y0, y1) - my;
  dx = __builtin_amdgcn_fmed3f(-B * dy * ia, x0 - mx, x1 - mx);
  const float qh = A * dx * dx + 2.f * B * dx * dy + C * dy * dy;
  return fminf(qv, qh);
}

// Bit k set if the entry (mean (mx, my) relative to the sub-tile origin, conic A B C, opacity o)
// may reach alpha >= 1/255 at a pixel centre of 8x8 quadrant k = (k % PW, k / PW).
template <int PW>
__device__ __forceinline__ uint32_t quad_mask(float mx, float my, float A, float B, float C, float o) {
  if (!(o * 255.0f > 0.999f)) return 0u;  // alpha <= o < 1/255 everywhere (with margin)
  // q <= 2 ln(255 o)  <=>  o exp(-q/2) >= 1/255; the margin keeps every kept decision
  // (hardware log2: 255 o > 1 here, and the margin covers its rounding)
  const float thr = (2.0f * 0.6931471805599453f) * __builtin_amdgcn_logf(255.0f * o) * 1.001f + 1e-3f;
  const float ia = A > 0.f ? __builtin_amdgcn_rcpf(A) : 0.f, ic = C > 0.f ? __builtin_amdgcn_rcpf(C) : 0.f;
  uint32_t m = 0;
  if constexpr (PW == 2) {
    // rect_min_q for the 2x2 grid of quadrants, sharing the work of each column and row: the
    // vertical segment of column cx sits at the same x (and the line minimiser there at the
    // same y) for both rows, and likewise for the horizontal segment of row cy; relative to the
    // mean, clamp(mx, x0, x1) - mx = clamp(0, x0 - mx, x1 - mx).
    const float xl[2] = {-mx, 8.f - mx}, xh[2] = {7.f - mx, 15.f - mx};
    const float yl[2] = {-my, 8.f - my}, yh[2] = {7.f - my, 15.f - my};
    const float nbc = -B * ic, nba = -B * ia, b2 = 2.f * B;
    float qv[4];
#pragma unroll
    for (int cx = 0; cx < 2; cx++) {
      const float dx = __builtin_amdgcn_fmed3f(0.f, xl[cx], xh[cx]);
      const float ys = dx * nbc, ax = A * dx * dx, bx = b2 * dx;
#pragma unroll
      for (int cy = 0; cy < 2; cy++) {
        const float dy = __builtin_amdgcn_fmed3f(ys, yl[cy], yh[cy]);
        qv[cx + 2 * cy] = fmaf(dy, fmaf(C, dy, bx), ax);  // A dx^2 + 2B dx dy + C dy^2
      }
    }
#pragma unroll
    for (int cy = 0; cy < 2; cy++) {
      const float dy = __builtin_amdgcn_fmed3f(0.f, yl[cy], yh[cy]);
      const float xs = dy * nba, cy2 = C * dy * dy, by = b2 * dy;
#pragma unroll
      for (int cx = 0; cx < 2; cx++) {
        const float dx = __builtin_amdgcn_fmed3f(xs, xl[cx], xh[cx]);
        const float qh = fmaf(dx, fmaf(A, dx, by), cy2);
        if (fminf(qv[cx + 2 * cy], qh) <= thr) m |= 1u << (cx + 2 * cy);
      }
    }
    return m;
  }
#pragma unroll 1  // rolled: unrolled, the four rectangles cost the forward an occupancy step
  for (int k = 0; k < PW * PW; k++) {
    const float x0 = (float)(8 * (k % PW)), y0 = (float)(8 * (k / PW));
    if (rect_min_q(mx, my, A, B, C, ia, ic, x0, x0 + 7.f, y0, y0 + 7.f) <= thr) m |= 1u << k;
  }
  return m;
}

template <int CTRL>
__device__ __forceinline__ float dppf(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Transposing reduction of 9 per-lane values over the wave: each step pairs values (x, y) and
// adds every value to its copy on the partner lane across one lane bit, keeping x's pair total
// on the lanes with that bit clear and y's on the lanes with it set, so the number of values
// per lane halves at each step without selects.
// Lane bits 5 and 4 (partners 32 or 16 lanes apart): gfx950's permlane swaps exchange the upper
// half of x with the lower half of y (the odd 16-lane rows of x with the even rows of y), after
// which x + y holds x's total on one side and y's on the other.
__device__ __forceinline__ float swap32_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Lane bits 3 and 2 (partners 8 or 4 lanes apart in a 16-lane row): two DPP adds whose bank
// masks (a bank is 4 consecutive lanes of a row) write complementary halves of the lanes.  The
// leading s_nop gives the DPP reads of x and y the two wait states they need after a VALU write.
__device__ __forceinline__ float dpp_pair8(float x, float y) {
  float o;
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"  // lanes with bit 3 clear
      "v_add_f32_dpp %0, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xc"       // lanes with bit 3 set
      : "=&v"(o)
      : "v"(x), "v"(y));
  return o;
}
__device__ __forceinline__ float dpp_pair4(float x, float y) {
  float o;
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %1, %1 row_shl:4 row_mask:0xf bank_mask:0x5\n\t"  // bit 2 clear: lane + 4
      "v_add_f32_dpp %0, %2, %2 row_shr:4 row_mask:0xf bank_mask:0xa"       // bit 2 set: lane - 4
      : "=&v"(o)
      : "v"(x), "v"(y));
  return o;
}

// Sums v[0..8] over the wave.  Afterwards lane 4 m + i (i < 4) holds the total of value
// kRedSlot[m] (-1: a duplicate of another lane's total, or none).
__device__ __forceinline__ float wave_reduce9(const float* v) {
  // bit 5 -> upper half of the lanes holds values 5, 6, 7, 8, 4
  const float a0 = swap32_sum(v[0], v[5]), a1 = swap32_sum(v[1], v[6]), a2 = swap32_sum(v[2], v[7]);
  const float a3 = swap32_sum(v[3], v[8]), a4 = swap32_sum(v[4], v[4]);
  // bit 4 -> (bit 5, bit 4) = 00: 0 1 2, 01: 3 4 2, 10: 5 6 7, 11: 8 4 7
  const float b0 = swap16_sum(a0, a3), b1 = swap16_sum(a1, a4), b2 = swap16_sum(a2, a2);
  // bit 3 -> (bits 5..3) = 000: 0 1, 001: 2 1, 010: 3 4, 011: 2 4, 100: 5 6, 101: 7 6, 110: 8 4, 111: 7 4
  const float c0 = dpp_pair8(b0, b2);
  const float c1 = b1 + dppf<0x128>(b1);  // row_ror 8
  // bit 2 -> one value per lane (bits 5..2 = m, kRedSlot[m])
  float d = dpp_pair4(c0, c1);
  d += dppf<0xB1>(d);  // bits 1, 0: the four lanes of a bank (quad_perm 1,0,3,2 then 2,3,0,1)
  d += dppf<0x4E>(d);
  return d;
}
__constant__ int kRedSlot[16] = {0, 1, 2, -1, 3, 4, -1, -1, 5, 6, 7, -1, 8, -1, -1, -1};

// A staged list entry in LDS: one 48-byte row, so a wave reads an entry's fields from one address.
struct FwdStage {
  float4 co;   // log2-scaled conic, log2 opacity
  float4 rgb;  // colour, (list position + 1) | quadrant mask << 28 (int bits)
  float2 xy;   // mean relative to the sub-tile origin
  float2 pad;
};
struct BwdStage {
  float4 co;   // as the forward's
  float4 rgb;  // colour, list position | clamp bit | quadrant mask << 28 (int bits)
  float2 xy;
  uint32_t p;  // record index = gradient row (view * n + Gaussian)
  float io;    // 1 / opacity
};

// L1: the epilogue also forms the L1 term against the view's target (dL/drgb, error map and
// this sub-tile's share of the loss, added into one of kLossSlots partial sums).
template <bool COUNT, bool L1, int SUB, int B>
__global__ __launch_bounds__(kLanes) void k_blend_fwd(ViewsIO io, int nv, int total_blocks, int per, float bg0,
                                                      float bg1, float bg2, const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals, const Rec* __restrict__ rec,
                                                      unsigned long long* __restrict__ pairs,
                                                      float* __restrict__ loss_slots) {
  constexpr int PW = SUB / 8, NP = PW * PW;  // quadrants per edge, pixels per lane
  __shared__ FwdStage s_st[B];
  const int lb = xcd_logical(blockIdx.x, per);
  if (lb >= total_blocks) return;
  const int b = lb / io.sn, sub = lb - b * io.sn;  // tile, SUB x SUB sub-tile of it
  const int v = view_of(io, nv, b);
  const ViewIO& V = io.v[v];
  const int t = b - V.tile_base;
  const int tx = t % V.TX, ty = t / V.TX;
  const int ox = tx * io.tw + (sub % io.sx) * SUB, oy = ty * io.th + (sub / io.sx) * SUB;
  if (ox >= V.W || oy >= V.H) return;  // sub-tile entirely outside the image
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const float fx0 = (float)ox, fy0 = (float)oy;
  const uint64_t lt = lane_lt_mask(lane);
  const uint2 r = ranges[b];
  if (r.y - r.x > (uint32_t)kPosMask) {  // positions would not fit their bits: reported, not drawn
    if (lane == 0) atomicOr(io.err, kErrListTooLong);
    return;
  }
  // thr[k]: the alpha a pixel's entries must reach to blend; 1/255 while it walks its list,
  // kNever once it has stopped (or for a pixel outside the image), so it never blends again and
  // keeps its transmittance
  float T[NP], thr[NP], c0[NP], c1[NP], c2[NP];
  uint32_t last[NP];  // (list position + 1) of the last blended entry, quadrant mask above it
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int px = ox + qx + 8 * (k % PW), py = oy + qy + 8 * (k / PW);
    T[k] = 1.f;
    thr[k] = (px < V.W && py < V.H) ? kAlphaMin : kNever;
    c0[k] = c1[k] = c2[k] = 0.f;
    last[k] = 0;
  }
  uint32_t n_eval = 0, n_blend = 0;
  for (uint32_t start = r.x; start < r.y; start += B) {
    const int n_in = (int)min((uint32_t)B, r.y - start);
    int n_kept = 0;
#pragma unroll
    for (int k = 0; k < B / kLanes; k++) {
      const int e = k * kLanes + lane;
      uint32_t qm = 0;
      float2 xy;
      float4 co, rgb;
      if (e < n_in) {
        const Rec R = rec[vals[start + e]];
        xy = make_float2((R.r0.x - fx0) + R.r0.z, (R.r0.y - fy0) + R.r0.w);
        qm = quad_mask<PW>(xy.x, xy.y, R.r1.x, R.r1.y, R.r1.z, R.r1.w);
        // exponent in base 2 with the opacity folded in: alpha = 2^(q' + log2 o)
        co = make_float4(-0.5f * kLog2e * R.r1.x, -kLog2e * R.r1.y, -0.5f * kLog2e * R.r1.z, __log2f(R.r1.w));
        rgb = make_float4(R.r2.x, R.r2.y, R.r2.z,
                          __uint_as_float(((uint32_t)(start - r.x) + e + 1) | (qm << kQmShift)));
      }
      const bool keep = qm != 0;
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int pos = n_kept + __popcll(m & lt);
        s_st[pos].co = co;
        s_st[pos].rgb = rgb;
        s_st[pos].xy = xy;
      }
      n_kept += __popcll(m);
    }
    // quadrants with a pixel still walking (a stopped pixel stays stopped); a quadrant leaves the
    // mask as soon as its last pixel stops, and the wave leaves the batch when none is left
    uint32_t qalive = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) qalive |= __ballot(thr[k] < 1.f) != 0 ? 1u << k : 0u;
    __syncthreads();
    for (int j = 0; j < n_kept && qalive != 0; j++) {
      const float2 xy = s_st[j].xy;
      const float4 co = s_st[j].co;
      const float4 c = s_st[j].rgb;
      const uint32_t wv = __float_as_uint(c.w);  // (position + 1) | quadrant mask << 28
      const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)wv);  // same for all lanes
      const uint32_t qm = (w >> kQmShift) & qalive;
      const float dxb = xy.x - (float)qx, dyb = xy.y - (float)qy;
#pragma unroll
      for (int k = 0; k < NP; k++) {
        if (NP > 1 && !((qm >> k) & 1u)) continue;  // uniform: no pixel of quadrant k can take it
        const float dx = dxb - (float)(8 * (k % PW)), dy = dyb - (float)(8 * (k / PW));
        // the conic is positive definite, so the exponent (before log2 o) is never above 0
        const float pw = fmaf(dx, fmaf(co.x, dx, co.y * dy), fmaf(co.z * dy, dy, co.w));
        const float a = fminf(kAlphaMax, __builtin_amdgcn_exp2f(pw));
        const bool ok = a >= thr[k];
        float wgt = ok ? a * T[k] : 0.f;
        T[k] -= wgt;  // updated in place: a pixel that stops here gets its transmittance back below
        bool take = ok;
        // only a pixel that passed the test can cross the stop: the others keep a transmittance at
        // or above it (a stopped pixel's is restored below, to within one rounding of the value
        // before its stop; were that under the stop, this branch would only repeat the restore)
        const bool stop = T[k] < kTStop;
        if (__builtin_expect(__ballot(stop) != 0, 0)) {  // uniform: a pixel of the quadrant stops here
          // T - w + w: the transmittance before this entry up to one rounding
          T[k] = stop ? T[k] + wgt : T[k];
          wgt = stop ? 0.f : wgt;
          take = ok && !stop;
          if (COUNT) n_eval += thr[k] < 1.f ? 1u : 0u;
          thr[k] = stop ? kNever : thr[k];
          if (__ballot(thr[k] < 1.f) == 0) qalive &= ~(1u << k);
        } else if (COUNT) {
          n_eval += thr[k] < 1.f ? 1u : 0u;
        }
        if (COUNT) n_blend += take ? 1u : 0u;
        c0[k] = fmaf(c.x, wgt, c0[k]);
        c1[k] = fmaf(c.y, wgt, c1[k]);
        c2[k] = fmaf(c.z, wgt, c2[k]);
        last[k] = take ? wv : last[k];
      }
    }
    bool alive = false;
#pragma unroll
    for (int k = 0; k < NP; k++) alive = alive || thr[k] < 1.f;
    if (__ballot(alive) == 0) break;
    __syncthreads();
  }
  float l1sum = 0.f;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int px = ox + qx + 8 * (k % PW), py = oy + qy + 8 * (k / PW);
    if (px < V.W && py < V.H) {
      const int64_t hw = (int64_t)V.W * V.H;
      const int64_t pix = (int64_t)py * V.W + px;
      const float col[3] = {c0[k] + T[k] * bg0, c1[k] + T[k] * bg1, c2[k] + T[k] * bg2};
      if (!L1 || V.rgb) {
#pragma unroll
        for (int c = 0; c < 3; c++) V.rgb[c * hw + pix] = col[c];
      }
      V.t_final[pix] = T[k];
      V.n_contrib[pix] = (int)(last[k] & kPosMask);
      if (L1) {
        const float sc = V.l1_scale;
        float e = 0.f;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const float d = col[c] - V.target[c * hw + pix];
          V.dl_out[c * hw + pix] = d > 0.f ? sc : (d < 0.f ? -sc : 0.f);
          e += fabsf(d);
        }
        if (V.err) V.err[pix] = e * (1.0f / 3.0f);
        l1sum += e;
      }
    }
  }
  if (L1) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) l1sum += __shfl_xor(l1sum, d, 64);
    if (lane == 0) atomicAdd(&loss_slots[lb % kLossSlots], l1sum * V.l1_scale);
  }
  if (COUNT) {
    atomicAdd(&pairs[0], (unsigned long long)n_eval);
    atomicAdd(&pairs[1], (unsigned long long)n_blend);
  }
}

template <int SUB, int B>
__global__ __launch_bounds__(kLanes) void k_blend_bwd(ViewsIO io, int nv, int total_blocks, int per, float bg0,
                                                      float bg1, float bg2, const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals, const Rec* __restrict__ rec,
                                                      float* __restrict__ g2d) {
  constexpr int PW = SUB / 8, NP = PW * PW;  // quadrants per edge, pixels per lane
  __shared__ BwdStage s_st[B];
  const int lb = xcd_logical(blockIdx.x, per);
  if (lb >= total_blocks) return;
  const int b = lb / io.sn, sub = lb - b * io.sn;  // tile, SUB x SUB sub-tile of it
  const int v = view_of(io, nv, b);
  const ViewIO& V = io.v[v];
  const int t = b - V.tile_base;
  const int tx = t % V.TX, ty = t / V.TX;
  const int ox = tx * io.tw + (sub % io.sx) * SUB, oy = ty * io.th + (sub / io.sx) * SUB;
  if (ox >= V.W || oy >= V.H) return;  // sub-tile entirely outside the image
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const float fx0 = (float)ox, fy0 = (float)oy;
  const uint64_t lt = lane_lt_mask(lane);
  const uint2 r = ranges[b];
  if (r.y - r.x > (uint32_t)kPosMask) return;  // the forward reported it
  const int64_t hw = (int64_t)V.W * V.H;
  // per pixel: transmittance, dL/d(pixel colour), nS = -dL/dC . (colour blended behind the
  // current entry, background included)
  float T[NP], dC0[NP], dC1[NP], dC2[NP], nS[NP];
  int last[NP];
  int qlast[NP];  // per quadrant: the largest n_contrib of its pixels (uniform)
  int max_all = 0;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int px = ox + qx + 8 * (k % PW), py = oy + qy + 8 * (k / PW);
    T[k] = 1.f;
    dC0[k] = dC1[k] = dC2[k] = 0.f;
    last[k] = 0;
    if (px < V.W && py < V.H) {
      const int64_t pix = (int64_t)py * V.W + px;
      T[k] = V.t_final[pix];
      last[k] = V.n_contrib[pix];
      dC0[k] = V.dl[pix];
      dC1[k] = V.dl[hw + pix];
      dC2[k] = V.dl[2 * hw + pix];
    }
    nS[k] = -(bg0 * dC0[k] + bg1 * dC1[k] + bg2 * dC2[k]);
    int mx = last[k];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
    qlast[k] = __builtin_amdgcn_readfirstlane(mx);
    max_all = max(max_all, qlast[k]);
  }
  const int max_last = min(max_all, (int)(r.y - r.x));  // n_contrib never exceeds the list length
  if (max_last <= 0) return;
  const int slot = kRedSlot[lane >> 2];
  const bool writes = (lane & 3) == 0 && slot >= 0;
  const int nbatch = (max_last + B - 1) / B;
  for (int bi = nbatch - 1; bi >= 0; bi--) {
    const uint32_t start = r.x + (uint32_t)bi * B;
    const int n_in = min(B, max_last - bi * B);
    __syncthreads();
    int n_kept = 0;
#pragma unroll
    for (int k = 0; k < B / kLanes; k++) {
      const int e = k * kLanes + lane;
      uint32_t qm = 0;
      float2 xy;
      float4 cn, rgb;
      uint32_t p = 0;
      if (e < n_in) {
        p = vals[start + e];
        const Rec R = rec[p];
        xy = make_float2((R.r0.x - fx0) + R.r0.z, (R.r0.y - fy0) + R.r0.w);
        cn = R.r1;
        qm = quad_mask<PW>(xy.x, xy.y, cn.x, cn.y, cn.z, cn.w);
        // and only the quadrants where some pixel's last contribution is at or after the entry
        // (a compare per lane and quadrant here instead of a scalar test per entry and quadrant
        // in the walk; an entry left with none is not staged)
#pragma unroll
        for (int k = 0; k < NP; k++)
          if (bi * B + e >= qlast[k]) qm &= ~(1u << k);
        const uint32_t cb = cn.w >= kAlphaMax ? kClampBit : 0u;  // as the forward's
        rgb = make_float4(R.r2.x, R.r2.y, R.r2.z, __uint_as_float((uint32_t)(bi * B + e) | cb | (qm << kQmShift)));
      }
      const bool keep = qm != 0;
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int pos = n_kept + __popcll(m & lt);
        s_st[pos].co = make_float4(-0.5f * kLog2e * cn.x, -kLog2e * cn.y, -0.5f * kLog2e * cn.z, __log2f(cn.w));
        s_st[pos].rgb = rgb;
        s_st[pos].xy = xy;
        s_st[pos].p = p;
        s_st[pos].io = 1.0f / cn.w;
      }
      n_kept += __popcll(m);
    }
    __syncthreads();
    for (int j = n_kept - 1; j >= 0; j--) {
      const float2 xy = s_st[j].xy;
      const float4 co = s_st[j].co;
      const float4 c = s_st[j].rgb;
      const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_int(c.w));  // same for all lanes
      const int idx = (int)(w & kPosMask);
      const uint32_t qm = w >> kQmShift;
      const float dxb = xy.x - (float)qx, dyb = xy.y - (float)qy;
      // per-lane sums over its pixels: m = (sum dP dx, sum dP dy, sum dP dx^2, sum dP dx dy,
      // sum dP dy^2, d opacity (times the opacity until the reduction), d rgb),
      // dP = dL/d(exponent), (dx, dy) = mean - pixel
      float m[9];
#pragma unroll
      for (int q = 0; q < 9; q++) m[q] = 0.f;
      bool any = false;
      const bool clampable = (w & kClampBit) != 0;  // uniform
#pragma unroll
      for (int k = 0; k < NP; k++) {
        // uniform: the entry misses quadrant k, or lies behind the last contribution of every
        // pixel there (both folded into the staged mask)
        if (NP > 1 && !((qm >> k) & 1u)) continue;
        const float dx = dxb - (float)(8 * (k % PW)), dy = dyb - (float)(8 * (k / PW));
        const float pw = fmaf(dx, fmaf(co.x, dx, co.y * dy), fmaf(co.z * dy, dy, co.w));  // + log2 o
        const float araw = __builtin_amdgcn_exp2f(pw);
        const float a = fminf(kAlphaMax, araw);
        const bool take = (idx < last[k]) && (a >= kAlphaMin);  // the forward blended this entry here
        if (__ballot(take) == 0) continue;  // uniform
        any = true;
        // branch-free over the lanes: a pixel that did not blend the entry sees alpha 0, which
        // leaves its transmittance and colour-behind unchanged and adds nothing
        const float ae = take ? a : 0.f;
        T[k] = T[k] * __builtin_amdgcn_rcpf(1.f - ae);  // transmittance before this entry
        const float wgt = ae * T[k];
        m[6] = fmaf(wgt, dC0[k], m[6]);
        m[7] = fmaf(wgt, dC1[k], m[7]);
        m[8] = fmaf(wgt, dC2[k], m[8]);
        // dL/d alpha = T (dL/dC . (colour - colour behind)); the colour behind moves by alpha of that
        const float ed = fmaf(c.x, dC0[k], fmaf(c.y, dC1[k], fmaf(c.z, dC2[k], nS[k])));
        nS[k] = fmaf(-ae, ed, nS[k]);
        // dP = alpha dL/d alpha = alpha T ed: dL/d(exponent), and the opacity times dL/d(opacity)
        float dP = wgt * ed;
        if (__builtin_expect(clampable, 0)) {
          __asm__ volatile("");  // keeps this rarely taken uniform branch a branch
          dP = araw < kAlphaMax ? dP : 0.f;  // no derivative through an active clamp
        }
        m[5] += dP;  // d alpha / d o = alpha / o, the 1 / o applied once per entry
        const float pdx = dP * dx, pdy = dP * dy;
        m[0] += pdx;
        m[1] += pdy;
        m[2] = fmaf(pdx, dx, m[2]);
        m[3] = fmaf(pdx, dy, m[3]);
        m[4] = fmaf(pdy, dy, m[4]);
      }
      if (any) {  // uniform
        // the sums are linear in the entry's conic, so the conic is applied once per
        // (view, Gaussian) by the projection adjoint, not here
        m[5] *= s_st[j].io;
        const float tot = wave_reduce9(m);
        if (writes) atomicAdd(&g2d[(int64_t)s_st[j].p * 9 + slot], tot);
      }
    }
  }
}

// Identity-feature render: the forward's walk (same lists, culling, alpha, transmittance and
// stop, so the weights alpha_i T_i are the colour render's) accumulating up to kFeatMaxC
// per-Gaussian features instead of colours, with no background.
template <int SUB, int B>
__global__ __launch_bounds__(kLanes) void k_blend_feat(ViewsIO io, int nv, int total_blocks, int per, FeatIO fo,
                                                       const uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ vals, const Rec* __restrict__ rec) {
  constexpr int PW = SUB / 8, NP = PW * PW;
  __shared__ float2 s_xy[B];
  __shared__ float4 s_co[B];
  __shared__ uint32_t s_qm[B];
  __shared__ float4 s_f[B][kFeatMaxC / 4];
  const int lb = xcd_logical(blockIdx.x, per);
  if (lb >= total_blocks) return;
  const int b = lb / io.sn, sub = lb - b * io.sn;
  const int v = view_of(io, nv, b);
  const ViewIO& V = io.v[v];
  const int t = b - V.tile_base;
  const int tx = t % V.TX, ty = t / V.TX;
  const int ox = tx * io.tw + (sub % io.sx) * SUB, oy = ty * io.th + (sub / io.sx) * SUB;
  if (ox >= V.W || oy >= V.H) return;
  const int lane = threadIdx.x;
  const int qx = lane & 7, qy = lane >> 3;
  const float fx0 = (float)ox, fy0 = (float)oy;
  const uint64_t lt = lane_lt_mask(lane);
  const uint2 r = ranges[b];
  if (r.y - r.x > (uint32_t)kPosMask) return;  // the colour forward reported it
  const uint32_t gbase = (uint32_t)v * (uint32_t)fo.n;  // record index = view * n + Gaussian
  float T[NP], thr[NP], acc[NP][kFeatMaxC];  // thr: as the colour forward's
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int px = ox + qx + 8 * (k % PW), py = oy + qy + 8 * (k / PW);
    T[k] = 1.f;
    thr[k] = (px < V.W && py < V.H) ? kAlphaMin : kNever;
#pragma unroll
    for (int c = 0; c < kFeatMaxC; c++) acc[k][c] = 0.f;
  }
  for (uint32_t start = r.x; start < r.y; start += B) {
    const int n_in = (int)min((uint32_t)B, r.y - start);
    int n_kept = 0;
#pragma unroll
    for (int k = 0; k < B / kLanes; k++) {
      const int e = k * kLanes + lane;
      uint32_t qm = 0, rid = 0;
      float2 xy;
      float4 co;
      if (e < n_in) {
        rid = vals[start + e];
        const Rec R = rec[rid];
        xy = make_float2((R.r0.x - fx0) + R.r0.z, (R.r0.y - fy0) + R.r0.w);
        qm = quad_mask<PW>(xy.x, xy.y, R.r1.x, R.r1.y, R.r1.z, R.r1.w);
        co = make_float4(-0.5f * kLog2e * R.r1.x, -kLog2e * R.r1.y, -0.5f * kLog2e * R.r1.z, __log2f(R.r1.w));
      }
      const bool keep = qm != 0;
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int pos = n_kept + __popcll(m & lt);
        s_xy[pos] = xy;
        s_co[pos] = co;
        s_qm[pos] = qm;
        // Gaussian-major copy: one 64-byte row per entry
        const float4* __restrict__ f = reinterpret_cast<const float4*>(fo.feat16) + (size_t)(rid - gbase) * (kFeatMaxC / 4);
#pragma unroll
        for (int c = 0; c < kFeatMaxC / 4; c++) s_f[pos][c] = f[c];
      }
      n_kept += __popcll(m);
    }
    uint32_t qalive = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) qalive |= __ballot(thr[k] < 1.f) != 0 ? 1u << k : 0u;
    __syncthreads();
    for (int j = 0; j < n_kept && qalive != 0; j++) {
      const float2 xy = s_xy[j];
      const float4 co = s_co[j];
      const uint32_t qm = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_qm[j]) & qalive;
      const float dxb = xy.x - (float)qx, dyb = xy.y - (float)qy;
      float4 fe[kFeatMaxC / 4];
#pragma unroll
      for (int c = 0; c < kFeatMaxC / 4; c++) fe[c] = s_f[j][c];
#pragma unroll
      for (int k = 0; k < NP; k++) {
        if (NP > 1 && !((qm >> k) & 1u)) continue;
        const float dx = dxb - (float)(8 * (k % PW)), dy = dyb - (float)(8 * (k / PW));
        // the colour forward's alpha, weight and stop, operation for operation
        const float pw = fmaf(dx, fmaf(co.x, dx, co.y * dy), fmaf(co.z * dy, dy, co.w));
        const float a = fminf(kAlphaMax, __builtin_amdgcn_exp2f(pw));
        const bool ok = a >= thr[k];
        float wgt = ok ? a * T[k] : 0.f;
        T[k] -= wgt;
        const bool stop = T[k] < kTStop;  // as the colour forward's: only a passing pixel can cross it
        if (__builtin_expect(__ballot(stop) != 0, 0)) {  // uniform: a pixel of the quadrant stops here
          T[k] = stop ? T[k] + wgt : T[k];
          wgt = stop ? 0.f : wgt;
          thr[k] = stop ? kNever : thr[k];
          if (__ballot(thr[k] < 1.f) == 0) qalive &= ~(1u << k);
        }
#pragma unroll
        for (int c = 0; c < kFeatMaxC / 4; c++) {
          acc[k][4 * c] += fe[c].x * wgt;
          acc[k][4 * c + 1] += fe[c].y * wgt;
          acc[k][4 * c + 2] += fe[c].z * wgt;
          acc[k][4 * c + 3] += fe[c].w * wgt;
        }
      }
    }
    bool alive = false;
#pragma unroll
    for (int k = 0; k < NP; k++) alive = alive || thr[k] < 1.f;
    if (__ballot(alive) == 0) break;
    __syncthreads();
  }
  float* __restrict__ out = fo.out[v];
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int px = ox + qx + 8 * (k % PW), py = oy + qy + 8 * (k / PW);
    if (px < V.W && py < V.H) {
      const int64_t hw = (int64_t)V.W * V.H;
      const int64_t pix = (int64_t)py * V.W + px;
#pragma unroll
      for (int c = 0; c < kFeatMaxC; c++)
        if (c < fo.C) out[c * hw + pix] = acc[k][c];
    }
  }
}

__global__ void k_debug_keys(uint32_t key_base, uint32_t row0, const uint32_t* __restrict__ keys,
                             const uint32_t* __restrict__ vals, const Rec* __restrict__ rec, uint32_t lo,
                             uint32_t cnt, uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t k = keys[lo + i];
  const uint32_t p = vals[lo + i];  // record index of the view's Gaussian
  kout[i] = ((uint64_t)(k - key_base) << 32) | (uint64_t)__float_as_uint(rec[p].r2.w);
  vout[i] = p - row0;
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
  k_gather_sorted<<<(unsigned)((vn + 255) / 256), 256, 0, st>>>(n, vn, sorted_gid, ws.rect_u, ws.tt_s,
                                                                 ws.rect_s);
}

void launch_emit_keys(int n, int64_t vn, const CamsK& cams, Workspace& ws, hipStream_t st) {
  scan_u32_to_u64(ws.tt_s, ws.off_s, vn, ws.scan_tmp, st);
  if (vn > 0)
    k_emit_keys<<<(unsigned)((vn + 255) / 256), 256, 0, st>>>(n, vn, cams, ws.tt_s, ws.rect_s, ws.gid_s, ws.off_s,
                                                               ws.cap_keys, ws.keys[0], ws.vals[0], ws.err);
  k_clamp_count<<<1, 1, 0, st>>>(ws.off_s + vn, ws.cap_keys, ws.counters);
}

void launch_ranges(const uint32_t* keys, int64_t total_tiles, const CamsK& cams, int nv, Workspace& ws,
                   hipStream_t st) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(ws.ranges), 0u, 2 * total_tiles, st);
  KeyTiles kt{};
  for (int v = 0; v < nv; v++) kt.tile_base[v] = cams.c[v].tile_base;
  kt.local_bits = cams.local_bits;
  kt.nv = nv;
  kt.total_tiles = (uint32_t)total_tiles;
  int64_t blocks = (ws.cap_keys + 1023) / 1024;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  k_ranges<<<(unsigned)blocks, 256, 0, st>>>(keys, ws.counters, kt, ws.ranges);
}

static inline int per_xcd(int64_t total_tiles) { return (int)((total_tiles + kNumXcd - 1) / kNumXcd); }

// One wave per (tile, sub-tile); the sub-tiles of a tile are consecutive logical blocks, so they
// run on the same XCD and share its L2 for the tile's list and records.
template <bool COUNT, bool L1, int B>
void blend_fwd_batch(const ViewsIO& io, int nv, int total, int per, const float bg[3], const Workspace& ws,
                     const uint32_t* vals, hipStream_t st) {
  const dim3 grid(per * kNumXcd), block(kLanes);
  if (io.sub == 8)
    k_blend_fwd<COUNT, L1, 8, B><<<grid, block, 0, st>>>(io, nv, total, per, bg[0], bg[1], bg[2], ws.ranges, vals,
                                                        ws.rec_u, ws.pairs, ws.loss_slots);
  else
    k_blend_fwd<COUNT, L1, 16, B><<<grid, block, 0, st>>>(io, nv, total, per, bg[0], bg[1], bg[2], ws.ranges, vals,
                                                         ws.rec_u, ws.pairs, ws.loss_slots);
}

template <bool COUNT, bool L1>
void blend_fwd_variant(const ViewsIO& io, int nv, int total, int per, const float bg[3], const Workspace& ws,
                       const uint32_t* vals, hipStream_t st) {
  if (io.batch == 64)
    blend_fwd_batch<COUNT, L1, 64>(io, nv, total, per, bg, ws, vals, st);
  else if (io.batch == 256)
    blend_fwd_batch<COUNT, L1, 256>(io, nv, total, per, bg, ws, vals, st);
  else
    blend_fwd_batch<COUNT, L1, 128>(io, nv, total, per, bg, ws, vals, st);
}

void launch_blend_fwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3], const Workspace& ws,
                      const uint32_t* vals, bool count_pairs, bool l1, hipStream_t st) {
  const int64_t total = total_tiles * io.sn;
  if (total == 0) return;
  const int per = per_xcd(total);
  ViewsIO iov = io;
  iov.err = ws.err;
  if (count_pairs) {
    if (l1)
      blend_fwd_variant<true, true>(iov, nv, (int)total, per, bg, ws, vals, st);
    else
      blend_fwd_variant<true, false>(iov, nv, (int)total, per, bg, ws, vals, st);
  } else {
    if (l1)
      blend_fwd_variant<false, true>(iov, nv, (int)total, per, bg, ws, vals, st);
    else
      blend_fwd_variant<false, false>(iov, nv, (int)total, per, bg, ws, vals, st);
  }
}

// features [C][stride] -> Gaussian-major rows of kFeatMaxC floats (zeros beyond C)
__global__ __launch_bounds__(256) void k_feat_rows(const float* __restrict__ feat, int64_t stride, int C, int n,
                                                   float4* __restrict__ rows) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= n) return;
  float v[kFeatMaxC];
#pragma unroll
  for (int c = 0; c < kFeatMaxC; c++) v[c] = c < C ? feat[c * stride + g] : 0.f;
#pragma unroll
  for (int c = 0; c < kFeatMaxC / 4; c++)
    rows[(size_t)g * (kFeatMaxC / 4) + c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}

void launch_blend_feat(const ViewsIO& io, int nv, int64_t total_tiles, const FeatIO& fo, const Workspace& ws,
                       const uint32_t* vals, hipStream_t st) {
  if (fo.n > 0)
    k_feat_rows<<<(fo.n + 255) / 256, 256, 0, st>>>(fo.feat, fo.stride, fo.C, fo.n, reinterpret_cast<float4*>(fo.feat16));
  const int64_t total = total_tiles * io.sn;
  if (total == 0) return;
  const int per = per_xcd(total);
  const dim3 grid(per * kNumXcd), block(kLanes);
#define DASS_FEAT(SUBT, BT) k_blend_feat<SUBT, BT><<<grid, block, 0, st>>>(io, nv, (int)total, per, fo, ws.ranges, vals, ws.rec_u)
  if (io.sub == 8) {
    if (io.batch == 64) DASS_FEAT(8, 64);
    else if (io.batch == 256) DASS_FEAT(8, 256);
    else DASS_FEAT(8, 128);
  } else {
    if (io.batch == 64) DASS_FEAT(16, 64);
    else if (io.batch == 256) DASS_FEAT(16, 256);
    else DASS_FEAT(16, 128);
  }
#undef DASS_FEAT
}

__global__ __launch_bounds__(256) void k_loss_finish(float* __restrict__ slots, float* __restrict__ loss, float add) {
  __shared__ float s_w[4];
  float acc = 0.f;
  for (int i = threadIdx.x; i < kLossSlots; i += 256) {
    acc += slots[i];
    slots[i] = 0.f;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) *loss += ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) + add;
}

void launch_loss_finish(float* slots, float* loss, float add, hipStream_t st) {
  k_loss_finish<<<1, 256, 0, st>>>(slots, loss, add);
}

void launch_blend_bwd(const ViewsIO& io, int nv, int64_t total_tiles, const float bg[3], const Workspace& ws,
                      const uint32_t* vals, int n, hipStream_t st) {
  const int64_t total = total_tiles * io.sn;
  if (total == 0) return;
  const int per = per_xcd(total);
  const dim3 grid(per * kNumXcd), block(kLanes);
#define DASS_BWD(SUBT, BT)                                                                                     \
  k_blend_bwd<SUBT, BT><<<grid, block, 0, st>>>(io, nv, (int)total, per, bg[0], bg[1], bg[2], ws.ranges, vals, \
                                                ws.rec_u, ws.g2d)
  if (io.sub == 8) {
    if (io.batch == 64) DASS_BWD(8, 64);
    else if (io.batch == 256) DASS_BWD(8, 256);
    else DASS_BWD(8, 128);
  } else {
    if (io.batch == 64) DASS_BWD(16, 64);
    else if (io.batch == 256) DASS_BWD(16, 256);
    else DASS_BWD(16, 128);
  }
#undef DASS_BWD
}

void launch_debug_keys(int view, int n, const Workspace& ws, const uint32_t* keys_sorted, const uint32_t* vals_sorted,
                       uint32_t lo, uint32_t cnt, const CamK& cam, uint64_t* kout, uint32_t* vout, hipStream_t st) {
  if (cnt > 0)
    k_debug_keys<<<(cnt + 255) / 256, 256, 0, st>>>(cam.key_base, (uint32_t)((int64_t)view * n), keys_sorted,
                                                     vals_sorted, ws.rec_u, lo, cnt, kout, vout);
}

}  // namespace dass
