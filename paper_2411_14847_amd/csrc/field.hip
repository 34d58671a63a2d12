// Hash-encoded deformation fields H_dyn / H_st (Sec. 3.3; table sizes in App. B): a
// multi-resolution hash encoding of a Gaussian's normalised position followed by an MLP with
// one ReLU hidden layer and seven outputs, the position offset (3) and the rotation offset (4,
// added to the identity quaternion).
//
// Forward: a quad of lanes per query (lane s encodes the levels l = s mod 4 and takes the hidden
// units h = s mod 4; DPP quad permutations complete the encoding and add the partial outputs), the
// MLP weights staged in LDS.
// Backward:
//  1. a quad of lanes per query, as the forward: the encoding and the MLP adjoint are recomputed
//     and the rows the gradients need (per hidden unit dL/d(pre-activation) and activation, the
//     encoding and its adjoint, the upstream gradient, the float64 position) go to a workspace,
//     feature-major.
//  2. weight gradients: each workgroup sums a contiguous part of the queries through LDS and
//     writes one partial row; the partials are then added in a fixed order.
//  3. table gradients without global atomics: each workgroup owns one slice (up to 128 KB) of
//     one level's table, accumulates every query's corner contributions that fall in it with
//     LDS atomics, then adds the slice to the gradient.  (Float atomics to global memory from
//     every query -- L x 8 x F per query -- ran at ~1.5e10 per second here, and many queries hit
//     the same rows of the coarse levels.)
#include <algorithm>

#include "dass_internal.h"

namespace dass {
namespace {

constexpr uint32_t kPrimeY = 2654435761u;  // the encoding's spatial-hash primes (x: 1)
constexpr uint32_t kPrimeZ = 805459861u;
constexpr int kSliceFloats = 32768;  // table-gradient slice held in LDS (128 KB)
constexpr int kSliceThreads = 1024;
constexpr int kSliceTargetBlocks = 512;
constexpr int kSliceBatch = 4;

template <int F>
constexpr int max_levels() { return (64 / F) < kFieldMaxLevels ? 64 / F : kFieldMaxLevels; }

template <int F>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float* v) {
  if constexpr (F == 1) {
    v[0] = p[0];
  } else if constexpr (F == 2) {
    const float2 a = *reinterpret_cast<const float2*>(p);
    v[0] = a.x;
    v[1] = a.y;
  } else {
#pragma unroll
    for (int i = 0; i < F; i += 4) {
      const float4 a = *reinterpret_cast<const float4*>(p + i);
      v[i] = a.x;
      v[i + 1] = a.y;
      v[i + 2] = a.z;
      v[i + 3] = a.w;
    }
  }
}

// The position in the box in float64: at the finest levels (N ~ 2^11) float32 rounding of the
// normalisation would move a query by ~1e-4 cells and decide some cells differently.
__device__ __forceinline__ void normalised(const FieldK& f, const QueryK& q, int g, double p[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = ((double)q.mean[d * q.stride + g] - f.lo[d]) / f.ext[d];
    p[d] = fmin(fmax(x, 0.0), 1.0);  // NaN -> 0
  }
}

// Calls fn(corner, row of the level's table, trilinear weight) for the 8 corners of level l's
// cell around p.
template <class Fn>
__device__ __forceinline__ void level_corners(const FieldK& f, int l, const double p[3], Fn&& fn) {
  const int N = f.res[l];
  int c[3];
  float fr[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = p[d] * (double)N;
    c[d] = min((int)floor(x), N - 1);
    fr[d] = (float)(x - (double)c[d]);
  }
  const bool dense = (f.dense >> l) & 1u;
  const uint32_t mask = (1u << f.log2T) - 1u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t x = (uint32_t)(c[0] + (k & 1)), y = (uint32_t)(c[1] + ((k >> 1) & 1)),
                   z = (uint32_t)(c[2] + ((k >> 2) & 1));
    const uint32_t row = dense ? x + (uint32_t)(N + 1) * (y + (uint32_t)(N + 1) * z)
                               : (x ^ (y * kPrimeY) ^ (z * kPrimeZ)) & mask;
    const float w = ((k & 1) ? fr[0] : 1.f - fr[0]) * ((k & 2) ? fr[1] : 1.f - fr[1]) *
                    ((k & 4) ? fr[2] : 1.f - fr[2]);
    fn(k, row, w);
  }
}

// ---- four lanes per query -------------------------------------------------------------------
// A quad of lanes shares a query: lane s encodes the levels l = s (mod 4) and takes the hidden
// units h = s (mod 4); the encoding is completed and the partial sums combined with DPP quad
// permutations.  Four times the waves of one lane per query, a quarter of the chain each, for the
// latency-bound small calls (the dynamic group's field queries a tenth of the Gaussians).
constexpr int kQuadThreads = 256;  // 64 queries per workgroup

template <int CTRL>
__device__ __forceinline__ float qdpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_sum(float x) {
  x += qdpp<0xB1>(x);  // quad_perm [1, 0, 3, 2]
  x += qdpp<0x4E>(x);  // quad_perm [2, 3, 0, 1]
  return x;
}
template <int K>
__device__ __forceinline__ float quad_bcast(float x) {
  return qdpp<K * 0x55>(x);  // quad_perm [K, K, K, K]
}

// MLP weights in LDS: w1 rows padded to LFM + 4 floats (zeros beyond L F), so the quad's four
// rows h = 4u + s fall in different banks
template <int F, int HID>
struct QuadW {
  static constexpr int LFM = max_levels<F>() * F, LS = LFM + 4;
  float4 w1[HID * LS / 4];
  float w2[7][HID];
  float b1[HID];
};

template <int F, int HID>
__device__ __forceinline__ void stage_weights(const FieldK& f, QuadW<F, HID>& s) {
  constexpr int LFM = QuadW<F, HID>::LFM, LS = QuadW<F, HID>::LS;
  const int LF = f.L * F;
  float* w1 = reinterpret_cast<float*>(s.w1);
  for (int e = threadIdx.x; e < HID * LS; e += kQuadThreads) {
    const int h = e / LS, k = e % LS;
    w1[e] = k < LF ? f.w1[h * LF + k] : 0.f;
  }
  for (int e = threadIdx.x; e < 7 * HID; e += kQuadThreads) s.w2[e / HID][e % HID] = f.w2[e];
  for (int e = threadIdx.x; e < HID; e += kQuadThreads) s.b1[e] = f.b1[e];
  (void)LFM;
  __syncthreads();
}

// This lane's levels (l = sub + 4 r) of the encoding, then the whole encoding in every lane of the quad.
template <int F>
__device__ __forceinline__ void quad_encode(const FieldK& f, const double p[3], int sub, float* mine, float* enc) {
  constexpr int KL = max_levels<F>(), KLQ = (KL + 3) / 4;
#pragma unroll
  for (int r = 0; r < KLQ; ++r) {
    const int l = sub + 4 * r;
#pragma unroll
    for (int i = 0; i < F; ++i) mine[r * F + i] = 0.f;
    if (l < f.L && l < KL) {
      const size_t base = (size_t)l << f.log2T;
      level_corners(f, l, p, [&](int, uint32_t row, float w) {
        float v[F];
        load_row<F>(f.table + (base + row) * F, v);
#pragma unroll
        for (int i = 0; i < F; ++i) mine[r * F + i] = fmaf(w, v[i], mine[r * F + i]);
      });
    }
  }
#pragma unroll
  for (int l = 0; l < KL; ++l) {
#pragma unroll
    for (int i = 0; i < F; ++i) {
      const float x = mine[(l >> 2) * F + i];
      float y;
      switch (l & 3) {
        case 0: y = quad_bcast<0>(x); break;
        case 1: y = quad_bcast<1>(x); break;
        case 2: y = quad_bcast<2>(x); break;
        default: y = quad_bcast<3>(x); break;
      }
      enc[l * F + i] = y;
    }
  }
}

template <int F, int HID>
__device__ __forceinline__ float quad_pre(const QuadW<F, HID>& s, int h, const float* enc) {
  constexpr int LFM = QuadW<F, HID>::LFM, LS = QuadW<F, HID>::LS;
  float a = s.b1[h];
#pragma unroll
  for (int c = 0; c < LFM / 4; ++c) {
    const float4 w = s.w1[(h * LS) / 4 + c];
    a = fmaf(w.x, enc[4 * c], a);
    a = fmaf(w.y, enc[4 * c + 1], a);
    a = fmaf(w.z, enc[4 * c + 2], a);
    a = fmaf(w.w, enc[4 * c + 3], a);
  }
  return a;
}

template <int F, int HID>
__global__ __launch_bounds__(kQuadThreads) void k_field_fwd4(const FieldK f, const QueryK q, float* __restrict__ dpos,
                                                            float* __restrict__ drot) {
  constexpr int KL = max_levels<F>(), LFM = KL * F, KLQ = (KL + 3) / 4;
  __shared__ QuadW<F, HID> s;
  stage_weights<F, HID>(f, s);
  const int sub = threadIdx.x & 3;
  const int j = blockIdx.x * (kQuadThreads / 4) + (threadIdx.x >> 2);
  if (j >= q.m) return;  // the whole quad
  int g = q.idx ? q.idx[j] : j;
  const bool valid = g >= 0 && g < q.n;
  float out[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    double p[3];
    normalised(f, q, g, p);
    float mine[KLQ * F], enc[LFM];
    quad_encode<F>(f, p, sub, mine, enc);
#pragma unroll
    for (int u = 0; u < HID / 4; ++u) {
      const int h = 4 * u + sub;
      const float a = fmaxf(quad_pre<F, HID>(s, h, enc), 0.f);
#pragma unroll
      for (int o = 0; o < 7; ++o) out[o] = fmaf(s.w2[o][h], a, out[o]);
    }
#pragma unroll
    for (int o = 0; o < 7; ++o) out[o] = quad_sum(out[o]);
#pragma unroll
    for (int o = 0; o < 7; ++o) out[o] += f.b2[o];
  }
  if (sub != 0) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) dpos[d * q.ld + j] = out[d];
  drot[j] = 1.f + out[3];
#pragma unroll
  for (int d = 1; d < 4; ++d) drot[d * q.ld + j] = out[3 + d];
}

// Backward per query with a quad per query: writes, feature-major over the queries, what the weight
// and table gradients need -- dL/d(pre-activation) and the activation of every hidden unit (by the
// lane that owns the unit), the encoding and its adjoint (by the lane that owns the level), the
// upstream gradient (zeros for rows outside [0, n)) and the float64 normalised position.
template <int F, int HID>
__global__ __launch_bounds__(kQuadThreads) void k_field_bwd_query4(const FieldK f, const QueryK q,
                                                                  const float* __restrict__ d_dpos,
                                                                  const float* __restrict__ d_drot, FieldRows rows) {
  constexpr int KL = max_levels<F>(), LFM = KL * F, KLQ = (KL + 3) / 4;
  constexpr int LS = QuadW<F, HID>::LS;
  __shared__ QuadW<F, HID> s;
  stage_weights<F, HID>(f, s);
  const int sub = threadIdx.x & 3;
  const int j = blockIdx.x * (kQuadThreads / 4) + (threadIdx.x >> 2);
  if (j >= q.m) return;
  const int64_t m = q.m;
  int g = q.idx ? q.idx[j] : j;
  if (g < 0 || g >= q.n) g = -1;
  double p[3] = {0.0, 0.0, 0.0};
  float dout[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float mine[KLQ * F], enc[LFM];
#pragma unroll
  for (int i = 0; i < KLQ * F; ++i) mine[i] = 0.f;
#pragma unroll
  for (int i = 0; i < LFM; ++i) enc[i] = 0.f;
  if (g >= 0) {
    normalised(f, q, g, p);
#pragma unroll
    for (int d = 0; d < 3; ++d) dout[d] = d_dpos[d * q.ld + j];
#pragma unroll
    for (int d = 0; d < 4; ++d) dout[3 + d] = d_drot[d * q.ld + j];
    quad_encode<F>(f, p, sub, mine, enc);
  }
  float denc[LFM];
#pragma unroll
  for (int i = 0; i < LFM; ++i) denc[i] = 0.f;
#pragma unroll
  for (int u = 0; u < HID / 4; ++u) {
    const int h = 4 * u + sub;
    const float a = quad_pre<F, HID>(s, h, enc);
    float dh = 0.f;
#pragma unroll
    for (int o = 0; o < 7; ++o) dh = fmaf(s.w2[o][h], dout[o], dh);
    const float dp = a > 0.f ? dh : 0.f;
    rows.dpre[h * m + j] = dp;
    rows.act[h * m + j] = fmaxf(a, 0.f);
#pragma unroll
    for (int c = 0; c < LFM / 4; ++c) {
      const float4 w = s.w1[(h * LS) / 4 + c];
      denc[4 * c] = fmaf(w.x, dp, denc[4 * c]);
      denc[4 * c + 1] = fmaf(w.y, dp, denc[4 * c + 1]);
      denc[4 * c + 2] = fmaf(w.z, dp, denc[4 * c + 2]);
      denc[4 * c + 3] = fmaf(w.w, dp, denc[4 * c + 3]);
    }
  }
#pragma unroll
  for (int i = 0; i < LFM; ++i) denc[i] = quad_sum(denc[i]);
#pragma unroll
  for (int l = 0; l < KL; ++l)
    if ((l & 3) == sub && l < f.L) {
#pragma unroll
      for (int i = 0; i < F; ++i) {
        rows.enc[(l * F + i) * m + j] = mine[(l >> 2) * F + i];
        rows.denc[(l * F + i) * m + j] = denc[l * F + i];
      }
    }
  if (sub == 0) {
#pragma unroll
    for (int o = 0; o < 7; ++o) rows.dout[o * m + j] = dout[o];
#pragma unroll
    for (int d = 0; d < 3; ++d) rows.pn[d * m + j] = p[d];
  }
}

// Weight gradients on the matrix cores: over a contiguous part of the queries, a workgroup forms
//   dW1 [HID][LF] = dpre [HID][q] . enc [LF][q]^T   and   dW2 [7][HID] = dout [7][q] . act [HID][q]^T
// with fp32 MFMA (v_mfma_f32_16x16x4f32: 16x16 output tiles, four queries per instruction), and
// the bias sums db1 = sum_q dpre, db2 = sum_q dout on the vector units beside them.  Queries
// are staged 64 at a time in LDS, feature-major as the rows are stored (row stride 66 floats:
// a tile operand's 16 rows x 4 queries land in 32 different banks); each thread prefetches its
// share of the next 64 queries into registers while the current ones are multiplied.  One
// partial row per workgroup, summed in a fixed order afterwards.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kWgThreads = 256;
constexpr int kWgQ = 64;        // queries per staged chunk
constexpr int kWgS = kWgQ + 2;  // LDS row stride (floats)

template <int F, int HID>
struct WgradShape {
  static constexpr int KL = max_levels<F>();
  static constexpr int LFM = KL * F;                     // encoding rows (a multiple of 16)
  static constexpr int R = 2 * HID + LFM + 8;            // staged rows: dpre, act, enc, dout (+1 zero)
  static constexpr int PER = (R * kWgQ) / kWgThreads;    // values each thread stages per chunk
  static constexpr int RT = HID / 16, CT = LFM / 16;     // dW1 tiles
  static constexpr int TILES = RT * CT + HID / 16;       // + dW2 tiles (7 rows padded to 16)
  static constexpr int TPW = (TILES + 3) / 4;            // tiles per wave
};

template <int F, int HID>
__global__ __launch_bounds__(kWgThreads) void k_field_wgrad(const FieldK f, int m, FieldRows rows,
                                                            float* __restrict__ part) {
  using S = WgradShape<F, HID>;
  static_assert(S::R * kWgQ % kWgThreads == 0, "staging split");
  static_assert(S::LFM % 16 == 0 && HID % 16 == 0, "tile split");
  __shared__ float s_v[S::R][kWgS];  // rows: dpre [HID], act [HID], enc [LFM], dout [8]
  __shared__ float s_b1[4][HID];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int LF = f.L * F;
  const int q0 = (int)((int64_t)m * blockIdx.x / gridDim.x), q1 = (int)((int64_t)m * (blockIdx.x + 1) / gridDim.x);
  // staging map: value i of this thread is row (t / kWgQ) + i * (kWgThreads / kWgQ), query t % kWgQ
  const int sc = t % kWgQ, sr = t / kWgQ;
  constexpr int RS = kWgThreads / kWgQ;  // rows apart of a thread's consecutive values
  float pre[S::PER];
  // value i: row sr + RS i of the stacked rows (dpre, act, enc padded to LFM, dout padded to 8)
  auto fetch = [&](int base) {
    const int q = base + sc;
    if (q >= q1) {
#pragma unroll
      for (int i = 0; i < S::PER; ++i) pre[i] = 0.f;
      return;
    }
    const int64_t step = (int64_t)RS * m;
    const float* pd = rows.dpre + (int64_t)sr * m + q;
    const float* pa = rows.act + (int64_t)sr * m + q;
    const float* pe = rows.enc + (int64_t)sr * m + q;
#pragma unroll
    for (int i = 0; i < HID / RS; ++i) pre[i] = pd[i * step];
#pragma unroll
    for (int i = 0; i < HID / RS; ++i) pre[HID / RS + i] = pa[i * step];
#pragma unroll
    for (int i = 0; i < S::LFM / RS; ++i) pre[2 * HID / RS + i] = (sr + RS * i) < LF ? pe[i * step] : 0.f;
#pragma unroll
    for (int i = 0; i < 8 / RS; ++i) {
      const int o = sr + RS * i;
      pre[(2 * HID + S::LFM) / RS + i] = o < 7 ? rows.dout[(int64_t)o * m + q] : 0.f;
    }
  };
  f32x4 acc[S::TPW];
#pragma unroll
  for (int k = 0; k < S::TPW; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float b1 = 0.f, b2 = 0.f;  // thread t: db1 of hidden unit t % HID over its quarter; db2 of o = t / 16
  const int i16 = lane & 15, k4 = lane >> 4;  // operand lane -> (tile row or column, query of 4)
  if (q0 < q1) fetch(q0);
  for (int base = q0; base < q1; base += kWgQ) {
#pragma unroll
    for (int i = 0; i < S::PER; ++i) s_v[sr + i * (kWgThreads / kWgQ)][sc] = pre[i];
    __syncthreads();
    if (base + kWgQ < q1) fetch(base + kWgQ);  // next chunk's loads in flight during the products
#pragma unroll
    for (int kq = 0; kq < kWgQ; kq += 4) {
#pragma unroll
      for (int k = 0; k < S::TPW; ++k) {
        const int tile = wave + 4 * k;
        if (tile >= S::TILES) break;
        float a, b;
        if (tile < S::RT * S::CT) {  // dW1 tile (row tile, column tile)
          const int rt = tile / S::CT, ct = tile % S::CT;
          a = s_v[rt * 16 + i16][kq + k4];                  // dpre[h][q]
          b = s_v[2 * HID + ct * 16 + i16][kq + k4];        // enc[k][q]
        } else {  // dW2 column tile: dout [7 -> 16 rows] x act
          const int ct = tile - S::RT * S::CT;
          a = s_v[2 * HID + S::LFM + (i16 < 8 ? i16 : 7)][kq + k4];  // row 7 of the dout block is zero
          a = i16 < 7 ? a : 0.f;
          b = s_v[HID + ct * 16 + i16][kq + k4];            // act[h][q]
        }
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
      }
    }
    // bias sums on the vector units
    if (t < 4 * HID) {
#pragma unroll 4
      for (int c = 0; c < kWgQ / 4; ++c) b1 += s_v[t % HID][(t / HID) * (kWgQ / 4) + c];
    }
    if (t < 7 * 16) {
#pragma unroll
      for (int c = 0; c < 4; ++c) b2 += s_v[2 * HID + S::LFM + t / 16][(t % 16) * 4 + c];
    }
    __syncthreads();
  }
  // partial row: [w1: HID][LF] [b1: HID] [w2: 7][HID] [b2: 7]
  float* P = part + (size_t)blockIdx.x * field_part_stride(HID, LF);
#pragma unroll
  for (int k = 0; k < S::TPW; ++k) {
    const int tile = wave + 4 * k;
    if (tile >= S::TILES) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * k4 + r, col = i16;  // D[row][col] of the tile
      if (tile < S::RT * S::CT) {
        const int h = (tile / S::CT) * 16 + row, kk = (tile % S::CT) * 16 + col;
        if (kk < LF) P[h * LF + kk] = acc[k][r];
      } else {
        const int h = (tile - S::RT * S::CT) * 16 + col;
        if (row < 7) P[HID * LF + HID + row * HID + h] = acc[k][r];
      }
    }
  }
  // db1: four quarters of the queries per hidden unit (HID * 4 <= 256 threads), added in order
  if (t < 4 * HID) s_b1[t / HID][t % HID] = b1;
  // db2: 16 consecutive lanes per output, summed across them in order
  float b2s = b2;
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) b2s += __shfl_xor(b2s, d, 64);
  __syncthreads();
  if (t < HID) P[HID * LF + t] = ((s_b1[0][t] + s_b1[1][t]) + s_b1[2][t]) + s_b1[3][t];
  if (t < 7 * 16 && (t % 16) == 0) P[HID * LF + 8 * HID + t / 16] = b2s;
}

// Level, first float and end of slice b of the table (slice_begin: prefix over levels).
__device__ __forceinline__ void slice_of(const FieldK& f, const SliceMap& sm, int b, int& l, int64_t& lo,
                                         int64_t& hi) {
  l = 0;
  while (l + 1 < f.L && sm.begin[l + 1] <= b) ++l;
  lo = (int64_t)(b - sm.begin[l]) * kSliceFloats;
  hi = min(lo + kSliceFloats, sm.level_floats[l]);
}

// Table gradient of one slice [lo, hi) (float offsets) of level l's table over the queries
// [m q_part / n_qparts, m (q_part + 1) / n_qparts), with (slice, q_part) from the workgroup
// index.  One query part: added to the gradient; several: written to partial[q_part][slice].
template <int F>
__global__ __launch_bounds__(kSliceThreads) void k_field_table_grad(const FieldK f, int m,
                                                                   const double* __restrict__ pn,
                                                                   const float* __restrict__ denc,
                                                                   SliceMap sm, float* __restrict__ gtable,
                                                                   float* __restrict__ partial) {
  __shared__ float s_g[kSliceFloats];
  const int b = blockIdx.x % sm.n_slices, qp = blockIdx.x / sm.n_slices;
  int l;
  int64_t lo, hi;
  slice_of(f, sm, b, l, lo, hi);
  const int q0 = (int)((int64_t)m * qp / sm.n_qparts), q1 = (int)((int64_t)m * (qp + 1) / sm.n_qparts);
  for (int i = threadIdx.x; i < kSliceFloats; i += kSliceThreads) s_g[i] = 0.f;
  __syncthreads();
  // kSliceBatch queries per thread at a time: their loads are issued together
  for (int q = q0 + threadIdx.x; q < q1; q += kSliceThreads * kSliceBatch) {
    double p[kSliceBatch][3];
    float dv[kSliceBatch][F];
#pragma unroll
    for (int u = 0; u < kSliceBatch; ++u) {
      const int qu = q + u * kSliceThreads;
      const bool in = qu < q1;
#pragma unroll
      for (int d = 0; d < 3; ++d) p[u][d] = in ? pn[(size_t)d * m + qu] : 0.0;
#pragma unroll
      for (int i = 0; i < F; ++i) dv[u][i] = in ? denc[(size_t)(l * F + i) * m + qu] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kSliceBatch; ++u) {
      if (q + u * kSliceThreads >= q1) break;
      level_corners(f, l, p[u], [&](int, uint32_t row, float w) {
        const int64_t off = (int64_t)row * F;
        if (off >= lo && off < hi) {
#pragma unroll
          for (int i = 0; i < F; ++i) atomicAdd(&s_g[off - lo + i], w * dv[u][i]);
        }
      });
    }
  }
  __syncthreads();
  if (sm.n_qparts == 1) {
    float* __restrict__ dst = gtable + ((size_t)l << f.log2T) * F + lo;
    for (int i = threadIdx.x; i < hi - lo; i += kSliceThreads) dst[i] += s_g[i];
  } else {
    float* __restrict__ dst = partial + ((size_t)qp * sm.n_slices + b) * kSliceFloats;
    for (int i = threadIdx.x; i < hi - lo; i += kSliceThreads) dst[i] = s_g[i];
  }
}

// gradient += the query parts' partial slices, added in part order
__global__ __launch_bounds__(256) void k_field_table_sum(const FieldK f, SliceMap sm, const float* __restrict__ partial,
                                                         float* __restrict__ gtable) {
  constexpr int kBlocksPerSlice = kSliceFloats / 256;
  const int b = blockIdx.x / kBlocksPerSlice;
  const int i = (blockIdx.x % kBlocksPerSlice) * 256 + threadIdx.x;
  int l;
  int64_t lo, hi;
  slice_of(f, sm, b, l, lo, hi);
  if (i >= hi - lo) return;
  float s = 0.f;
  for (int qp = 0; qp < sm.n_qparts; ++qp) s += partial[((size_t)qp * sm.n_slices + b) * kSliceFloats + i];
  gtable[((size_t)l << f.log2T) * sm.features + lo + i] += s;
}

// grad += sum over the workgroups' partials (fixed order): a workgroup takes kRedCols columns,
// its kRedGroups row groups each sum every kRedGroups-th partial row, then the groups are added
// in order.
constexpr int kRedCols = 32, kRedGroups = 32;
__global__ __launch_bounds__(kRedCols * kRedGroups) void k_field_reduce(const float* __restrict__ part, int rows,
                                                                        int stride, int n_w1, int hid,
                                                                        float* __restrict__ gw1, float* __restrict__ gb1,
                                                                        float* __restrict__ gw2, float* __restrict__ gb2) {
  __shared__ float s_sum[kRedGroups][kRedCols];
  const int col = threadIdx.x % kRedCols, rg = threadIdx.x / kRedCols;
  const int c = blockIdx.x * kRedCols + col;
  float s = 0.f;
  if (c < stride)
    for (int r = rg; r < rows; r += kRedGroups) s += part[(size_t)r * stride + c];
  s_sum[rg][col] = s;
  __syncthreads();
  if (rg != 0 || c >= stride) return;
  s = s_sum[0][col];
  for (int k = 1; k < kRedGroups; ++k) s += s_sum[k][col];
  float* dst;
  int i;
  if (c < n_w1) {
    dst = gw1;
    i = c;
  } else if (c < n_w1 + hid) {
    dst = gb1;
    i = c - n_w1;
  } else if (c < n_w1 + hid + 7 * hid) {
    dst = gw2;
    i = c - n_w1 - hid;
  } else {
    dst = gb2;
    i = c - n_w1 - 8 * hid;
  }
  if (dst) dst[i] += s;
}

template <int HID>
void fwd_f(int F, const FieldK& f, const QueryK& q, float* dpos, float* drot, hipStream_t st) {
  const int blocks = (q.m + kQuadThreads / 4 - 1) / (kQuadThreads / 4);
  switch (F) {
    case 1: k_field_fwd4<1, HID><<<blocks, kQuadThreads, 0, st>>>(f, q, dpos, drot); break;
    case 2: k_field_fwd4<2, HID><<<blocks, kQuadThreads, 0, st>>>(f, q, dpos, drot); break;
    case 4: k_field_fwd4<4, HID><<<blocks, kQuadThreads, 0, st>>>(f, q, dpos, drot); break;
    default: k_field_fwd4<8, HID><<<blocks, kQuadThreads, 0, st>>>(f, q, dpos, drot); break;
  }
}

template <int HID>
void bwd_f(int F, int blocks, const FieldK& f, const QueryK& q, const float* d_dpos, const float* d_drot,
           const FieldRows& rows, float* part, hipStream_t st) {
  const int qb4 = (q.m + kQuadThreads / 4 - 1) / (kQuadThreads / 4);
  switch (F) {
    case 1:
      k_field_bwd_query4<1, HID><<<qb4, kQuadThreads, 0, st>>>(f, q, d_dpos, d_drot, rows);
      k_field_wgrad<1, HID><<<blocks, kWgThreads, 0, st>>>(f, q.m, rows, part);
      break;
    case 2:
      k_field_bwd_query4<2, HID><<<qb4, kQuadThreads, 0, st>>>(f, q, d_dpos, d_drot, rows);
      k_field_wgrad<2, HID><<<blocks, kWgThreads, 0, st>>>(f, q.m, rows, part);
      break;
    case 4:
      k_field_bwd_query4<4, HID><<<qb4, kQuadThreads, 0, st>>>(f, q, d_dpos, d_drot, rows);
      k_field_wgrad<4, HID><<<blocks, kWgThreads, 0, st>>>(f, q.m, rows, part);
      break;
    default:
      k_field_bwd_query4<8, HID><<<qb4, kQuadThreads, 0, st>>>(f, q, d_dpos, d_drot, rows);
      k_field_wgrad<8, HID><<<blocks, kWgThreads, 0, st>>>(f, q.m, rows, part);
      break;
  }
}

}  // namespace

void launch_field_fwd(const FieldK& f, int F, int hidden, const QueryK& q, float* dpos, float* drot,
                      hipStream_t st) {
  if (q.m <= 0) return;
  if (hidden == 32)
    fwd_f<32>(F, f, q, dpos, drot, st);
  else
    fwd_f<64>(F, f, q, dpos, drot, st);
}

void launch_field_bwd(const FieldK& f, int F, int hidden, const QueryK& q, const float* d_dpos,
                      const float* d_drot, const FieldGradsK& g, const FieldScratch& ws, hipStream_t st) {
  if (q.m <= 0) return;
  // at least 64 queries per weight-gradient workgroup (small calls still spread over the CUs), at
  // most kFieldMaxBlocks partial rows
  int blocks = (q.m + 63) / 64;
  if (blocks > kFieldMaxBlocks) blocks = kFieldMaxBlocks;
  if (hidden == 32)
    bwd_f<32>(F, blocks, f, q, d_dpos, d_drot, ws.rows, ws.part, st);
  else
    bwd_f<64>(F, blocks, f, q, d_dpos, d_drot, ws.rows, ws.part, st);
  const int LF = f.L * F;
  const int stride = field_part_stride(hidden, LF);
  k_field_reduce<<<(stride + kRedCols - 1) / kRedCols, kRedCols * kRedGroups, 0, st>>>(
      ws.part, blocks, stride, hidden * LF, hidden, g.w1, g.b1, g.w2, g.b2);
  if (g.table) {
    SliceMap sm{};
    int total = 0;
    for (int l = 0; l < f.L; l++) {
      const int64_t N1 = (int64_t)f.res[l] + 1;
      const int64_t rows = ((f.dense >> l) & 1u) ? N1 * N1 * N1 : (int64_t(1) << f.log2T);
      sm.begin[l] = total;
      sm.level_floats[l] = rows * F;
      total += (int)((rows * F + kSliceFloats - 1) / kSliceFloats);
    }
    // split the queries so that about kSliceTargetBlocks workgroups run, within the partial buffer
    // and with at least kSliceThreads queries per workgroup
    int64_t parts = (kSliceTargetBlocks + total - 1) / total;
    parts = std::min<int64_t>(parts, kFieldPartialFloats / ((int64_t)total * kSliceFloats));
    parts = std::min<int64_t>(parts, (q.m + kSliceThreads - 1) / kSliceThreads);
    if (parts < 1) parts = 1;
    sm.n_slices = total;
    sm.n_qparts = (int)parts;
    sm.features = F;
    const unsigned grid = (unsigned)(total * parts);
    switch (F) {
      case 1: k_field_table_grad<1><<<grid, kSliceThreads, 0, st>>>(f, q.m, ws.rows.pn, ws.rows.denc, sm, g.table, ws.tpart); break;
      case 2: k_field_table_grad<2><<<grid, kSliceThreads, 0, st>>>(f, q.m, ws.rows.pn, ws.rows.denc, sm, g.table, ws.tpart); break;
      case 4: k_field_table_grad<4><<<grid, kSliceThreads, 0, st>>>(f, q.m, ws.rows.pn, ws.rows.denc, sm, g.table, ws.tpart); break;
      default: k_field_table_grad<8><<<grid, kSliceThreads, 0, st>>>(f, q.m, ws.rows.pn, ws.rows.denc, sm, g.table, ws.tpart); break;
    }
    if (parts > 1)
      k_field_table_sum<<<(unsigned)total * (kSliceFloats / 256), 256, 0, st>>>(f, sm, ws.tpart, g.table);
  }
}

}  // namespace dass
