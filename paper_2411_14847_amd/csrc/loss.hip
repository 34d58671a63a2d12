// D-SSIM term of the fidelity loss, Eq. (3): L = (1/V) sum_v [(1 - lambda) L1_v + lambda (1 -
// SSIM_v)], with SSIM_v the mean over the three channels and all pixels of the SSIM map (11x11
// Gaussian window, sigma 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2 for images in [0, 1]).
//
// Two passes, one workgroup per 32x32 pixel tile (channels in turn), each staging the tile plus
// its 5-pixel halo in LDS and applying the separable window as a horizontal then a vertical
// 11-tap sum; every thread slides the window over 4 consecutive outputs, so each staged value
// is read from LDS about once per 4 outputs instead of 11 times:
//   forward: the five window moments (mu_x, mu_y, E[x^2], E[y^2], E[xy]) of every pixel, the
//     SSIM map and its derivatives with respect to mu_x, E[x^2] and E[xy], scaled by
//     dL/dSSIM; these three maps go to the caller's scratch;
//   backward: the window sums of the three maps (the window is symmetric, so the adjoint of a
//     window sum is the same sum) give dL/dx = W*P1 + 2 x W*P2 + y W*P3, to which the L1 term
//     and the error map of Sec. 3.4 are added.
#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kT = 32;           // output tile edge
constexpr int kR = 5;            // window radius
constexpr int kTaps = 2 * kR + 1;
constexpr int kE = kT + 2 * kR;  // staged edge (42)
constexpr int kEP = kE + 1;      // padded staged row
constexpr int kHP = kT + 1;      // padded row of horizontal sums
constexpr int kRun = 4;          // consecutive outputs per thread and pass
constexpr int kThreads = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

// Workgroups are dealt to the XCDs round-robin; remapping gives each XCD a contiguous range of
// tiles, so the halos a tile shares with its neighbours are read through the same L2.
__device__ __forceinline__ int64_t tile_of_block(int64_t bid, int64_t per) {
  return (bid % kNumXcd) * per + bid / kNumXcd;
}

__device__ __forceinline__ int view_of_block(const SsimArgs& a, int64_t blk) {
  int v = 0;
  while (v + 1 < a.nv && blk >= a.v[v + 1].block_begin) v++;
  return v;
}

// Sum over the workgroup of x, added times `scale` into one loss slot.
__device__ __forceinline__ void add_to_slot(float x, float scale, float* s_w, float* loss_slots) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(&loss_slots[blockIdx.x % kLossSlots], ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) * scale);
}

// Stages rows [oy - 5, oy + 37) x cols [ox - 5, ox + 37) of the NS planes src[k] into dst[k]
// (zero outside the image).  All loads are issued before the first LDS store, so their
// latencies overlap.
constexpr int kStageIters = (kE * kE + kThreads - 1) / kThreads;
template <int NS>
__device__ __forceinline__ void stage(float (*dst)[kE][kEP], const float* const (&src)[NS], int ox, int oy, int W,
                                      int H) {
  float v[NS][kStageIters];
#pragma unroll
  for (int u = 0; u < kStageIters; u++) {
    const int e = threadIdx.x + u * kThreads;
    const int r = e / kE, q = e % kE;
    const int gx = ox - kR + q, gy = oy - kR + r;
    const bool in = e < kE * kE && gx >= 0 && gy >= 0 && gx < W && gy < H;
    const int64_t p = in ? (int64_t)gy * W + gx : 0;
#pragma unroll
    for (int k = 0; k < NS; k++) v[k][u] = in ? src[k][p] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kStageIters; u++) {
    const int e = threadIdx.x + u * kThreads;
    if (e < kE * kE) {
#pragma unroll
      for (int k = 0; k < NS; k++) dst[k][e / kE][e % kE] = v[k][u];
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(SsimArgs a, int64_t total, int64_t per,
                                                           float* __restrict__ loss_slots) {
  __shared__ float s_xy[2][kE][kEP];  // render, target
  __shared__ float s_h[5][kE][kHP];    // horizontal sums of x, y, x^2, y^2, xy
  __shared__ float s_w[4];
  const int tid = threadIdx.x;
  const int64_t blk = tile_of_block(blockIdx.x, per);
  if (blk >= total) return;  // uniform over the workgroup
  const int vi = view_of_block(a, blk);
  const SsimView& V = a.v[vi];
  const int t = (int)(blk - V.block_begin);
  const int ox = (t % V.TX) * kT, oy = (t / V.TX) * kT;
  const int64_t hw = (int64_t)V.W * V.H;
  const int col = tid % kT, i0 = (tid / kT) * kRun;  // vertical pass: pixels (col, i0 .. i0 + 3)
  const float gS = a.gS[vi];                          // dL/dSSIM(pixel, channel)
  float ssum = 0.f;
  for (int c = 0; c < 3; c++) {
    const float* const planes[2] = {V.render + c * hw, V.target + c * hw};
    stage<2>(s_xy, planes, ox, oy, V.W, V.H);
    __syncthreads();
    // horizontal: row r, outputs q0 .. q0 + 3
    for (int task = tid; task < kE * (kT / kRun); task += kThreads) {
      const int r = task / (kT / kRun), q0 = (task % (kT / kRun)) * kRun;
      float h[5][kRun];
#pragma unroll
      for (int m = 0; m < 5; m++)
#pragma unroll
        for (int o = 0; o < kRun; o++) h[m][o] = 0.f;
#pragma unroll
      for (int n = 0; n < kTaps + kRun - 1; n++) {
        const float xv = s_xy[0][r][q0 + n], yv = s_xy[1][r][q0 + n];
        const float xx = xv * xv, yy = yv * yv, xy = xv * yv;
#pragma unroll
        for (int o = 0; o < kRun; o++) {
          const int k = n - o;
          if (k < 0 || k >= kTaps) continue;
          const float w = a.w[k];
          h[0][o] += w * xv;
          h[1][o] += w * yv;
          h[2][o] += w * xx;
          h[3][o] += w * yy;
          h[4][o] += w * xy;
        }
      }
#pragma unroll
      for (int m = 0; m < 5; m++)
#pragma unroll
        for (int o = 0; o < kRun; o++) s_h[m][r][q0 + o] = h[m][o];
    }
    __syncthreads();
    // vertical: column col, rows i0 .. i0 + 3
    float mo[5][kRun];
#pragma unroll
    for (int m = 0; m < 5; m++) {
#pragma unroll
      for (int o = 0; o < kRun; o++) mo[m][o] = 0.f;
#pragma unroll
      for (int n = 0; n < kTaps + kRun - 1; n++) {
        const float hv = s_h[m][i0 + n][col];
#pragma unroll
        for (int o = 0; o < kRun; o++) {
          const int k = n - o;
          if (k >= 0 && k < kTaps) mo[m][o] += a.w[k] * hv;
        }
      }
    }
    float* P = V.scratch + (int64_t)(3 * c) * hw;
#pragma unroll
    for (int o = 0; o < kRun; o++) {
      const int px = ox + col, py = oy + i0 + o;
      if (px >= V.W || py >= V.H) continue;
      const float mx = mo[0][o], my = mo[1][o];
      const float A = 2.f * mx * my + kC1;                                // luminance numerator
      const float B = 2.f * (mo[4][o] - mx * my) + kC2;                   // 2 sigma_xy + C2
      const float Cc = mx * mx + my * my + kC1;                           // luminance denominator
      const float D = (mo[2][o] - mx * mx) + (mo[3][o] - my * my) + kC2;  // sigma_x^2 + sigma_y^2 + C2
      const float iCD = 1.f / (Cc * D);
      const float S = A * B * iCD;
      const float dmx = (2.f * my * B - 2.f * my * A) * iCD - S * (2.f * mx / Cc - 2.f * mx / D);
      const float dxx = -S / D;
      const float dxy = 2.f * A * iCD;
      const int64_t p = (int64_t)py * V.W + px;
      P[p] = gS * dmx;
      P[hw + p] = gS * dxx;
      P[2 * hw + p] = gS * dxy;
      ssum += S;
    }
    __syncthreads();  // the next channel restages
  }
  add_to_slot(ssum, gS, s_w, loss_slots);
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(SsimArgs a, int64_t total, int64_t per,
                                                           float* __restrict__ loss_slots) {
  __shared__ float s_p[3][kE][kEP];
  __shared__ float s_h[3][kE][kHP];
  __shared__ float s_w[4];
  const int tid = threadIdx.x;
  const int64_t blk = tile_of_block(blockIdx.x, per);
  if (blk >= total) return;  // uniform over the workgroup
  const int vi = view_of_block(a, blk);
  const SsimView& V = a.v[vi];
  const int t = (int)(blk - V.block_begin);
  const int ox = (t % V.TX) * kT, oy = (t / V.TX) * kT;
  const int64_t hw = (int64_t)V.W * V.H;
  const int col = tid % kT, i0 = (tid / kT) * kRun;
  const float sl1 = a.l1_scale[vi];  // (1 - lambda) / (3 H W V)
  float e[kRun] = {0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < 3; c++) {
    const float* P = V.scratch + (int64_t)(3 * c) * hw;
    const float* const planes[3] = {P, P + hw, P + 2 * hw};
    stage<3>(s_p, planes, ox, oy, V.W, V.H);
    __syncthreads();
    for (int task = tid; task < kE * (kT / kRun); task += kThreads) {
      const int r = task / (kT / kRun), q0 = (task % (kT / kRun)) * kRun;
#pragma unroll
      for (int m = 0; m < 3; m++) {
        float h[kRun] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < kTaps + kRun - 1; n++) {
          const float pv = s_p[m][r][q0 + n];
#pragma unroll
          for (int o = 0; o < kRun; o++) {
            const int k = n - o;
            if (k >= 0 && k < kTaps) h[o] += a.w[k] * pv;
          }
        }
#pragma unroll
        for (int o = 0; o < kRun; o++) s_h[m][r][q0 + o] = h[o];
      }
    }
    __syncthreads();
    float Q[3][kRun];
#pragma unroll
    for (int m = 0; m < 3; m++) {
#pragma unroll
      for (int o = 0; o < kRun; o++) Q[m][o] = 0.f;
#pragma unroll
      for (int n = 0; n < kTaps + kRun - 1; n++) {
        const float hv = s_h[m][i0 + n][col];
#pragma unroll
        for (int o = 0; o < kRun; o++) {
          const int k = n - o;
          if (k >= 0 && k < kTaps) Q[m][o] += a.w[k] * hv;
        }
      }
    }
#pragma unroll
    for (int o = 0; o < kRun; o++) {
      const int px = ox + col, py = oy + i0 + o;
      if (px >= V.W || py >= V.H) continue;
      const int64_t pix = (int64_t)py * V.W + px;
      const float x = V.render[c * hw + pix], y = V.target[c * hw + pix];
      const float d = x - y;
      const float l1 = d > 0.f ? sl1 : (d < 0.f ? -sl1 : 0.f);
      V.dl[c * hw + pix] = l1 + (Q[0][o] + 2.f * x * Q[1][o] + y * Q[2][o]);
      e[o] += fabsf(d);  // summed over channels in channel order
    }
    __syncthreads();  // the next channel restages
  }
  float l1sum = 0.f;
#pragma unroll
  for (int o = 0; o < kRun; o++) {
    const int px = ox + col, py = oy + i0 + o;
    if (px >= V.W || py >= V.H) continue;
    if (V.err) V.err[(int64_t)py * V.W + px] = e[o] * (1.0f / 3.0f);
    l1sum += e[o];
  }
  add_to_slot(l1sum, sl1, s_w, loss_slots);
}

}  // namespace

int64_t ssim_tiles(int W, int H) { return (int64_t)((W + kT - 1) / kT) * ((H + kT - 1) / kT); }
int ssim_tile_edge() { return kT; }

void launch_ssim(const SsimArgs& a, int64_t total_blocks, float* loss_slots, hipStream_t st) {
  if (total_blocks <= 0) return;
  const int64_t per = (total_blocks + kNumXcd - 1) / kNumXcd;
  k_ssim_fwd<<<(unsigned)(per * kNumXcd), kThreads, 0, st>>>(a, total_blocks, per, loss_slots);
  k_ssim_bwd<<<(unsigned)(per * kNumXcd), kThreads, 0, st>>>(a, total_blocks, per, loss_slots);
}

}  // namespace dass
