// D-SSIM term of the fidelity loss, Eq. (3): L = (1/V) sum_v [(1 - lambda) L1_v + lambda (1 -
// SSIM_v)], with SSIM_v the mean over the three channels and all pixels of the SSIM map (11x11
// Gaussian window, sigma 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2 for images in [0, 1]).
//
// Two passes over 16x16 pixel tiles, each staging a tile plus its 5-pixel halo in LDS and
// applying the separable window as a horizontal then a vertical 11-tap sum:
//   forward: the five window moments (mu_x, mu_y, E[x^2], E[y^2], E[xy]) of every pixel, the
//     SSIM map and its derivatives with respect to mu_x, E[x^2] and E[xy], scaled by
//     dL/dSSIM; these three maps go to the caller's scratch;
//   backward: the window sums of the three maps (the window is symmetric, so the adjoint of a
//     window sum is the same sum) give dL/dx = W*P1 + 2 x W*P2 + y W*P3, to which the L1 term
//     and the error map of Sec. 3.4 are added.
#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kT = 16;             // output tile edge
constexpr int kR = 5;              // window radius
constexpr int kE = kT + 2 * kR;    // staged edge (26)
constexpr int kEP = kE + 1;        // padded LDS row
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

__device__ __forceinline__ int view_of_block(const SsimArgs& a, int64_t blk) {
  int v = 0;
  while (v + 1 < a.nv && blk >= a.v[v + 1].block_begin) v++;
  return v;
}

__global__ __launch_bounds__(kT* kT) void k_ssim_fwd(SsimArgs a, float* __restrict__ loss_slots) {
  __shared__ float s_x[kE][kEP], s_y[kE][kEP];
  __shared__ float s_h[5][kE][kT];  // horizontal sums: x, y, x^2, y^2, xy
  __shared__ float s_w[4];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int vi = view_of_block(a, blk);
  const SsimView& V = a.v[vi];
  const int t = (int)(blk - V.block_begin);
  const int ox = (t % V.TX) * kT, oy = (t / V.TX) * kT;
  const int64_t hw = (int64_t)V.W * V.H;
  const int i = tid / kT, j = tid % kT;  // output pixel (ox + j, oy + i)
  const int px = ox + j, py = oy + i;
  const bool inside = px < V.W && py < V.H;
  const float gS = a.gS[vi];  // dL/dSSIM(pixel, channel)
  float ssum = 0.f;
  for (int c = 0; c < 3; c++) {
    const float* X = V.render + c * hw;
    const float* Y = V.target + c * hw;
    for (int e = tid; e < kE * kE; e += kT * kT) {
      const int r = e / kE, q = e % kE;
      const int gx = ox - kR + q, gy = oy - kR + r;
      const bool in = gx >= 0 && gy >= 0 && gx < V.W && gy < V.H;
      const int64_t p = (int64_t)gy * V.W + gx;
      s_x[r][q] = in ? X[p] : 0.f;
      s_y[r][q] = in ? Y[p] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < kE * kT; e += kT * kT) {
      const int r = e / kT, q = e % kT;
      float mx = 0.f, my = 0.f, xx = 0.f, yy = 0.f, xy = 0.f;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; k++) {
        const float xv = s_x[r][q + k], yv = s_y[r][q + k];
        const float wx = a.w[k] * xv, wy = a.w[k] * yv;
        mx += wx;
        my += wy;
        xx += wx * xv;
        yy += wy * yv;
        xy += wx * yv;
      }
      s_h[0][r][q] = mx;
      s_h[1][r][q] = my;
      s_h[2][r][q] = xx;
      s_h[3][r][q] = yy;
      s_h[4][r][q] = xy;
    }
    __syncthreads();
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 2 * kR + 1; k++) {
#pragma unroll
      for (int q = 0; q < 5; q++) m[q] += a.w[k] * s_h[q][i + k][j];
    }
    if (inside) {
      const float mx = m[0], my = m[1];
      const float A = 2.f * mx * my + kC1;
      const float B = 2.f * (m[4] - mx * my) + kC2;
      const float Cc = mx * mx + my * my + kC1;
      const float D = (m[2] - mx * mx) + (m[3] - my * my) + kC2;
      const float iCD = 1.f / (Cc * D);
      const float S = A * B * iCD;
      const float dmx = (2.f * my * B - 2.f * my * A) * iCD - S * (2.f * mx / Cc - 2.f * mx / D);
      const float dxx = -S / D;
      const float dxy = 2.f * A * iCD;
      const int64_t p = (int64_t)py * V.W + px;
      float* P = V.scratch + (int64_t)(3 * c) * hw;
      P[p] = gS * dmx;
      P[hw + p] = gS * dxx;
      P[2 * hw + p] = gS * dxy;
      ssum += S;
    }
    __syncthreads();  // the next channel reuses the staging buffers
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) ssum += __shfl_xor(ssum, d, 64);
  if ((tid & 63) == 0) s_w[tid >> 6] = ssum;
  __syncthreads();
  if (tid == 0) atomicAdd(&loss_slots[blk % kLossSlots], ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) * gS);
}

__global__ __launch_bounds__(kT* kT) void k_ssim_bwd(SsimArgs a, float* __restrict__ loss_slots) {
  __shared__ float s_p[3][kE][kEP];
  __shared__ float s_h[3][kE][kT];
  __shared__ float s_w[4];
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int vi = view_of_block(a, blk);
  const SsimView& V = a.v[vi];
  const int t = (int)(blk - V.block_begin);
  const int ox = (t % V.TX) * kT, oy = (t / V.TX) * kT;
  const int64_t hw = (int64_t)V.W * V.H;
  const int i = tid / kT, j = tid % kT;
  const int px = ox + j, py = oy + i;
  const bool inside = px < V.W && py < V.H;
  const int64_t pix = (int64_t)py * V.W + px;
  const float sl1 = a.l1_scale[vi];  // (1 - lambda) / (3 H W V)
  float e = 0.f, l1sum = 0.f;
  for (int c = 0; c < 3; c++) {
    const float* P = V.scratch + (int64_t)(3 * c) * hw;
    for (int n = tid; n < kE * kE; n += kT * kT) {
      const int r = n / kE, q = n % kE;
      const int gx = ox - kR + q, gy = oy - kR + r;
      const bool in = gx >= 0 && gy >= 0 && gx < V.W && gy < V.H;
      const int64_t p = (int64_t)gy * V.W + gx;
#pragma unroll
      for (int m = 0; m < 3; m++) s_p[m][r][q] = in ? P[m * hw + p] : 0.f;
    }
    __syncthreads();
    for (int n = tid; n < kE * kT; n += kT * kT) {
      const int r = n / kT, q = n % kT;
      float h[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; k++) {
#pragma unroll
        for (int m = 0; m < 3; m++) h[m] += a.w[k] * s_p[m][r][q + k];
      }
#pragma unroll
      for (int m = 0; m < 3; m++) s_h[m][r][q] = h[m];
    }
    __syncthreads();
    float Q[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 2 * kR + 1; k++) {
#pragma unroll
      for (int m = 0; m < 3; m++) Q[m] += a.w[k] * s_h[m][i + k][j];
    }
    if (inside) {
      const float x = V.render[c * hw + pix], y = V.target[c * hw + pix];
      const float d = x - y;
      const float l1 = d > 0.f ? sl1 : (d < 0.f ? -sl1 : 0.f);
      V.dl[c * hw + pix] = l1 + (Q[0] + 2.f * x * Q[1] + y * Q[2]);
      e += fabsf(d);
    }
    __syncthreads();
  }
  if (inside && V.err) V.err[pix] = e * (1.0f / 3.0f);
  l1sum = e;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) l1sum += __shfl_xor(l1sum, d, 64);
  if ((tid & 63) == 0) s_w[tid >> 6] = l1sum;
  __syncthreads();
  if (tid == 0) atomicAdd(&loss_slots[blk % kLossSlots], ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) * sl1);
}

}  // namespace

int64_t ssim_tiles(int W, int H) { return (int64_t)((W + kT - 1) / kT) * ((H + kT - 1) / kT); }
int ssim_tile_edge() { return kT; }

void launch_ssim(const SsimArgs& a, int64_t total_blocks, float* loss_slots, hipStream_t st) {
  if (total_blocks <= 0) return;
  k_ssim_fwd<<<(unsigned)total_blocks, kT * kT, 0, st>>>(a, loss_slots);
  k_ssim_bwd<<<(unsigned)total_blocks, kT * kT, 0, st>>>(a, loss_slots);
}

}  // namespace dass
