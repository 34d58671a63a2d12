// Selective inheritance of G^var (Sec. 3.2, straight-through estimator of App. B) and the
// compaction of G^var rows that removes the masked-out Gaussians after the inheritance stage and
// the low-opacity ones after densification (Sec. 3.4).
//
// The mask M = Quant(sigmoid(m)) is 1 exactly when m >= 0.  It multiplies the activated opacity
// and scale, so in the renderer's parametrisation a masked Gaussian is drawn with
// logit = log_scale = -inf (opacity and scale 0) and an unmasked one with its own values.
// All kernels are elementwise over rows and bound by HBM traffic.
#include <cmath>

#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float sigmoidf(float x) { return 1.f / (1.f + __expf(-x)); }

// rows [0, n): base rows copied, G^var rows copied or masked
__global__ __launch_bounds__(kThreads) void k_inherit_apply(const float* __restrict__ logit,
                                                            const float* __restrict__ log_scale, int n, int nb,
                                                            int64_t stride, const float* __restrict__ m,
                                                            float* __restrict__ lg_out, float* __restrict__ ls_out) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const bool on = i < nb || m[i - nb] >= 0.f;
  const float ninf = -INFINITY;
  lg_out[i] = on ? logit[i] : ninf;
#pragma unroll
  for (int d = 0; d < 3; ++d) ls_out[d * stride + i] = on ? log_scale[d * stride + i] : ninf;
}

// dm[j] += (dL/dM + lambda) sigmoid'(m_j) for G^var row nb + j; *loss += lambda sum sigmoid(m)
__global__ __launch_bounds__(kThreads) void k_inherit_adjoint(const float* __restrict__ logit, int nb, int nv,
                                                              int64_t stride, const float* __restrict__ m,
                                                              const float* __restrict__ g_logit,
                                                              const float* __restrict__ g_ls, float lam,
                                                              float* __restrict__ dm, float* __restrict__ loss) {
  __shared__ float s_w[kThreads / 64];
  const int j = blockIdx.x * kThreads + threadIdx.x;
  float sig = 0.f;
  if (j < nv) {
    const int i = nb + j;
    const float mj = m[j];
    sig = sigmoidf(mj);
    float dM = 0.f;
    if (mj >= 0.f) {
      // dL/do_r o + sum_d dL/ds_r,d s_d with o_r = sigmoid(logit), s_r = exp(log_scale):
      // g_logit / (1 - o) + sum_d g_log_scale,d, and 1 / (1 - o) = 1 + exp(logit)
      const float gl = g_logit[i];
      dM = (gl != 0.f ? gl * (1.f + __expf(logit[i])) : 0.f) + g_ls[i] + g_ls[stride + i] + g_ls[2 * stride + i];
    }
    dm[j] += (dM + lam) * sig * (1.f - sig);
  }
  if (!loss) return;
  float v = sig;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, lam * ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])));
}

// keep flag of G^var row nb + j
__global__ __launch_bounds__(kThreads) void k_keep_flags(const float* __restrict__ logit, int nb, int nv,
                                                         const float* __restrict__ m, float min_logit,
                                                         uint32_t* __restrict__ keep) {
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= nv) return;
  bool k = !m || m[j] >= 0.f;
  k = k && logit[nb + j] >= min_logit;
  keep[j] = k ? 1u : 0u;
}

// kept rows' planes gathered into the staging buffer at their compacted positions
__global__ __launch_bounds__(kThreads) void k_compact_gather(const CompactPlanes P, int nb, int nv,
                                                             const uint32_t* __restrict__ keep,
                                                             const uint64_t* __restrict__ dest,
                                                             float* __restrict__ stage, int64_t sstride) {
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= nv || !keep[j]) return;
  const int64_t k = (int64_t)dest[j];
  for (int p = 0; p < P.count; ++p) stage[p * sstride + k] = P.plane[p][nb + j];
}

// staging buffer back into rows [nb, nb + kept); the kept count is read on the device
__global__ __launch_bounds__(kThreads) void k_compact_scatter(const CompactPlanes P, int nb, int nv,
                                                              const uint64_t* __restrict__ dest,
                                                              const float* __restrict__ stage, int64_t sstride,
                                                              int32_t* __restrict__ n_kept) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  const int64_t total = (int64_t)dest[nv];
  if (k == 0) *n_kept = (int32_t)total;
  if (k >= total) return;
  for (int p = 0; p < P.count; ++p) P.plane[p][nb + k] = stage[p * sstride + k];
}

}  // namespace

void launch_inherit_apply(const SceneK& s, int nb, const float* m, float* lg_out, float* ls_out, hipStream_t st) {
  if (s.n <= 0) return;
  k_inherit_apply<<<(s.n + kThreads - 1) / kThreads, kThreads, 0, st>>>(s.logit, s.log_scale, s.n, nb, s.stride, m,
                                                                        lg_out, ls_out);
}

void launch_inherit_adjoint(const SceneK& s, int nb, const float* m, const float* g_logit, const float* g_ls,
                            float lam, float* dm, float* loss, hipStream_t st) {
  const int nv = s.n - nb;
  if (nv <= 0) return;
  k_inherit_adjoint<<<(nv + kThreads - 1) / kThreads, kThreads, 0, st>>>(s.logit, nb, nv, s.stride, m, g_logit, g_ls,
                                                                          lam, dm, loss);
}

void launch_compact_var(const CompactPlanes& P, const float* logit, int nb, int nv, const float* m, float min_logit,
                        uint32_t* keep, uint64_t* dest, uint64_t* scan_tmp, float* stage, int64_t sstride,
                        int32_t* n_kept, hipStream_t st) {
  const int blocks = nv > 0 ? (nv + kThreads - 1) / kThreads : 1;
  if (nv > 0) k_keep_flags<<<blocks, kThreads, 0, st>>>(logit, nb, nv, m, min_logit, keep);
  scan_u32_to_u64(keep, dest, nv, scan_tmp, st);
  if (nv > 0)
    k_compact_gather<<<blocks, kThreads, 0, st>>>(P, nb, nv, keep, dest, stage, sstride);
  k_compact_scatter<<<blocks, kThreads, 0, st>>>(P, nb, nv, dest, stage, sstride, n_kept);
}

}  // namespace dass
