// The 3D half of the per-Gaussian dynamics mask (Sec. 3.3): pixels whose optical flow exceeds
// gamma_op are dynamic areas; the rendered identity features there are classified into objects
// (Gaussian Grouping's linear classifier, argmax), those objects are dynamic, and a Gaussian is
// dynamic when the classification of its own identity feature is one of them.  The flow itself
// comes from an optical-flow network outside this library.
#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kThreads = 256;

// argmax_k (cls_w[k] . x + cls_b[k]), first index on ties; weights read with uniform addresses
__device__ __forceinline__ int classify(const float* __restrict__ w, const float* __restrict__ bias, int K, int C,
                                        const float* x) {
  float best = -INFINITY;
  int id = 0;
  for (int k = 0; k < K; ++k) {
    float s = bias[k];
#pragma unroll
    for (int c = 0; c < kFeatMaxC; ++c)
      if (c < C) s = fmaf(w[k * C + c], x[c], s);
    if (s > best) {
      best = s;
      id = k;
    }
  }
  return id;
}

__global__ __launch_bounds__(kThreads) void k_dynamic_objects(const float* __restrict__ feat_img, int64_t hw,
                                                              const float* __restrict__ flow, float gamma_op,
                                                              const float* __restrict__ w, const float* __restrict__ bias,
                                                              int K, int C, uint32_t* __restrict__ dyn_obj) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= hw || !(flow[p] > gamma_op)) return;
  float x[kFeatMaxC];
#pragma unroll
  for (int c = 0; c < kFeatMaxC; ++c) x[c] = c < C ? feat_img[c * hw + p] : 0.f;
  dyn_obj[classify(w, bias, K, C, x)] = 1u;
}

__global__ __launch_bounds__(kThreads) void k_dynamic_flags(const float* __restrict__ feat, int64_t stride, int n,
                                                            const float* __restrict__ w, const float* __restrict__ bias,
                                                            int K, int C, const uint32_t* __restrict__ dyn_obj,
                                                            uint32_t* __restrict__ keep) {
  const int g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  float x[kFeatMaxC];
#pragma unroll
  for (int c = 0; c < kFeatMaxC; ++c) x[c] = c < C ? feat[c * stride + g] : 0.f;
  keep[g] = dyn_obj[classify(w, bias, K, C, x)] ? 1u : 0u;
}

__global__ __launch_bounds__(kThreads) void k_dynamic_scatter(int n, const uint32_t* __restrict__ keep,
                                                              const uint64_t* __restrict__ dest,
                                                              int32_t* __restrict__ dyn_idx, int32_t* __restrict__ n_dyn) {
  const int g = blockIdx.x * kThreads + threadIdx.x;
  if (g == 0) *n_dyn = (int32_t)dest[n];
  if (g < n && keep[g]) dyn_idx[dest[g]] = g;
}

}  // namespace

void launch_dynamic_mask(const DynMaskArgs& a, uint32_t* dyn_obj, uint32_t* keep, uint64_t* dest, uint64_t* scan_tmp,
                         int32_t* dyn_idx, int32_t* n_dyn, hipStream_t st) {
  launch_fill_u32(dyn_obj, 0u, a.K, st);
  for (int v = 0; v < a.nv; ++v) {
    const int64_t hw = a.hw[v];
    if (hw > 0)
      k_dynamic_objects<<<(unsigned)((hw + kThreads - 1) / kThreads), kThreads, 0, st>>>(
          a.feat_img[v], hw, a.flow[v], a.gamma_op, a.w, a.b, a.K, a.C, dyn_obj);
  }
  const int blocks = a.n > 0 ? (a.n + kThreads - 1) / kThreads : 1;
  if (a.n > 0)
    k_dynamic_flags<<<blocks, kThreads, 0, st>>>(a.feat, a.stride, a.n, a.w, a.b, a.K, a.C, dyn_obj, keep);
  scan_u32_to_u64(keep, dest, a.n, scan_tmp, st);
  k_dynamic_scatter<<<blocks, kThreads, 0, st>>>(a.n, keep, dest, dyn_idx, n_dyn);
}

}  // namespace dass
