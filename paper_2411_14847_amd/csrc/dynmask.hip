// The 3D half of the per-Gaussian dynamics mask (Sec. 3.3): pixels whose optical flow exceeds
// gamma_op are dynamic areas; the rendered identity features there are classified into objects
// (Gaussian Grouping's linear classifier, argmax), those objects are dynamic, and a Gaussian is
// dynamic when the classification of its own identity feature is one of them.  The flow itself
// comes from an optical-flow network outside this library.
#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kThreads = 256;

// The classifier in LDS, padded to kFeatMaxC weights per object (zeros beyond C).
struct ClsLds {
  float4 w[kMaxObjects][kFeatMaxC / 4];
  float b[kMaxObjects];
};

__device__ __forceinline__ void load_classifier(ClsLds& s, const float* __restrict__ w, const float* __restrict__ bias,
                                                int K, int C) {
  for (int e = threadIdx.x; e < K * kFeatMaxC; e += kThreads) {
    const int k = e / kFeatMaxC, c = e % kFeatMaxC;
    reinterpret_cast<float*>(&s.w[k][0])[c] = c < C ? w[k * C + c] : 0.f;
  }
  for (int k = threadIdx.x; k < K; k += kThreads) s.b[k] = bias[k];
  __syncthreads();
}

// argmax_k (cls_w[k] . x + cls_b[k]), first index on ties
__device__ __forceinline__ int classify(const ClsLds& s, int K, const float* x) {
  float best = -INFINITY;
  int id = 0;
  for (int k = 0; k < K; ++k) {
    float v = s.b[k];
#pragma unroll
    for (int c = 0; c < kFeatMaxC / 4; ++c) {
      const float4 w = s.w[k][c];
      v = fmaf(w.x, x[4 * c], v);
      v = fmaf(w.y, x[4 * c + 1], v);
      v = fmaf(w.z, x[4 * c + 2], v);
      v = fmaf(w.w, x[4 * c + 3], v);
    }
    if (v > best) {
      best = v;
      id = k;
    }
  }
  return id;
}

// blockIdx.y = view
__global__ __launch_bounds__(kThreads) void k_dynamic_objects(const DynMaskArgs a, uint32_t* __restrict__ dyn_obj) {
  __shared__ ClsLds s;
  const int v = blockIdx.y;
  const int64_t hw = a.hw[v];
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool dyn = p < hw && a.flow[v][p] > a.gamma_op;
  if (__syncthreads_or(dyn) == 0) return;  // uniform: no dynamic pixel in this block
  load_classifier(s, a.w, a.b, a.K, a.C);
  if (!dyn) return;
  float x[kFeatMaxC];
#pragma unroll
  for (int c = 0; c < kFeatMaxC; ++c) x[c] = c < a.C ? a.feat_img[v][c * hw + p] : 0.f;
  dyn_obj[classify(s, a.K, x)] = 1u;
}

__global__ __launch_bounds__(kThreads) void k_dynamic_flags(const DynMaskArgs a, const uint32_t* __restrict__ dyn_obj,
                                                            uint32_t* __restrict__ keep) {
  __shared__ ClsLds s;
  load_classifier(s, a.w, a.b, a.K, a.C);
  const int g = blockIdx.x * kThreads + threadIdx.x;
  if (g >= a.n) return;
  float x[kFeatMaxC];
#pragma unroll
  for (int c = 0; c < kFeatMaxC; ++c) x[c] = c < a.C ? a.feat[c * a.stride + g] : 0.f;
  keep[g] = dyn_obj[classify(s, a.K, x)] ? 1u : 0u;
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
  int64_t hw_max = 0;
  for (int v = 0; v < a.nv; ++v) hw_max = a.hw[v] > hw_max ? a.hw[v] : hw_max;
  if (hw_max > 0)
    k_dynamic_objects<<<dim3((unsigned)((hw_max + kThreads - 1) / kThreads), (unsigned)a.nv), kThreads, 0, st>>>(
        a, dyn_obj);
  const int blocks = a.n > 0 ? (a.n + kThreads - 1) / kThreads : 1;
  if (a.n > 0) k_dynamic_flags<<<blocks, kThreads, 0, st>>>(a, dyn_obj, keep);
  scan_u32_to_u64(keep, dest, a.n, scan_tmp, st);
  k_dynamic_scatter<<<blocks, kThreads, 0, st>>>(a.n, keep, dest, dyn_idx, n_dyn);
}

}  // namespace dass
