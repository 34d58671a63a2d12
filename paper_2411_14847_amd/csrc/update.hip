// Per-iteration updates around the rasterizer: dynamics-aware shift (Sec. 3.3) and its
// adjoint, a multi-tensor Adam step, the L1 fidelity gradient with the error map (Sec. 3.4),
// and error-guided densification (Sec. 3.4, Alg. 1, Eq. 4).  All are memory-bound
// elementwise passes; each is one launch over all of its groups / views.
#include "dass_internal.h"

namespace dass {
namespace {

// Hamilton product (w, x, y, z).
__device__ __forceinline__ void qmul(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

__global__ __launch_bounds__(256) void k_copy_mq(const float* __restrict__ mean, const float* __restrict__ quat,
                                                 float* __restrict__ om, float* __restrict__ oq, int n, int stride) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int i = 0; i < 3; i++) om[(int64_t)i * stride + g] = mean[(int64_t)i * stride + g];
  for (int i = 0; i < 4; i++) oq[(int64_t)i * stride + g] = quat[(int64_t)i * stride + g];
}

__global__ __launch_bounds__(256) void k_shift_fwd(const float* __restrict__ mean, const float* __restrict__ quat,
                                                   float* __restrict__ om, float* __restrict__ oq, int stride, int n,
                                                   const int32_t* __restrict__ idx, int n_dyn,
                                                   const float* __restrict__ dpos, const float* __restrict__ drot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_dyn) return;
  const int64_t g = idx[j];
  if (g < 0 || g >= n) return;  // out-of-range index: ignored
  double q[4], s[4], o[4], qn = 0.0, sn = 0.0;
  for (int i = 0; i < 4; i++) {
    q[i] = quat[i * (int64_t)stride + g];
    s[i] = drot[(int64_t)i * n_dyn + j];
    qn += q[i] * q[i];
    sn += s[i] * s[i];
  }
  const double iq = 1.0 / sqrt(qn), is = 1.0 / sqrt(sn);
  for (int i = 0; i < 4; i++) { q[i] *= iq; s[i] *= is; }
  qmul(q, s, o);
  for (int i = 0; i < 3; i++)
    om[i * (int64_t)stride + g] = (float)((double)mean[i * (int64_t)stride + g] + (double)dpos[(int64_t)i * n_dyn + j]);
  for (int i = 0; i < 4; i++) oq[i * (int64_t)stride + g] = (float)o[i];
}

// d sigma_hat = L(q_hat)^T dq' = conj(q_hat) (x) dq'; then back through sigma_hat = sigma/|sigma|.
__global__ __launch_bounds__(256) void k_shift_adj(const float* __restrict__ quat, const float* __restrict__ dmean,
                                                   const float* __restrict__ dquat, int stride, int n,
                                                   const int32_t* __restrict__ idx, int n_dyn,
                                                   const float* __restrict__ drot, float* __restrict__ d_dpos,
                                                   float* __restrict__ d_drot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_dyn) return;
  const int64_t g = idx[j];
  if (g < 0 || g >= n) return;  // out-of-range index: ignored
  if (dmean)
    for (int i = 0; i < 3; i++) d_dpos[(int64_t)i * n_dyn + j] += dmean[i * (int64_t)stride + g];
  if (!dquat) return;
  double qc[4], s[4], d[4], e[4], qn = 0.0, sn = 0.0;
  for (int i = 0; i < 4; i++) {
    qc[i] = quat[i * (int64_t)stride + g];
    s[i] = drot[(int64_t)i * n_dyn + j];
    d[i] = dquat[i * (int64_t)stride + g];
    qn += qc[i] * qc[i];
    sn += s[i] * s[i];
  }
  qn = sqrt(qn);
  sn = sqrt(sn);
  qc[0] /= qn;
  for (int i = 1; i < 4; i++) qc[i] = -qc[i] / qn;  // conjugate of the unit quaternion
  qmul(qc, d, e);
  double dot = 0.0;
  for (int i = 0; i < 4; i++) { s[i] /= sn; dot += s[i] * e[i]; }
  for (int i = 0; i < 4; i++) d_drot[(int64_t)i * n_dyn + j] += (float)((e[i] - s[i] * dot) / sn);
}

// ---- Adam ------------------------------------------------------------------------------------
constexpr int kAdamPerBlock = 1024;  // elements per block

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int64_t blk = blockIdx.x;
  int gi = 0;
  while (gi + 1 < a.n_groups && blk >= a.g[gi + 1].block_begin) gi++;
  const AdamGroupK& G = a.g[gi];
  const int64_t base = (blk - G.block_begin) * kAdamPerBlock;
  const float omb1 = 1.f - a.b1, omb2 = 1.f - a.b2;
  float bc1 = a.bc1, bc2 = a.bc2;
  if (a.d_step) {
    const double st = (double)*a.d_step;
    bc1 = (float)(1.0 - pow((double)a.b1, st));
    bc2 = (float)(1.0 - pow((double)a.b2, st));
  }
  for (int k = threadIdx.x; k < kAdamPerBlock; k += blockDim.x) {
    const int64_t i = base + k;
    if (i >= G.n) break;
    const float g = G.g[i];
    const float m = a.b1 * G.m[i] + omb1 * g;
    const float v = a.b2 * G.v[i] + omb2 * g * g;
    G.m[i] = m;
    G.v[i] = v;
    const float mh = m / bc1, vh = v / bc2;
    G.p[i] -= G.lr * mh / (sqrtf(vh) + a.eps);
  }
}

// ---- L1 + error map ---------------------------------------------------------------------------
constexpr int kL1PerBlock = 2048;

__global__ __launch_bounds__(256) void k_l1(L1Args a, float* __restrict__ loss) {
  __shared__ float s_w[4];
  const int64_t blk = blockIdx.x;
  int vi = 0;
  while (vi + 1 < a.nv && blk >= a.v[vi + 1].block_begin) vi++;
  const L1View& V = a.v[vi];
  const float sc = a.scale / (3.0f * (float)V.hw);
  const int64_t base = (blk - V.block_begin) * kL1PerBlock;
  float acc = 0.f;
  for (int k = threadIdx.x; k < kL1PerBlock; k += blockDim.x) {
    const int64_t p = base + k;
    if (p >= V.hw) break;
    float e = 0.f;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const float d = V.render[c * V.hw + p] - V.target[c * V.hw + p];
      V.dl[c * V.hw + p] = d > 0.f ? sc : (d < 0.f ? -sc : 0.f);
      e += fabsf(d);
    }
    if (V.err) V.err[p] = e * (1.0f / 3.0f);
    acc += e;
  }
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (s_w[0] + s_w[1] + s_w[2] + s_w[3]) * sc);
}

// ---- densification ----------------------------------------------------------------------------
// Alg. 1: [P, 1] T with T the full (row-vector) projection built from the intrinsics; pixel
// x = Round(0.5((x_norm + 1) W - 1)), y likewise with y_norm and H, Round(z) = floor(z + 0.5).
// Columns 0 (x), 1 (y) and 3 (homogeneous) of T, rows P0, P1, P2, 1, for one camera:
__device__ void alg1_columns(const CamK& c, double* T /* [3][4] */) {
#pragma clang fp contract(off)
  const double W = (double)c.W, H = (double)c.H;
  const double sx = (2.0 * (double)c.fx) / W, sy = (2.0 * (double)c.fy) / H;
  const double kx = (2.0 * (double)c.cx + 1.0) / W - 1.0;
  const double ky = (2.0 * (double)c.cy + 1.0) / H - 1.0;
  for (int i = 0; i < 3; i++) {
    T[i] = sx * (double)c.R[i] + kx * (double)c.R[6 + i];
    T[4 + i] = sy * (double)c.R[3 + i] + ky * (double)c.R[6 + i];
    T[8 + i] = (double)c.R[6 + i];
  }
  T[3] = sx * (double)c.t[0] + kx * (double)c.t[2];
  T[7] = sy * (double)c.t[1] + ky * (double)c.t[2];
  T[11] = (double)c.t[2];
}

__device__ bool alg1_pixel(const double* T, int Wi, int Hi, double X, double Y, double Z, int& xn, int& yn) {
#pragma clang fp contract(off)
  const double W = (double)Wi, H = (double)Hi;
  const double hx = ((X * T[0] + Y * T[1]) + Z * T[2]) + T[3];
  const double hy = ((X * T[4] + Y * T[5]) + Z * T[6]) + T[7];
  const double hw = ((X * T[8] + Y * T[9]) + Z * T[10]) + T[11];
  if (!(hw > 0.0)) return false;
  const double xnorm = hx / hw, ynorm = hy / hw;
  const double xf = floor(0.5 * ((xnorm + 1.0) * W - 1.0) + 0.5);
  const double yf = floor(0.5 * ((ynorm + 1.0) * H - 1.0) + 0.5);
  if (xf < 0.0 || yf < 0.0 || xf >= W || yf >= H) return false;
  xn = (int)xf;
  yn = (int)yf;
  return true;
}

// Selection (Alg. 1): a workgroup takes 64 base Gaussians, its wave w the views w, w + 4, ...
// (the view index stays uniform over a wave); the score is the largest error at the Gaussian's
// pixel over the views that see it.  Wave 0 combines the four waves and writes, per Gaussian, the
// membership flag and the rank key (complemented score bits: ascending key = descending score);
// a scan then packs the members in index order, so a stable sort on the 32-bit key alone ranks
// them with ties by index.
constexpr int kSelWaves = 4;
__global__ __launch_bounds__(64 * kSelWaves) void k_densify_select(SceneK s, DensifyArgs a,
                                                                   const float* __restrict__ gsum,
                                                                   const int32_t* __restrict__ gcnt, int n_base,
                                                                   uint32_t* __restrict__ keep,
                                                                   uint32_t* __restrict__ score_key) {
  __shared__ double s_T[DASS_MAX_VIEWS][12];
  __shared__ float s_score[kSelWaves][64];
  __shared__ int s_ie[kSelWaves][64];
  for (int v = threadIdx.x; v < a.nv; v += blockDim.x) alg1_columns(a.cams[v], s_T[v]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = blockIdx.x * 64 + lane;
  bool in_err = false;
  float score = 0.f;
  if (g < n_base) {
    const double X = s.mean[g], Y = s.mean[(int64_t)s.stride + g], Z = s.mean[2 * (int64_t)s.stride + g];
    for (int v = wave; v < a.nv; v += kSelWaves) {
      int x, y;
      if (alg1_pixel(s_T[v], a.cams[v].W, a.cams[v].H, X, Y, Z, x, y)) {
        const float e = a.err[v][(int64_t)y * a.cams[v].W + x];
        in_err |= e > a.gamma_err;
        score = fmaxf(score, e);
      }
    }
  }
  s_score[wave][lane] = score;
  s_ie[wave][lane] = in_err ? 1 : 0;
  __syncthreads();
  if (wave != 0) return;
  int ie = 0;
#pragma unroll
  for (int w = 0; w < kSelWaves; w++) {
    score = fmaxf(score, s_score[w][lane]);
    ie |= s_ie[w][lane];
  }
  if (g >= n_base) return;
  const int32_t c = gcnt[g];
  const float gbar = c > 0 ? gsum[g] / (float)c : 0.f;
  const bool in_s = (gbar > a.tau_pos) || (ie != 0 && gbar > a.tau_err);
  keep[g] = in_s ? 1u : 0u;
  score_key[g] = ~__float_as_uint(score);
}

// members packed in index order: key and Gaussian index at the member's rank in the scan
__global__ __launch_bounds__(256) void k_densify_pack(int n_base, const uint32_t* __restrict__ keep,
                                                      const uint64_t* __restrict__ pos,
                                                      const uint32_t* __restrict__ score_key,
                                                      uint32_t* __restrict__ sel_keys, uint32_t* __restrict__ sel_vals,
                                                      uint32_t* __restrict__ d_count) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g == 0) *d_count = (uint32_t)pos[n_base];
  if (g >= n_base || !keep[g]) return;
  sel_keys[pos[g]] = score_key[g];
  sel_vals[pos[g]] = (uint32_t)g;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// A quad of lanes per child, so the float64 chains run side by side: lane i < 3 forms the
// child's i-th normal draw and scale, lane 3 copies the quaternion and the opacity logit; every
// lane then forms its mean component from the quad's draws (the same products and sums as
// written for one thread) and copies a quarter of the SH planes.
__global__ __launch_bounds__(256) void k_densify_spawn(float* __restrict__ mean, float* __restrict__ quat,
                                                       float* __restrict__ log_scale, float* __restrict__ logit,
                                                       float* __restrict__ sh, int n_sh, int stride, int n, int capacity,
                                                       const uint32_t* __restrict__ sel_idx,
                                                       const uint32_t* __restrict__ d_count, int k_max, uint64_t seed,
                                                       int32_t* __restrict__ n_appended) {
  const uint32_t ns = *d_count;
  const int room = capacity - n;
  const int n_app = ns == 0 ? 0 : (k_max < room ? k_max : room);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = tid >> 2, l = tid & 3;
  if (tid == 0 && n_appended) *n_appended = n_app < 0 ? 0 : n_app;
  if (j >= n_app) return;  // uniform over a quad (n_app whole children)
  const int64_t p = (int64_t)sel_idx[j % ns];  // parents in rank order
  const int64_t c = (int64_t)n + j;
  const int64_t st = stride;
  // lane l < 3: scale l and normal draw l (Box-Muller on draws 4j .. 4j+3: z0, z1 from the
  // first pair, z2 from the second)
  double scl = 0.0, zl = 0.0;
  if (l < 3) {
    const double TWO_PI = 6.283185307179586476925;
    const uint64_t d0 = 4ull * (uint64_t)j + (l == 2 ? 2u : 0u);
    const double ua = 1.0 - u01(splitmix64(seed, d0)), ub = u01(splitmix64(seed, d0 + 1));
    const double r = sqrt(-2.0 * log(ua));
    zl = l == 1 ? r * sin(TWO_PI * ub) : r * cos(TWO_PI * ub);
    scl = exp((double)log_scale[l * st + p]);
  }
  const int q0 = (int)(threadIdx.x & 63) & ~3;  // the quad's first lane in the wave
  double sc[3], z[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    sc[k] = __shfl(scl, q0 + k, 64);
    z[k] = __shfl(zl, q0 + k, 64);
  }
  if (l < 3) {
    double q[4], qn = 0.0;
    for (int i = 0; i < 4; i++) {
      q[i] = quat[i * st + p];
      qn += q[i] * q[i];
    }
    qn = sqrt(qn);
    for (int i = 0; i < 4; i++) q[i] /= qn;
    const double w = q[0], x = q[1], y = q[2], zq = q[3];
    const double R[9] = {1.0 - 2.0 * (y * y + zq * zq), 2.0 * (x * y - w * zq), 2.0 * (x * zq + w * y),
                         2.0 * (x * y + w * zq), 1.0 - 2.0 * (x * x + zq * zq), 2.0 * (y * zq - w * x),
                         2.0 * (x * zq - w * y), 2.0 * (y * zq + w * x), 1.0 - 2.0 * (x * x + y * y)};
    const int i = l;
    const double off = R[i * 3 + 0] * sc[0] * z[0] + R[i * 3 + 1] * sc[1] * z[1] + R[i * 3 + 2] * sc[2] * z[2];
    mean[i * st + c] = (float)((double)mean[i * st + p] + off);
    const double ln16 = 0.47000362924573558;  // ln 1.6
    log_scale[i * st + c] = (float)((double)log_scale[i * st + p] - ln16);
  } else {
    for (int i = 0; i < 4; i++) quat[i * st + c] = quat[i * st + p];
    logit[c] = logit[p];
  }
  // the child row c >= n never overlaps a parent row p < n: a quarter of the planes per lane,
  // loaded together, then stored
  float shv[12];
#pragma unroll
  for (int k = 0; k < 12; k++) shv[k] = 4 * k + l < n_sh ? sh[(int64_t)(4 * k + l) * st + p] : 0.f;
#pragma unroll
  for (int k = 0; k < 12; k++)
    if (4 * k + l < n_sh) sh[(int64_t)(4 * k + l) * st + c] = shv[k];
}

}  // namespace

void launch_shift_fwd(const SceneK& in, float* out_mean, float* out_quat, const int32_t* dyn_idx, int n_dyn,
                      const float* dpos, const float* drot, hipStream_t st) {
  if (in.n > 0)
    k_copy_mq<<<(in.n + 255) / 256, 256, 0, st>>>(in.mean, in.quat, out_mean, out_quat, in.n, in.stride);
  if (n_dyn > 0)
    k_shift_fwd<<<(n_dyn + 255) / 256, 256, 0, st>>>(in.mean, in.quat, out_mean, out_quat, in.stride, in.n, dyn_idx,
                                                      n_dyn, dpos, drot);
}

void launch_shift_adj(const SceneK& in, const float* dmean, const float* dquat, const int32_t* dyn_idx, int n_dyn,
                      const float* drot, float* d_dpos, float* d_drot, hipStream_t st) {
  if (n_dyn > 0)
    k_shift_adj<<<(n_dyn + 255) / 256, 256, 0, st>>>(in.quat, dmean, dquat, in.stride, in.n, dyn_idx, n_dyn, drot,
                                                      d_dpos, d_drot);
}

__global__ void k_step_increment(int32_t* s) { *s += 1; }

void launch_step_increment(int32_t* d_step, hipStream_t st) { k_step_increment<<<1, 1, 0, st>>>(d_step); }

void launch_adam(const AdamArgs& a, int64_t total_blocks, hipStream_t st) {
  if (total_blocks > 0) k_adam<<<(unsigned)total_blocks, 256, 0, st>>>(a);
}

void launch_l1(const L1Args& a, int64_t total_blocks, float* loss, hipStream_t st) {
  if (total_blocks > 0) k_l1<<<(unsigned)total_blocks, 256, 0, st>>>(a, loss);
}

void launch_densify_select(const SceneK& s, const DensifyArgs& a, const float* gsum, const int32_t* gcnt, int n_base,
                           uint32_t* keep, uint64_t* pos, uint64_t* scan_tmp, uint32_t* score_key, uint32_t* sel_keys,
                           uint32_t* sel_vals, uint32_t* d_count, hipStream_t st) {
  if (n_base <= 0) return;  // *d_count stays at the zero the caller wrote
  k_densify_select<<<(n_base + 63) / 64, 64 * kSelWaves, 0, st>>>(s, a, gsum, gcnt, n_base, keep, score_key);
  scan_u32_to_u64(keep, pos, n_base, scan_tmp, st);
  k_densify_pack<<<(n_base + 255) / 256, 256, 0, st>>>(n_base, keep, pos, score_key, sel_keys, sel_vals, d_count);
}

void launch_densify_spawn(float* mean, float* quat, float* log_scale, float* logit, float* sh, int n_planes_sh,
                          int stride, int n, int capacity, const uint32_t* sel_idx, const uint32_t* d_count, int k_max,
                          uint64_t seed, int32_t* n_appended, hipStream_t st) {
  const int blocks = k_max > 0 ? (int)(((int64_t)k_max * 4 + 255) / 256) : 1;
  k_densify_spawn<<<blocks, 256, 0, st>>>(mean, quat, log_scale, logit, sh, n_planes_sh, stride, n, capacity, sel_idx,
                                           d_count, k_max, seed, n_appended);
}

int adam_per_block() { return kAdamPerBlock; }
int l1_per_block() { return kL1PerBlock; }

}  // namespace dass
