// Projection of 3D Gaussians into every view (App. A.1) and its adjoint.
//
// One thread per Gaussian walks all views of the call, so the Gaussian's 59 parameters are
// read from HBM once (coalesced structure-of-arrays planes) and kept in registers.  The
// arithmetic is fp64: it is a few hundred flops per Gaussian-view (negligible next to the
// blend), and it makes the integer decisions taken here -- cull, radius, tile rectangle,
// float32 depth bits of the key -- agree with an fp64 definition except within ~1e-15 of a
// boundary.  The pixel-space mean is handed to the fp32 blend as hi + lo floats.
#include "dass_internal.h"

namespace dass {
namespace {

// Real orthonormal spherical harmonics up to degree 3 (no Condon-Shortley sign), index
// k = l*l + l + m, evaluated at a unit direction; optional gradient w.r.t. (x, y, z) of the
// polynomial form.
constexpr double kY0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double kY2b = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double kY2c = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double kY3a = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double kY3b = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double kY3c = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double kY3d = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double kY3e = 1.445305721320277;    // sqrt(105/pi)/4

template <int DEG, bool GRAD, typename F = double>
__device__ __forceinline__ void sh_basis(F x, F y, F z, F* Y, F* gx, F* gy, F* gz) {
  Y[0] = F(kY0);
  if (GRAD) { gx[0] = gy[0] = gz[0] = F(0.0); }
  if (DEG >= 1) {
    Y[1] = F(kY1) * y; Y[2] = F(kY1) * z; Y[3] = F(kY1) * x;
    if (GRAD) {
      gx[1] = F(0.0); gy[1] = F(kY1); gz[1] = F(0.0);
      gx[2] = F(0.0); gy[2] = F(0.0); gz[2] = F(kY1);
      gx[3] = F(kY1); gy[3] = F(0.0); gz[3] = F(0.0);
    }
  }
  if (DEG >= 2) {
    F xx = x * x, yy = y * y, zz = z * z;
    Y[4] = F(kY2a) * x * y;
    Y[5] = F(kY2a) * y * z;
    Y[6] = F(kY2b) * (F(2.0) * zz - xx - yy);
    Y[7] = F(kY2a) * x * z;
    Y[8] = F(kY2c) * (xx - yy);
    if (GRAD) {
      gx[4] = F(kY2a) * y; gy[4] = F(kY2a) * x; gz[4] = F(0.0);
      gx[5] = F(0.0); gy[5] = F(kY2a) * z; gz[5] = F(kY2a) * y;
      gx[6] = -F(2.0) * F(kY2b) * x; gy[6] = -F(2.0) * F(kY2b) * y; gz[6] = F(4.0) * F(kY2b) * z;
      gx[7] = F(kY2a) * z; gy[7] = F(0.0); gz[7] = F(kY2a) * x;
      gx[8] = F(2.0) * F(kY2c) * x; gy[8] = -F(2.0) * F(kY2c) * y; gz[8] = F(0.0);
    }
  }
  if (DEG >= 3) {
    F xx = x * x, yy = y * y, zz = z * z;
    Y[9] = F(kY3a) * y * (F(3.0) * xx - yy);
    Y[10] = F(kY3b) * x * y * z;
    Y[11] = F(kY3c) * y * (F(4.0) * zz - xx - yy);
    Y[12] = F(kY3d) * z * (F(2.0) * zz - F(3.0) * xx - F(3.0) * yy);
    Y[13] = F(kY3c) * x * (F(4.0) * zz - xx - yy);
    Y[14] = F(kY3e) * z * (xx - yy);
    Y[15] = F(kY3a) * x * (xx - F(3.0) * yy);
    if (GRAD) {
      gx[9] = F(kY3a) * F(6.0) * x * y; gy[9] = F(kY3a) * F(3.0) * (xx - yy); gz[9] = F(0.0);
      gx[10] = F(kY3b) * y * z; gy[10] = F(kY3b) * x * z; gz[10] = F(kY3b) * x * y;
      gx[11] = -F(2.0) * F(kY3c) * x * y; gy[11] = F(kY3c) * (F(4.0) * zz - xx - F(3.0) * yy); gz[11] = F(8.0) * F(kY3c) * y * z;
      gx[12] = -F(6.0) * F(kY3d) * x * z; gy[12] = -F(6.0) * F(kY3d) * y * z; gz[12] = F(kY3d) * (F(6.0) * zz - F(3.0) * xx - F(3.0) * yy);
      gx[13] = F(kY3c) * (F(4.0) * zz - F(3.0) * xx - yy); gy[13] = -F(2.0) * F(kY3c) * x * y; gz[13] = F(8.0) * F(kY3c) * x * z;
      gx[14] = F(2.0) * F(kY3e) * x * z; gy[14] = -F(2.0) * F(kY3e) * y * z; gz[14] = F(kY3e) * (xx - yy);
      gx[15] = F(kY3a) * F(3.0) * (xx - yy); gy[15] = -F(6.0) * F(kY3a) * x * y; gz[15] = F(0.0);
    }
  }
}

// d/d(x,y,z) of sum_k w_k Y_k(x,y,z) (the polynomial forms above), without materialising the
// per-basis gradient arrays.
template <int DEG, typename F = double>
__device__ __forceinline__ void sh_weighted_grad(F x, F y, F z, const F* w, F& gx, F& gy, F& gz) {
  gx = gy = gz = F(0.0);
  if (DEG >= 1) {
    gy += w[1] * F(kY1);
    gz += w[2] * F(kY1);
    gx += w[3] * F(kY1);
  }
  if (DEG >= 2) {
    gx += w[4] * F(kY2a) * y + w[6] * (-F(2.0) * F(kY2b) * x) + w[7] * F(kY2a) * z + w[8] * (F(2.0) * F(kY2c) * x);
    gy += w[4] * F(kY2a) * x + w[5] * F(kY2a) * z + w[6] * (-F(2.0) * F(kY2b) * y) + w[8] * (-F(2.0) * F(kY2c) * y);
    gz += w[5] * F(kY2a) * y + w[6] * (F(4.0) * F(kY2b) * z) + w[7] * F(kY2a) * x;
  }
  if (DEG >= 3) {
    const F xx = x * x, yy = y * y, zz = z * z;
    gx += w[9] * (F(6.0) * F(kY3a) * x * y) + w[10] * (F(kY3b) * y * z) + w[11] * (-F(2.0) * F(kY3c) * x * y) +
          w[12] * (-F(6.0) * F(kY3d) * x * z) + w[13] * (F(kY3c) * (F(4.0) * zz - F(3.0) * xx - yy)) +
          w[14] * (F(2.0) * F(kY3e) * x * z) + w[15] * (F(3.0) * F(kY3a) * (xx - yy));
    gy += w[9] * (F(3.0) * F(kY3a) * (xx - yy)) + w[10] * (F(kY3b) * x * z) + w[11] * (F(kY3c) * (F(4.0) * zz - xx - F(3.0) * yy)) +
          w[12] * (-F(6.0) * F(kY3d) * y * z) + w[13] * (-F(2.0) * F(kY3c) * x * y) + w[14] * (-F(2.0) * F(kY3e) * y * z) +
          w[15] * (-F(6.0) * F(kY3a) * x * y);
    gz += w[10] * (F(kY3b) * x * y) + w[11] * (F(8.0) * F(kY3c) * y * z) + w[12] * (F(kY3d) * (F(6.0) * zz - F(3.0) * xx - F(3.0) * yy)) +
          w[13] * (F(8.0) * F(kY3c) * x * z) + w[14] * (F(kY3e) * (xx - yy));
  }
}

// View-independent part of one Gaussian.
struct GaussD {
  double mu[3], qhat[4], qn, s[3], Rq[9], M[9], Sig[6], o;  // Sig: xx, xy, xz, yy, yz, zz
  bool ok;
};

__device__ __forceinline__ void load_gaussian(const SceneK& sc, int g, GaussD& G) {
  const int64_t st = sc.stride;
  for (int i = 0; i < 3; i++) G.mu[i] = (double)sc.mean[i * st + g];
  double q[4];
  for (int i = 0; i < 4; i++) q[i] = (double)sc.quat[i * st + g];
  G.qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  G.ok = G.qn > 0.0;
  double inv = G.ok ? 1.0 / G.qn : 0.0;
  for (int i = 0; i < 4; i++) G.qhat[i] = q[i] * inv;
  for (int i = 0; i < 3; i++) G.s[i] = exp((double)sc.log_scale[i * st + g]);
  double w = G.qhat[0], x = G.qhat[1], y = G.qhat[2], z = G.qhat[3];
  double* R = G.Rq;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) G.M[i * 3 + j] = R[i * 3 + j] * G.s[j];
  const double* M = G.M;
  G.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  G.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  G.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  G.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  G.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  G.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  G.o = 1.0 / (1.0 + exp(-(double)sc.logit[g]));
}

// What the per-view projection needs of a Gaussian.
struct GaussLite {
  double mu[3], Sig[6];
  bool ok;
};

// View-dependent part.
struct ViewD {
  double t[3], limx, limy, txc, tyc, J0, J2, J4, J5;  // J = [[J0, 0, J2], [0, J4, J5]]
  double T[6];                                      // J W
  double a, b, c, det, A, B, C, u, v;
  bool clipx, clipy, visible;
  int radius, x0, y0, x1, y1;
  uint32_t depth_bits;
};

// Half-FOV clip limits of the tangents t_x / t_z and t_y / t_z (1.3 times the half-FOV tangent).
__device__ __forceinline__ void clip_limits(const CamK& cam, double& limx, double& limy) {
#pragma clang fp contract(off)
  limx = kClip * ((double)cam.W / (2.0 * (double)cam.fx));
  limy = kClip * ((double)cam.H / (2.0 * (double)cam.fy));
}

// Views' clip limits computed once per workgroup (threads 0..nv-1; the caller synchronises).
struct ClipTable {
  double lim[DASS_MAX_VIEWS][2];
};

__device__ __forceinline__ void fill_clip_table(const CamsK& cams, int nv, ClipTable& t) {
  for (int v = threadIdx.x + threadIdx.y * blockDim.x; v < nv; v += blockDim.x * blockDim.y)
    clip_limits(cams.c[v], t.lim[v][0], t.lim[v][1]);
}

template <typename GT>
__device__ __forceinline__ void project_view(const GT& G, const CamK& cam, double limx, double limy, ViewD& V) {
#pragma clang fp contract(off)
  double W[9];
  for (int i = 0; i < 9; i++) W[i] = (double)cam.R[i];
  // camera space, fixed evaluation order, no fused multiply-add (compared bit-for-bit)
  for (int i = 0; i < 3; i++)
    V.t[i] = ((W[i * 3 + 0] * G.mu[0] + W[i * 3 + 1] * G.mu[1]) + W[i * 3 + 2] * G.mu[2]) + (double)cam.t[i];
  const double tx = V.t[0], ty = V.t[1], tz = V.t[2];
  V.visible = false;
  V.radius = 0;
  V.x0 = V.y0 = V.x1 = V.y1 = 0;
  V.depth_bits = 0xFFFFFFFFu;
  if (!G.ok || !(tz > kNearZ)) return;
  const double fx = (double)cam.fx, fy = (double)cam.fy;
  V.limx = limx;
  V.limy = limy;
  const double rx = tx / tz, ry = ty / tz;
  V.clipx = (rx < -V.limx) || (rx > V.limx);
  V.clipy = (ry < -V.limy) || (ry > V.limy);
  V.txc = fmin(fmax(rx, -V.limx), V.limx) * tz;
  V.tyc = fmin(fmax(ry, -V.limy), V.limy) * tz;
  const double tz2 = tz * tz;
  V.J0 = fx / tz;
  V.J2 = -fx * V.txc / tz2;
  V.J4 = fy / tz;
  V.J5 = -fy * V.tyc / tz2;
  for (int j = 0; j < 3; j++) {
    V.T[j] = V.J0 * W[j] + V.J2 * W[6 + j];
    V.T[3 + j] = V.J4 * W[3 + j] + V.J5 * W[6 + j];
  }
  // Sigma_2D = T Sigma T^T + dilation
  const double* S = G.Sig;
  double TS[6];
  for (int i = 0; i < 2; i++) {
    const double* Ti = V.T + 3 * i;
    TS[3 * i + 0] = Ti[0] * S[0] + Ti[1] * S[1] + Ti[2] * S[2];
    TS[3 * i + 1] = Ti[0] * S[1] + Ti[1] * S[3] + Ti[2] * S[4];
    TS[3 * i + 2] = Ti[0] * S[2] + Ti[1] * S[4] + Ti[2] * S[5];
  }
  V.a = (TS[0] * V.T[0] + TS[1] * V.T[1] + TS[2] * V.T[2]) + kDilation;
  V.b = TS[0] * V.T[3] + TS[1] * V.T[4] + TS[2] * V.T[5];
  V.c = (TS[3] * V.T[3] + TS[4] * V.T[4] + TS[5] * V.T[5]) + kDilation;
  V.det = V.a * V.c - V.b * V.b;
  if (!(V.det > 0.0)) return;
  V.A = V.c / V.det;
  V.B = -V.b / V.det;
  V.C = V.a / V.det;
  const double mid = 0.5 * (V.a + V.c);
  const double d = 0.5 * (V.a - V.c);
  const double lmax = mid + sqrt(fmax(d * d + V.b * V.b, 0.0));
  double r = ceil(3.0 * sqrt(lmax));
  r = fmin(r, 1.0e7);
  V.radius = (int)r;
  V.u = ((fx * tx) / tz) + (double)cam.cx;
  V.v = ((fy * ty) / tz) + (double)cam.cy;
  // tile edges are powers of two (16, 32 or 64), so scaling by the edge's exponent is the exact
  // quotient
  const double tw = (double)cam.tw, th = (double)cam.th;
  const int ew = __builtin_ctz((unsigned)cam.tw), eh = __builtin_ctz((unsigned)cam.th);
  const double fx0 = floor(ldexp(V.u - r, -ew));
  const double fx1 = floor(ldexp((V.u + r) + (tw - 1.0), -ew));
  const double fy0 = floor(ldexp(V.v - r, -eh));
  const double fy1 = floor(ldexp((V.v + r) + (th - 1.0), -eh));
  V.x0 = (int)fmin(fmax(fx0, 0.0), (double)cam.TX);
  V.x1 = (int)fmin(fmax(fx1, 0.0), (double)cam.TX);
  V.y0 = (int)fmin(fmax(fy0, 0.0), (double)cam.TY);
  V.y1 = (int)fmin(fmax(fy1, 0.0), (double)cam.TY);
  V.visible = (V.radius > 0) && (V.x1 > V.x0) && (V.y1 > V.y0);
  V.depth_bits = V.visible ? __float_as_uint((float)tz) : 0xFFFFFFFFu;
}

// What the adjoint needs of a (view, Gaussian) that the forward found visible: the camera-space
// mean and the clip decisions and clamped tangents exactly as the forward computes them (so the
// adjoint takes the same branch of the clamp), then the Jacobian, T = J W and the conic from
// reciprocals of tz and det (gradients: a rounding apart from the forward's quotients).
struct ViewAdj {
  double t[3], limx, limy, txc, tyc, itz, J0, J2, J4, J5, T[6], A, B, C;
  bool clipx, clipy;
};

__device__ __forceinline__ void adjoint_view(const GaussLite& G, const CamK& cam, double limx, double limy,
                                             ViewAdj& V) {
  double W[9];
  for (int i = 0; i < 9; i++) W[i] = (double)cam.R[i];
  const double fx = (double)cam.fx, fy = (double)cam.fy;
  {
#pragma clang fp contract(off)
    for (int i = 0; i < 3; i++)
      V.t[i] = ((W[i * 3 + 0] * G.mu[0] + W[i * 3 + 1] * G.mu[1]) + W[i * 3 + 2] * G.mu[2]) + (double)cam.t[i];
    V.limx = limx;
    V.limy = limy;
    const double rx = V.t[0] / V.t[2], ry = V.t[1] / V.t[2];
    V.clipx = (rx < -V.limx) || (rx > V.limx);
    V.clipy = (ry < -V.limy) || (ry > V.limy);
    V.txc = fmin(fmax(rx, -V.limx), V.limx) * V.t[2];
    V.tyc = fmin(fmax(ry, -V.limy), V.limy) * V.t[2];
  }
  V.itz = 1.0 / V.t[2];
  const double itz2 = V.itz * V.itz;
  V.J0 = fx * V.itz;
  V.J2 = -fx * V.txc * itz2;
  V.J4 = fy * V.itz;
  V.J5 = -fy * V.tyc * itz2;
  for (int j = 0; j < 3; j++) {
    V.T[j] = V.J0 * W[j] + V.J2 * W[6 + j];
    V.T[3 + j] = V.J4 * W[3 + j] + V.J5 * W[6 + j];
  }
  const double* S = G.Sig;
  double TS[6];
  for (int i = 0; i < 2; i++) {
    const double* Ti = V.T + 3 * i;
    TS[3 * i + 0] = Ti[0] * S[0] + Ti[1] * S[1] + Ti[2] * S[2];
    TS[3 * i + 1] = Ti[0] * S[1] + Ti[1] * S[3] + Ti[2] * S[4];
    TS[3 * i + 2] = Ti[0] * S[2] + Ti[1] * S[4] + Ti[2] * S[5];
  }
  const double a = (TS[0] * V.T[0] + TS[1] * V.T[1] + TS[2] * V.T[2]) + kDilation;
  const double b = TS[0] * V.T[3] + TS[1] * V.T[4] + TS[2] * V.T[5];
  const double c = (TS[3] * V.T[3] + TS[4] * V.T[4] + TS[5] * V.T[5]) + kDilation;
  const double rdet = 1.0 / (a * c - b * b);
  V.A = c * rdet;
  V.B = -b * rdet;
  V.C = a * rdet;
}

template <int DEG, typename GT>
__device__ __forceinline__ void colour(const GT& G, const CamK& cam, const float* shc, double* rgb_pre,
                                       double* dhat, double& dn) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double dir[3];
  for (int i = 0; i < 3; i++) dir[i] = G.mu[i] - (double)cam.campos[i];
  dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  const double inv = dn > 0.0 ? 1.0 / dn : 0.0;
  for (int i = 0; i < 3; i++) dhat[i] = dir[i] * inv;
  double Y[16];
  sh_basis<DEG, false, double>(dhat[0], dhat[1], dhat[2], Y, nullptr, nullptr, nullptr);
#pragma unroll
  for (int ch = 0; ch < 3; ch++) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) acc += (double)shc[k * 3 + ch] * Y[k];
    rgb_pre[ch] = acc + 0.5;
  }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(SceneK sc, CamsK cams, int nv, Rec* __restrict__ rec,
                                                    uint2* __restrict__ rect,
                                                    uint8_t* __restrict__ vis, uint64_t* __restrict__ dkey,
                                                    uint32_t* __restrict__ dval) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ ClipTable s_clip;
  fill_clip_table(cams, nv, s_clip);
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sc.n) return;
  GaussD G;
  load_gaussian(sc, g, G);
  float shc[3 * K];
#pragma unroll
  for (int k = 0; k < 3 * K; k++) shc[k] = sc.sh[(int64_t)k * sc.stride + g];
  // views blockIdx.y, blockIdx.y + gridDim.y, ...: a Gaussian's views are split over gridDim.y
  // threads (each forms the Gaussian's 3D covariance itself), so the launch has enough waves
  for (int v = blockIdx.y; v < nv; v += gridDim.y) {
    const CamK& cam = cams.c[v];
    const int64_t i = (int64_t)v * sc.n + g;
    ViewD V;
    project_view(G, cam, s_clip.lim[v][0], s_clip.lim[v][1], V);
    Rec r;
    if (V.visible) {
      double rgb_pre[3], dhat[3], dn;
      colour<DEG>(G, cam, shc, rgb_pre, dhat, dn);
      const float uh = (float)V.u, vh = (float)V.v;
      r.r0 = make_float4(uh, vh, (float)(V.u - (double)uh), (float)(V.v - (double)vh));
      r.r1 = make_float4((float)V.A, (float)V.B, (float)V.C, (float)G.o);
      r.r2 = make_float4((float)fmax(rgb_pre[0], 0.0), (float)fmax(rgb_pre[1], 0.0),
                         (float)fmax(rgb_pre[2], 0.0), (float)V.t[2]);
      vis[i] = (uint8_t)(8u | (r.r2.x > 0.f ? 1u : 0u) | (r.r2.y > 0.f ? 2u : 0u) | (r.r2.z > 0.f ? 4u : 0u));
      rect[i] = make_uint2((uint32_t)V.x0 | ((uint32_t)V.y0 << 16), (uint32_t)V.x1 | ((uint32_t)V.y1 << 16));
    } else {
      r.r0 = r.r1 = r.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
      vis[i] = 0;
      rect[i] = make_uint2(0, 0);
    }
    rec[i] = r;
    // the depth is a positive float (or the all-ones sentinel), so 31 bits order it
    dkey[i] = ((uint64_t)v << 31) | (uint64_t)(V.depth_bits & 0x7FFFFFFFu);
    dval[i] = (uint32_t)g;
  }
}

// ---------------------------------------------------------------------------------------------
// Adjoint.  Per Gaussian: for every view where it is visible, read the per-view 2D gradient
// (du, dv, dA, dB, dC, do, dr, dg, db) at its sorted position, chain it back through the
// conic inverse, the EWA projection, the pixel mean, the colour and the opacity; quantities
// linear in the view (dSigma, dlogit) are summed over views first and chained once.
// ---------------------------------------------------------------------------------------------
constexpr int kBwdSplit = 4;  // lanes per Gaussian in the adjoint (views split round-robin)

__device__ __forceinline__ float quad_sumf(float x) {
  x += __shfl_xor(x, 1, 64);
  x += __shfl_xor(x, 2, 64);
  return x;
}

// Geometry part: pixel mean and conic back to mean, quaternion and log-scale; opacity.  A
// workgroup takes 64 Gaussians; its wave w takes the views w, w + 4, ... (the view index stays
// uniform over a wave, so camera data are scalar loads); wave 0 adds the other waves' sums
// and chains them back to the parameters with every lane busy.
constexpr int kAdjWaves = 4;
__global__ __launch_bounds__(64 * kAdjWaves) void k_preprocess_bwd_geom(SceneK sc, CamsK cams, int nv,
                                                                        const uint8_t* __restrict__ vis,
                                                                        const float* __restrict__ g2d, dass_grads gr,
                                                                        float* __restrict__ gradnorm,
                                                                        int32_t* __restrict__ gcount) {
  __shared__ double s_part[kAdjWaves - 1][11][64];  // dmu[3], dSig[6], dop, gnorm of waves 1..3
  __shared__ int s_cnt[kAdjWaves - 1][64];
  __shared__ ClipTable s_clip;
  fill_clip_table(cams, nv, s_clip);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g_raw = blockIdx.x * 64 + lane;
  const bool live = g_raw < sc.n;
  const int g = live ? g_raw : sc.n - 1;
  GaussLite L;
  double o;
  {
    GaussD G;
    load_gaussian(sc, g, G);
    for (int i = 0; i < 3; i++) L.mu[i] = G.mu[i];
    for (int i = 0; i < 6; i++) L.Sig[i] = G.Sig[i];
    L.ok = G.ok;
    o = G.o;
  }
  double dmu[3] = {0.0, 0.0, 0.0};
  double dSig[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double dop = 0.0, gnorm = 0.0;
  int cnt = 0;
  for (int v = wave; v < nv && live; v += kAdjWaves) {
    // the forward's visibility flag of this (view, Gaussian): its projection is not redone
    // where it did not draw
    if (!(vis[(int64_t)v * sc.n + g] & 8u)) continue;
    const CamK& cam = cams.c[v];
    const float* gd = g2d + ((int64_t)v * sc.n + g) * 9;
    float gv[6];  // issued before the projection so that the loads overlap it
#pragma unroll
    for (int i = 0; i < 6; i++) gv[i] = gd[i];
    ViewAdj V;
    adjoint_view(L, cam, s_clip.lim[v][0], s_clip.lim[v][1], V);
    // blend sums of this (view, Gaussian): M = (sum dP dx, sum dP dy, sum dP dx^2, sum dP dx dy,
    // sum dP dy^2, d opacity, d rgb) with dP = dL/d(exponent), exponent = -(A dx^2 + 2B dx dy +
    // C dy^2)/2 and (dx, dy) = mean - pixel, so dL/du = -(A M0 + B M1), dL/dv = -(B M0 + C M1),
    // dL/dA = -M2/2, dL/dB = -M3, dL/dC = -M4/2
    const double A = V.A, B = V.B, C = V.C;
    const double M0 = gv[0], M1 = gv[1];
    const double du = -(A * M0 + B * M1), dv = -(B * M0 + C * M1);
    const double dA = -0.5 * (double)gv[2], dB = -(double)gv[3], dC = -0.5 * (double)gv[4];
    dop += (double)gv[5];
    gnorm += sqrt(du * du + dv * dv);
    cnt++;
    // conic (A, B, C) = inverse of [[a, b], [b, c]]: dSigma2D = -Q G Q with G = [[dA, dB/2], [dB/2, dC]]
    const double hB = 0.5 * dB;
    const double qg00 = A * dA + B * hB, qg01 = A * hB + B * dC;
    const double qg10 = B * dA + C * hB, qg11 = B * hB + C * dC;
    const double da = -(qg00 * A + qg01 * B);
    const double db2 = -(qg00 * B + qg01 * C);  // (0,1) entry of the symmetric matrix gradient
    const double dc = -(qg10 * B + qg11 * C);
    // Sigma_2D = T Sigma T^T: dSigma += T^T G2 T, dT = 2 G2 T Sigma, with G2 = [[da, db2], [db2, dc]]
    const double* T = V.T;
    double G2T[6];
    for (int j = 0; j < 3; j++) {
      G2T[j] = da * T[j] + db2 * T[3 + j];
      G2T[3 + j] = db2 * T[j] + dc * T[3 + j];
    }
    dSig[0] += T[0] * G2T[0] + T[3] * G2T[3];
    dSig[1] += T[0] * G2T[1] + T[3] * G2T[4];
    dSig[2] += T[0] * G2T[2] + T[3] * G2T[5];
    dSig[3] += T[1] * G2T[1] + T[4] * G2T[4];
    dSig[4] += T[1] * G2T[2] + T[4] * G2T[5];
    dSig[5] += T[2] * G2T[2] + T[5] * G2T[5];
    const double* S = L.Sig;
    double dT[6];
    for (int i = 0; i < 2; i++) {
      const double* rr = G2T + 3 * i;
      dT[3 * i + 0] = 2.0 * (rr[0] * S[0] + rr[1] * S[1] + rr[2] * S[2]);
      dT[3 * i + 1] = 2.0 * (rr[0] * S[1] + rr[1] * S[3] + rr[2] * S[4]);
      dT[3 * i + 2] = 2.0 * (rr[0] * S[2] + rr[1] * S[4] + rr[2] * S[5]);
    }
    // T = J W: dJ_ij = sum_k dT_ik W_jk
    double W[9];
    for (int i = 0; i < 9; i++) W[i] = (double)cam.R[i];
    const double dJ0 = dT[0] * W[0] + dT[1] * W[1] + dT[2] * W[2];
    const double dJ2 = dT[0] * W[6] + dT[1] * W[7] + dT[2] * W[8];
    const double dJ4 = dT[3] * W[3] + dT[4] * W[4] + dT[5] * W[5];
    const double dJ5 = dT[3] * W[6] + dT[4] * W[7] + dT[5] * W[8];
    const double fx = (double)cam.fx, fy = (double)cam.fy;
    const double tx = V.t[0], ty = V.t[1];
    const double itz = V.itz, itz2 = itz * itz, itz3 = itz2 * itz;
    double dt[3] = {0.0, 0.0, 0.0};
    dt[2] += -dJ0 * fx * itz2 - dJ4 * fy * itz2;
    dt[2] += 2.0 * dJ2 * fx * V.txc * itz3 + 2.0 * dJ5 * fy * V.tyc * itz3;
    const double dtxc = -dJ2 * fx * itz2, dtyc = -dJ5 * fy * itz2;
    if (!V.clipx) dt[0] += dtxc; else dt[2] += dtxc * (tx > 0.0 ? V.limx : -V.limx);
    if (!V.clipy) dt[1] += dtyc; else dt[2] += dtyc * (ty > 0.0 ? V.limy : -V.limy);
    // pixel-space mean
    dt[0] += du * fx * itz;
    dt[1] += dv * fy * itz;
    dt[2] -= (du * fx * tx + dv * fy * ty) * itz2;
    for (int i = 0; i < 3; i++) dmu[i] += W[i] * dt[0] + W[3 + i] * dt[1] + W[6 + i] * dt[2];
  }
  // combine the waves of this Gaussian (fixed order)
  if (wave > 0) {
    double* p = &s_part[wave - 1][0][lane];
    for (int i = 0; i < 3; i++) p[i * 64] = dmu[i];
    for (int i = 0; i < 6; i++) p[(3 + i) * 64] = dSig[i];
    p[9 * 64] = dop;
    p[10 * 64] = gnorm;
    s_cnt[wave - 1][lane] = cnt;
  }
  __syncthreads();
  if (wave > 0) return;
  for (int w = 0; w < kAdjWaves - 1; w++) {
    const double* p = &s_part[w][0][lane];
    for (int i = 0; i < 3; i++) dmu[i] += p[i * 64];
    for (int i = 0; i < 6; i++) dSig[i] += p[(3 + i) * 64];
    dop += p[9 * 64];
    gnorm += p[10 * 64];
    cnt += s_cnt[w][lane];
  }
  if (!live || cnt == 0) return;
  GaussD G;
  load_gaussian(sc, g, G);
  // Sigma = M M^T -> dM = 2 dSigma M (dSigma symmetric)
  const double* M = G.M;
  const double dS[9] = {dSig[0], dSig[1], dSig[2], dSig[1], dSig[3], dSig[4], dSig[2], dSig[4], dSig[5]};
  double dM[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      dM[i * 3 + j] = 2.0 * (dS[i * 3 + 0] * M[0 * 3 + j] + dS[i * 3 + 1] * M[1 * 3 + j] + dS[i * 3 + 2] * M[2 * 3 + j]);
  double dR[9], dls[3];
  for (int j = 0; j < 3; j++) {
    double acc = 0.0;
    for (int i = 0; i < 3; i++) {
      dR[i * 3 + j] = dM[i * 3 + j] * G.s[j];
      acc += dM[i * 3 + j] * G.Rq[i * 3 + j];
    }
    dls[j] = acc * G.s[j];
  }
  const double w = G.qhat[0], x = G.qhat[1], y = G.qhat[2], z = G.qhat[3];
  double dw = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  double dx = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                     2.0 * x * dR[8]);
  double dy = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                     2.0 * y * dR[8]);
  double dz = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                     y * dR[7]);
  const double dot = w * dw + x * dx + y * dy + z * dz;
  const double dq[4] = {(dw - w * dot) / G.qn, (dx - x * dot) / G.qn, (dy - y * dot) / G.qn, (dz - z * dot) / G.qn};
  const int64_t st = sc.stride;
  if (gr.mean)
    for (int i = 0; i < 3; i++) gr.mean[i * st + g] += (float)dmu[i];
  if (gr.quat)
    for (int i = 0; i < 4; i++) gr.quat[i * st + g] += (float)dq[i];
  if (gr.log_scale)
    for (int i = 0; i < 3; i++) gr.log_scale[i * st + g] += (float)dls[i];
  if (gr.opacity_logit) gr.opacity_logit[g] += (float)(dop * o * (1.0 - o));
  if (gradnorm) gradnorm[g] += (float)gnorm;
  if (gcount) gcount[g] += cnt;
}

// Colour part: rgb_c = max(0, sum_k sh[k,c] Y_k(dhat) + 0.5), dhat = normalise(mu - campos).
// Four lanes per Gaussian: lane c < 3 owns channel c (its K coefficients and their gradients,
// over all views); the direction gradients of the three channels are summed at the end.
// Visibility in a view and the clamp of each channel are read from the forward's per-(view,
// Gaussian) flags (taken from its stored colour, 0 where the clamp was active), so neither is
// recomputed; the gradient arithmetic itself is float32.
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_bwd_colour(SceneK sc, CamsK cams, int nv,
                                                               const uint8_t* __restrict__ vis,
                                                               const float* __restrict__ g2d, dass_grads gr) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int g_raw = tid / kBwdSplit, ch = tid % kBwdSplit;
  const bool live = g_raw < sc.n && ch < 3;
  const int g = g_raw < sc.n ? g_raw : sc.n - 1;
  const int c = ch < 3 ? ch : 2;
  float mu[3];
  for (int i = 0; i < 3; i++) mu[i] = sc.mean[(int64_t)i * sc.stride + g];
  float shc[K], dsh[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    shc[k] = sc.sh[(int64_t)(k * 3 + c) * sc.stride + g];
    dsh[k] = 0.f;
  }
  float dmu[3] = {0.f, 0.f, 0.f};
  constexpr int kAhead = 4;  // views whose inputs are loaded together
  for (int v0 = 0; v0 < nv && live; v0 += kAhead) {
    uint32_t f4[kAhead];
    float d4[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; u++) {
      f4[u] = 0;
      if (v0 + u < nv) {
        const int64_t row = (int64_t)(v0 + u) * sc.n + g;
        f4[u] = vis[row];
        d4[u] = g2d[row * 9 + 6 + c];
      }
    }
#pragma unroll
    for (int u = 0; u < kAhead; u++) {
      const int v = v0 + u;
      // not visible in this view (or past the last view), or a clamped channel (no derivative)
      if ((f4[u] & (8u | (1u << c))) != (8u | (1u << c))) continue;
      const CamK& cam = cams.c[v];
      float dir[3];
      for (int i = 0; i < 3; i++) dir[i] = mu[i] - cam.campos[i];
      const float dn = sqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
      const float inv_dn = dn > 0.f ? 1.f / dn : 0.f;
      float dhat[3];
      for (int i = 0; i < 3; i++) dhat[i] = dir[i] * inv_dn;
      float Y[16];
      sh_basis<DEG, false, float>(dhat[0], dhat[1], dhat[2], Y, nullptr, nullptr, nullptr);
      const float d = d4[u];
      float w[16];
#pragma unroll
      for (int k = 0; k < K; k++) {
        dsh[k] += d * Y[k];
        w[k] = d * shc[k];
      }
      float dd[3];
      sh_weighted_grad<DEG, float>(dhat[0], dhat[1], dhat[2], w, dd[0], dd[1], dd[2]);
      if (dn > 0.f) {
        const float dot = dhat[0] * dd[0] + dhat[1] * dd[1] + dhat[2] * dd[2];
        for (int i = 0; i < 3; i++) dmu[i] += (dd[i] - dhat[i] * dot) * inv_dn;
      }
    }
  }
  for (int i = 0; i < 3; i++) dmu[i] = quad_sumf(dmu[i]);
  if (g_raw >= sc.n) return;
  const int64_t st = sc.stride;
  if (live && gr.sh) {
#pragma unroll
    for (int k = 0; k < K; k++) gr.sh[(int64_t)(k * 3 + c) * st + g] += dsh[k];
  }
  if (ch == 0 && gr.mean)
    for (int i = 0; i < 3; i++) gr.mean[i * st + g] += dmu[i];
}

__global__ void k_debug_projection(SceneK sc, CamK cam, double* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sc.n) return;
  GaussD G;
  load_gaussian(sc, g, G);
  double limx, limy;
  clip_limits(cam, limx, limy);
  ViewD V;
  project_view(G, cam, limx, limy, V);
  double* o = out + (int64_t)g * 16;
  double rgb_pre[3] = {0, 0, 0}, dhat[3], dn;
  float shc[48];
  const int K = (sc.deg + 1) * (sc.deg + 1);
  for (int k = 0; k < 48; k++) shc[k] = k < 3 * K ? sc.sh[(int64_t)k * sc.stride + g] : 0.f;
  colour<3>(G, cam, shc, rgb_pre, dhat, dn);
  o[0] = V.u; o[1] = V.v; o[2] = V.A; o[3] = V.B; o[4] = V.C; o[5] = G.o;
  for (int c = 0; c < 3; c++) o[6 + c] = fmax(rgb_pre[c], 0.0);
  o[9] = V.t[2]; o[10] = V.radius; o[11] = V.x0; o[12] = V.y0; o[13] = V.x1; o[14] = V.y1;
  o[15] = V.visible ? 1.0 : 0.0;
}

}  // namespace

void launch_preprocess(const SceneK& s, const CamsK& cams, int nv, Workspace& ws, hipStream_t st) {
  if (s.n == 0) return;
  // view groups per Gaussian: about 3,000+ workgroups in flight once there are enough views
  const int blocks_g = (s.n + 255) / 256;
  int vs = 1;
  while (vs < 4 && vs * 2 <= nv && (int64_t)blocks_g * vs < 4096) vs *= 2;
  dim3 grid(blocks_g, vs), block(256);
  switch (s.deg) {
    case 0: k_preprocess<0><<<grid, block, 0, st>>>(s, cams, nv, ws.rec_u, ws.rect_u, ws.vis, ws.dkey[0],
                                                     ws.dval[0]);
      break;
    case 1: k_preprocess<1><<<grid, block, 0, st>>>(s, cams, nv, ws.rec_u, ws.rect_u, ws.vis, ws.dkey[0],
                                                     ws.dval[0]);
      break;
    case 2: k_preprocess<2><<<grid, block, 0, st>>>(s, cams, nv, ws.rec_u, ws.rect_u, ws.vis, ws.dkey[0],
                                                     ws.dval[0]);
      break;
    default: k_preprocess<3><<<grid, block, 0, st>>>(s, cams, nv, ws.rec_u, ws.rect_u, ws.vis, ws.dkey[0],
                                                     ws.dval[0]);
      break;
  }
}

void launch_preprocess_bwd(const SceneK& s, const CamsK& cams, int nv, const Workspace& ws, const dass_grads& grads,
                           float* gradnorm, int32_t* gcount, hipStream_t st) {
  if (s.n == 0) return;
  const int64_t threads = (int64_t)s.n * kBwdSplit;
  dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  k_preprocess_bwd_geom<<<(s.n + 63) / 64, 64 * kAdjWaves, 0, st>>>(s, cams, nv, ws.vis, ws.g2d, grads, gradnorm,
                                                                 gcount);
  if (!grads.mean && !grads.sh) return;
  switch (s.deg) {
    case 0: k_preprocess_bwd_colour<0><<<grid, block, 0, st>>>(s, cams, nv, ws.vis, ws.g2d, grads); break;
    case 1: k_preprocess_bwd_colour<1><<<grid, block, 0, st>>>(s, cams, nv, ws.vis, ws.g2d, grads); break;
    case 2: k_preprocess_bwd_colour<2><<<grid, block, 0, st>>>(s, cams, nv, ws.vis, ws.g2d, grads); break;
    default: k_preprocess_bwd_colour<3><<<grid, block, 0, st>>>(s, cams, nv, ws.vis, ws.g2d, grads); break;
  }
}

void launch_debug_projection(const SceneK& s, const CamsK& cams, int view, double* out, hipStream_t st) {
  if (s.n == 0) return;
  k_debug_projection<<<(s.n + 255) / 256, 256, 0, st>>>(s, cams.c[view], out);
}

}  // namespace dass
