/*
 * dass_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, double-precision CPU definition of what the streaming
 * Gaussian-splatting hot path computes (DASS, arXiv 2411.14847):
 *   - projection of 3D Gaussians: Sigma = R S S^T R^T and the EWA 2D
 *     covariance Sigma_2D = J W Sigma W^T J^T (App. A.1, eqs. for G(x),
 *     Sigma and Sigma_2D), colour from real spherical harmonics;
 *   - tile keys, their sort and per-tile ranges ("tile-based
 *     differentiable rasterization", Sec. 1 / Sec. 4.2);
 *   - front-to-back alpha compositing C = sum c_i a_i prod_{j<i}(1-a_j)
 *     (App. A.1, blending equation) and its exact adjoint;
 *   - the dynamics-aware shift p' = p + mu, q' = norm(q) x norm(sigma)
 *     (Sec. 3.3) and its adjoint;
 *   - the Adam update, the L1 fidelity gradient and error map (Sec. 3.4);
 *   - error-guided densification: Alg. 1 projection, the set of Eq. (4),
 *     and spawning of children (Sec. 3.4).
 *
 * Only the test suite, the smoke entry and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the HIP path.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC
 * (contraction off: the few decision quantities that are compared bit-for-bit
 * with the GPU -- camera-space depth, pixel mean, tile rectangle, Alg. 1 pixel
 * -- are evaluated in a fixed operation order with no fused multiply-add.)
 *
 * Readings of points the paper leaves open (all documented in the design
 * notes): blend order = ascending camera-space depth of the centre, ties by
 * index; alpha clamp 0.99, skip below 1/255, stop before blending an entry
 * that would take transmittance below 1e-4 (the float32 values of these
 * constants, widened); 0.3 px^2 dilation; cull at depth <= 0.2; radius
 * ceil(3 sqrt(lambda_max)); the Jacobian clamp at 1.3x the half field of
 * view; pixel centres at integer coordinates with the principal point at
 * ((W-1)/2,(H-1)/2); real orthonormal SH up to degree 3 with +0.5 offset and
 * clamp at 0; opacity = sigmoid(logit); scale = exp(log_scale).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ALPHA_MAX ((double)0.99f)
#define ALPHA_MIN ((double)(float)(1.0 / 255.0))
#define T_STOP ((double)1e-4f)
#define DILATION ((double)0.3f)
#define NEAR_Z ((double)0.2f)
#define CLIP_FAC ((double)1.3f)

/* decision-margin flags (bit set => the item sits within rounding of a decision) */
enum {
  FLAG_RADIUS = 1,  /* 3 sqrt(lambda_max) within rounding of an integer         */
  FLAG_CLIP = 2,    /* t_x/t_z or t_y/t_z within rounding of the Jacobian clamp */
  FLAG_RGB = 4,     /* a colour channel within rounding of the clamp at 0        */
  FLAG_SKIP = 8,    /* some alpha within rounding of the 1/255 skip threshold    */
  FLAG_STOP = 16,   /* some transmittance within rounding of the 1e-4 stop       */
  FLAG_PSIGN = 32,  /* some exponent within rounding of zero from below          */
  FLAG_CLAMP = 64   /* some alpha within rounding of the 0.99 clamp               */
};

typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float campos[3];
  int32_t width, height;
} orc_cam;

/* ---------------------------------------------------------------------------------------- */
/* Real spherical harmonics, degree <= 3, index k = l*l + (m + l), m = -l..l.               */
/* Standard real orthonormal basis (no Condon-Shortley sign), as polynomials in the unit     */
/* direction (x,y,z).  Constants from their closed forms.                                    */
/* ---------------------------------------------------------------------------------------- */
static void sh_basis(int deg, double x, double y, double z, double* Y, double* dYx, double* dYy,
                     double* dYz) {
  const double PI = 3.14159265358979323846;
  const double c0 = 0.5 * sqrt(1.0 / PI);
  const double c1 = sqrt(3.0 / (4.0 * PI));
  const double c2a = 0.5 * sqrt(15.0 / PI);
  const double c2b = 0.25 * sqrt(5.0 / PI);
  const double c2c = 0.25 * sqrt(15.0 / PI);
  const double c3a = 0.25 * sqrt(35.0 / (2.0 * PI));
  const double c3b = 0.5 * sqrt(105.0 / PI);
  const double c3c = 0.25 * sqrt(21.0 / (2.0 * PI));
  const double c3d = 0.25 * sqrt(7.0 / PI);
  const double c3e = 0.25 * sqrt(105.0 / PI);
  int K = (deg + 1) * (deg + 1);
  for (int k = 0; k < K; k++) Y[k] = dYx[k] = dYy[k] = dYz[k] = 0.0;
  Y[0] = c0;
  if (deg >= 1) {
    Y[1] = c1 * y; dYy[1] = c1;
    Y[2] = c1 * z; dYz[2] = c1;
    Y[3] = c1 * x; dYx[3] = c1;
  }
  if (deg >= 2) {
    Y[4] = c2a * x * y; dYx[4] = c2a * y; dYy[4] = c2a * x;
    Y[5] = c2a * y * z; dYy[5] = c2a * z; dYz[5] = c2a * y;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    dYx[6] = -2.0 * c2b * x; dYy[6] = -2.0 * c2b * y; dYz[6] = 4.0 * c2b * z;
    Y[7] = c2a * x * z; dYx[7] = c2a * z; dYz[7] = c2a * x;
    Y[8] = c2c * (x * x - y * y); dYx[8] = 2.0 * c2c * x; dYy[8] = -2.0 * c2c * y;
  }
  if (deg >= 3) {
    Y[9] = c3a * y * (3.0 * x * x - y * y);
    dYx[9] = c3a * 6.0 * x * y; dYy[9] = c3a * (3.0 * x * x - 3.0 * y * y);
    Y[10] = c3b * x * y * z;
    dYx[10] = c3b * y * z; dYy[10] = c3b * x * z; dYz[10] = c3b * x * y;
    Y[11] = c3c * y * (4.0 * z * z - x * x - y * y);
    dYx[11] = c3c * (-2.0 * x * y); dYy[11] = c3c * (4.0 * z * z - x * x - 3.0 * y * y);
    dYz[11] = c3c * 8.0 * y * z;
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    dYx[12] = c3d * (-6.0 * x * z); dYy[12] = c3d * (-6.0 * y * z);
    dYz[12] = c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = c3c * x * (4.0 * z * z - x * x - y * y);
    dYx[13] = c3c * (4.0 * z * z - 3.0 * x * x - y * y); dYy[13] = c3c * (-2.0 * x * y);
    dYz[13] = c3c * 8.0 * x * z;
    Y[14] = c3e * z * (x * x - y * y);
    dYx[14] = c3e * 2.0 * x * z; dYy[14] = -c3e * 2.0 * y * z; dYz[14] = c3e * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3.0 * y * y);
    dYx[15] = c3a * (3.0 * x * x - 3.0 * y * y); dYy[15] = c3a * (-6.0 * x * y);
  }
}

void orc_sh_eval(int32_t deg, int32_t n, const double* dirs /*[n][3]*/, double* out /*[n][K]*/) {
  int K = (deg + 1) * (deg + 1);
  double Y[16], a[16], b[16], c[16];
  for (int i = 0; i < n; i++) {
    sh_basis(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], Y, a, b, c);
    for (int k = 0; k < K; k++) out[(size_t)i * K + k] = Y[k];
  }
}

/* ---------------------------------------------------------------------------------------- */
/* Projection of one Gaussian into one view (App. A.1).                                      */
/* ---------------------------------------------------------------------------------------- */
typedef struct {
  /* inputs (widened) */
  double mu[3], q[4], qn, qhat[4], s[3], logit;
  /* intermediates */
  double Rq[9], M[9], Sig[9], t[3], txc, tyc; int clipx, clipy; double limx, limy;
  double J[6], T[6], a, b, c, det, lmax;
  double dir[3], dn, dhat[3], rgb_pre[3];
  /* outputs */
  double u, v, A, B, C, o, rgb[3], depth;
  int32_t radius, rect[4], visible, flags;
  uint32_t depth_bits;
} proj_t;

static void quat_to_rot(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

static void project_one(const double* mean, const double* quat, const double* log_scale,
                        const double* logit, const double* sh, int deg, int64_t stride, int64_t g,
                        const orc_cam* cam, int tile_w, int tile_h, proj_t* P) {
  memset(P, 0, sizeof(*P));
  for (int i = 0; i < 3; i++) P->mu[i] = mean[i * stride + g];
  for (int i = 0; i < 4; i++) P->q[i] = quat[i * stride + g];
  for (int i = 0; i < 3; i++) P->s[i] = exp(log_scale[i * stride + g]);
  P->logit = logit[g];
  const double* q = P->q;
  P->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(P->qn > 0.0)) { P->visible = 0; return; }
  for (int i = 0; i < 4; i++) P->qhat[i] = q[i] / P->qn;
  quat_to_rot(P->qhat, P->Rq);
  /* Sigma = (R S)(R S)^T */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) P->M[i * 3 + j] = P->Rq[i * 3 + j] * P->s[j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += P->M[i * 3 + k] * P->M[j * 3 + k];
      P->Sig[i * 3 + j] = acc;
    }
  /* camera space: t = W mu + t_v, fixed order ((r0 x + r1 y) + r2 z) + t */
  double W[9];
  for (int i = 0; i < 9; i++) W[i] = (double)cam->R[i];
  for (int i = 0; i < 3; i++)
    P->t[i] = ((W[i * 3 + 0] * P->mu[0] + W[i * 3 + 1] * P->mu[1]) + W[i * 3 + 2] * P->mu[2]) +
              (double)cam->t[i];
  double tx = P->t[0], ty = P->t[1], tz = P->t[2];
  P->depth = tz;
  P->depth_bits = 0;
  if (!(tz > NEAR_Z)) { P->visible = 0; return; }
  {
    float d32 = (float)tz;
    memcpy(&P->depth_bits, &d32, 4);
  }
  double fx = (double)cam->fx, fy = (double)cam->fy;
  P->limx = CLIP_FAC * ((double)cam->width / (2.0 * fx));
  P->limy = CLIP_FAC * ((double)cam->height / (2.0 * fy));
  double rx = tx / tz, ry = ty / tz;
  P->clipx = (rx < -P->limx || rx > P->limx);
  P->clipy = (ry < -P->limy || ry > P->limy);
  if (fabs(fabs(rx) - P->limx) <= 1e-7 * P->limx) P->flags |= FLAG_CLIP;
  if (fabs(fabs(ry) - P->limy) <= 1e-7 * P->limy) P->flags |= FLAG_CLIP;
  P->txc = clampd(rx, -P->limx, P->limx) * tz;
  P->tyc = clampd(ry, -P->limy, P->limy) * tz;
  /* J = [[fx/tz, 0, -fx txc/tz^2], [0, fy/tz, -fy tyc/tz^2]] */
  P->J[0] = fx / tz; P->J[1] = 0.0; P->J[2] = -fx * P->txc / (tz * tz);
  P->J[3] = 0.0; P->J[4] = fy / tz; P->J[5] = -fy * P->tyc / (tz * tz);
  /* T = J W (2x3) */
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += P->J[i * 3 + k] * W[k * 3 + j];
      P->T[i * 3 + j] = acc;
    }
  /* Sigma_2D = T Sigma T^T + dilation I */
  double S2[4];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) acc += P->T[i * 3 + k] * P->Sig[k * 3 + l] * P->T[j * 3 + l];
      S2[i * 2 + j] = acc;
    }
  P->a = S2[0] + DILATION;
  P->b = 0.5 * (S2[1] + S2[2]);
  P->c = S2[3] + DILATION;
  P->det = P->a * P->c - P->b * P->b;
  if (!(P->det > 0.0)) { P->visible = 0; return; }
  P->A = P->c / P->det;
  P->B = -P->b / P->det;
  P->C = P->a / P->det;
  double mid = 0.5 * (P->a + P->c);
  double disc = 0.25 * (P->a - P->c) * (P->a - P->c) + P->b * P->b;
  P->lmax = mid + sqrt(disc > 0.0 ? disc : 0.0);
  double r3 = 3.0 * sqrt(P->lmax);
  double rr = ceil(r3);
  if (fabs(r3 - floor(r3 + 0.5)) <= 1e-9 * (r3 > 1.0 ? r3 : 1.0)) P->flags |= FLAG_RADIUS;
  if (rr > 1.0e7) rr = 1.0e7;
  P->radius = (int32_t)rr;
  /* pixel-space mean, fixed order ((f t)/tz) + c */
  P->u = ((fx * tx) / tz) + (double)cam->cx;
  P->v = ((fy * ty) / tz) + (double)cam->cy;
  /* tile rectangle [x0,x1) x [y0,y1) */
  int TX = (cam->width + tile_w - 1) / tile_w, TY = (cam->height + tile_h - 1) / tile_h;
  double r = (double)P->radius;
  double fx0 = floor((P->u - r) / (double)tile_w);
  double fx1 = floor(((P->u + r) + (double)(tile_w - 1)) / (double)tile_w);
  double fy0 = floor((P->v - r) / (double)tile_h);
  double fy1 = floor(((P->v + r) + (double)(tile_h - 1)) / (double)tile_h);
  P->rect[0] = (int32_t)clampd(fx0, 0.0, (double)TX);
  P->rect[1] = (int32_t)clampd(fy0, 0.0, (double)TY);
  P->rect[2] = (int32_t)clampd(fx1, 0.0, (double)TX);
  P->rect[3] = (int32_t)clampd(fy1, 0.0, (double)TY);
  P->visible = (P->radius > 0) && (P->rect[2] > P->rect[0]) && (P->rect[3] > P->rect[1]);
  /* colour */
  for (int i = 0; i < 3; i++) P->dir[i] = P->mu[i] - (double)cam->campos[i];
  P->dn = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
  for (int i = 0; i < 3; i++) P->dhat[i] = P->dn > 0.0 ? P->dir[i] / P->dn : 0.0;
  double Y[16], d1[16], d2[16], d3[16];
  sh_basis(deg, P->dhat[0], P->dhat[1], P->dhat[2], Y, d1, d2, d3);
  int K = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ch++) {
    double acc = 0.0;
    for (int k = 0; k < K; k++) acc += sh[(int64_t)(k * 3 + ch) * stride + g] * Y[k];
    P->rgb_pre[ch] = acc + 0.5;
    P->rgb[ch] = P->rgb_pre[ch] > 0.0 ? P->rgb_pre[ch] : 0.0;
    if (fabs(P->rgb_pre[ch]) <= 1e-7) P->flags |= FLAG_RGB;
  }
  P->o = 1.0 / (1.0 + exp(-P->logit));
}

/* Project all n Gaussians into one view.  Output arrays are per Gaussian. */
void orc_project(int32_t n, const double* mean, const double* quat, const double* log_scale,
                 const double* logit, const double* sh, int32_t deg, int64_t stride,
                 const orc_cam* cam, int32_t tile_w, int32_t tile_h, double* uv /*[n][2]*/,
                 double* conic /*[n][3]*/, double* opacity, double* rgb /*[n][3]*/,
                 double* depth, int32_t* radius, int32_t* rect /*[n][4]*/,
                 uint32_t* depth_bits, int32_t* visible, int32_t* flags) {
  proj_t P;
  for (int64_t g = 0; g < n; g++) {
    project_one(mean, quat, log_scale, logit, sh, deg, stride, g, cam, tile_w, tile_h, &P);
    uv[2 * g] = P.u; uv[2 * g + 1] = P.v;
    conic[3 * g] = P.A; conic[3 * g + 1] = P.B; conic[3 * g + 2] = P.C;
    opacity[g] = P.o;
    for (int c = 0; c < 3; c++) rgb[3 * g + c] = P.rgb[c];
    depth[g] = P.depth;
    radius[g] = P.visible ? P.radius : 0;
    for (int c = 0; c < 4; c++) rect[4 * g + c] = P.visible ? P.rect[c] : 0;
    depth_bits[g] = P.depth_bits;
    visible[g] = P.visible;
    flags[g] = P.flags;
  }
}

/* ---------------------------------------------------------------------------------------- */
/* Keys: for each visible Gaussian (index order), for each tile of its rectangle in          */
/* row-major order: key = (tile_id << 32) | bits(float depth), value = index.                */
/* ---------------------------------------------------------------------------------------- */
int64_t orc_count_keys(int32_t n, const int32_t* rect, const int32_t* visible) {
  int64_t total = 0;
  for (int64_t g = 0; g < n; g++)
    if (visible[g])
      total += (int64_t)(rect[4 * g + 2] - rect[4 * g]) * (rect[4 * g + 3] - rect[4 * g + 1]);
  return total;
}

void orc_emit_keys(int32_t n, const int32_t* rect, const int32_t* visible,
                   const uint32_t* depth_bits, int32_t tiles_x, uint64_t* keys, uint32_t* vals) {
  int64_t k = 0;
  for (int64_t g = 0; g < n; g++) {
    if (!visible[g]) continue;
    for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; y++)
      for (int x = rect[4 * g]; x < rect[4 * g + 2]; x++) {
        uint64_t tile = (uint64_t)y * (uint64_t)tiles_x + (uint64_t)x;
        keys[k] = (tile << 32) | (uint64_t)depth_bits[g];
        vals[k] = (uint32_t)g;
        k++;
      }
  }
}

/* Stable sort by key: (key, value) pairs are unique and emitted in increasing value order for
 * equal keys, so ordering by (key, value) is the stable order. Plain merge sort. */
static int pair_less(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

void orc_sort_pairs(int64_t n, uint64_t* keys, uint32_t* vals) {
  if (n < 2) return;
  uint64_t* tk = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint32_t* tv = (uint32_t*)malloc(sizeof(uint32_t) * n);
  for (int64_t width = 1; width < n; width *= 2) {
    for (int64_t lo = 0; lo < n; lo += 2 * width) {
      int64_t mid = lo + width < n ? lo + width : n;
      int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
      int64_t i = lo, j = mid, o = lo;
      while (i < mid && j < hi) {
        if (pair_less(keys[j], vals[j], keys[i], vals[i])) { tk[o] = keys[j]; tv[o++] = vals[j++]; }
        else { tk[o] = keys[i]; tv[o++] = vals[i++]; }
      }
      while (i < mid) { tk[o] = keys[i]; tv[o++] = vals[i++]; }
      while (j < hi) { tk[o] = keys[j]; tv[o++] = vals[j++]; }
    }
    memcpy(keys, tk, sizeof(uint64_t) * n);
    memcpy(vals, tv, sizeof(uint32_t) * n);
  }
  free(tk);
  free(tv);
}

/* ranges[t] = [first, last+1) of sorted keys with tile id t; (0,0) if none */
void orc_ranges(int64_t count, const uint64_t* keys, int32_t n_tiles, int64_t* ranges) {
  for (int t = 0; t < n_tiles; t++) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (int64_t i = 0; i < count; i++) {
    int64_t t = (int64_t)(keys[i] >> 32);
    if (i == 0 || (int64_t)(keys[i - 1] >> 32) != t) ranges[2 * t] = i;
    if (i == count - 1 || (int64_t)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = i + 1;
  }
}

/* ---------------------------------------------------------------------------------------- */
/* Front-to-back blend of one tile (App. A.1 blending equation).                             */
/* ---------------------------------------------------------------------------------------- */
typedef struct {
  int32_t width, height, tile_w, tile_h, tiles_x;
  const int64_t* ranges;
  const uint32_t* vals;
  const double *uv, *conic, *opacity, *rgb;
  double bg[3];
} blend_in;

/* Walks one pixel's list.  If rec_* are given, records blended entries (gid, alpha, T_i,
 * clamped) for the backward pass.  Returns number of blended entries. */
static int64_t blend_pixel(const blend_in* in, int64_t lo, int64_t hi, double px, double py,
                           double* C, double* T_out, int32_t* n_contrib, int32_t* flags,
                           uint32_t* rec_g, double* rec_a, double* rec_T, uint8_t* rec_clamp,
                           uint64_t* sig) {
  double T = 1.0;
  uint64_t h = 1469598103934665603ULL;
  double acc[3] = {0.0, 0.0, 0.0};
  int32_t last = 0;
  int64_t nb = 0;
  for (int64_t i = lo; i < hi; i++) {
    uint32_t g = in->vals[i];
    double dx = in->uv[2 * g] - px, dy = in->uv[2 * g + 1] - py;
    double A = in->conic[3 * g], B = in->conic[3 * g + 1], Cc = in->conic[3 * g + 2];
    double P = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    double scale = fabs(A) * dx * dx + fabs(Cc) * dy * dy + 2.0 * fabs(B * dx * dy);
    if (P < 0.0 && -P <= 1e-5 * scale) *flags |= FLAG_PSIGN;
    if (P > 0.0) { if (P <= 1e-5 * scale) *flags |= FLAG_PSIGN; continue; }
    double araw = in->opacity[g] * exp(P);
    if (fabs(araw - ALPHA_MIN) <= 1e-5 * ALPHA_MIN) *flags |= FLAG_SKIP;
    if (fabs(araw - ALPHA_MAX) <= 1e-5 * ALPHA_MAX) *flags |= FLAG_CLAMP;
    double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
    if (a < ALPHA_MIN) continue;
    double Tn = T * (1.0 - a);
    if (fabs(Tn - T_STOP) <= 1e-3 * T_STOP) *flags |= FLAG_STOP;
    if (Tn < T_STOP) break;
    for (int c = 0; c < 3; c++) acc[c] += in->rgb[3 * g + c] * a * T;
    if (rec_g) {
      rec_g[nb] = g; rec_a[nb] = a; rec_T[nb] = T; rec_clamp[nb] = (araw >= ALPHA_MAX);
    }
    nb++;
    T = Tn;
    last = (int32_t)(i - lo + 1);
    h = (h ^ (uint64_t)(i - lo + 1)) * 1099511628211ULL;
  }
  if (sig) *sig = h;
  for (int c = 0; c < 3; c++) C[c] = acc[c] + T * in->bg[c];
  *T_out = T;
  *n_contrib = last;
  return nb;
}

/* Forward over a list of tiles (all tiles if tile_list == NULL).  Images are [3][H][W]. */
void orc_blend_fwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                   const int64_t* ranges, const uint32_t* vals, const double* uv,
                   const double* conic, const double* opacity, const double* rgb,
                   const double* bg, int32_t n_list, const int32_t* tile_list, double* out_rgb,
                   double* out_T, int32_t* out_ncontrib, int32_t* out_flags, uint64_t* out_sig) {
  blend_in in = {width, height, tile_w, tile_h, (width + tile_w - 1) / tile_w, ranges, vals,
                 uv, conic, opacity, rgb, {bg[0], bg[1], bg[2]}};
  int TY = (height + tile_h - 1) / tile_h;
  int nt = n_list > 0 ? n_list : in.tiles_x * TY;
  for (int it = 0; it < nt; it++) {
    int tile = n_list > 0 ? tile_list[it] : it;
    int tx = tile % in.tiles_x, ty = tile / in.tiles_x;
    int64_t lo = ranges[2 * tile], hi = ranges[2 * tile + 1];
    for (int y = ty * tile_h; y < (ty + 1) * tile_h && y < height; y++)
      for (int x = tx * tile_w; x < (tx + 1) * tile_w && x < width; x++) {
        double C[3], T;
        int32_t nc, fl = 0;
        uint64_t sg = 0;
        blend_pixel(&in, lo, hi, (double)x, (double)y, C, &T, &nc, &fl, NULL, NULL, NULL, NULL, &sg);
        int64_t p = (int64_t)y * width + x;
        if (out_sig) out_sig[p] = sg;
        for (int c = 0; c < 3; c++) out_rgb[(int64_t)c * width * height + p] = C[c];
        out_T[p] = T;
        out_ncontrib[p] = nc;
        out_flags[p] = fl;
      }
  }
}

/* Backward of the blend.  Accumulates (+=) per-Gaussian gradients g2d[g][9] =
 * (du, dv, dA, dB, dC, dopacity, dr, dg, db) from the pixels of the listed tiles. */
void orc_blend_bwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                   const int64_t* ranges, const uint32_t* vals, const double* uv,
                   const double* conic, const double* opacity, const double* rgb,
                   const double* bg, const float* dl_drgb /*[3][H][W]*/, int32_t n_list,
                   const int32_t* tile_list, double* g2d) {
  blend_in in = {width, height, tile_w, tile_h, (width + tile_w - 1) / tile_w, ranges, vals,
                 uv, conic, opacity, rgb, {bg[0], bg[1], bg[2]}};
  int TY = (height + tile_h - 1) / tile_h;
  int nt = n_list > 0 ? n_list : in.tiles_x * TY;
  int64_t maxlen = 0;
  for (int it = 0; it < nt; it++) {
    int tile = n_list > 0 ? tile_list[it] : it;
    int64_t len = ranges[2 * tile + 1] - ranges[2 * tile];
    if (len > maxlen) maxlen = len;
  }
  uint32_t* rg = (uint32_t*)malloc(sizeof(uint32_t) * (maxlen + 1));
  double* ra = (double*)malloc(sizeof(double) * (maxlen + 1));
  double* rT = (double*)malloc(sizeof(double) * (maxlen + 1));
  uint8_t* rc = (uint8_t*)malloc(maxlen + 1);
  for (int it = 0; it < nt; it++) {
    int tile = n_list > 0 ? tile_list[it] : it;
    int tx = tile % in.tiles_x, ty = tile / in.tiles_x;
    int64_t lo = ranges[2 * tile], hi = ranges[2 * tile + 1];
    for (int y = ty * tile_h; y < (ty + 1) * tile_h && y < height; y++)
      for (int x = tx * tile_w; x < (tx + 1) * tile_w && x < width; x++) {
        double C[3], T;
        int32_t nc, fl = 0;
        int64_t nb = blend_pixel(&in, lo, hi, (double)x, (double)y, C, &T, &nc, &fl, rg, ra, rT, rc, NULL);
        int64_t p = (int64_t)y * width + x;
        double dC[3];
        for (int c = 0; c < 3; c++) dC[c] = (double)dl_drgb[(int64_t)c * width * height + p];
        /* colour behind entry i: B_K = bg, B_{i-1} = a_i c_i + (1-a_i) B_i */
        double Bk[3] = {bg[0], bg[1], bg[2]};
        for (int64_t k = nb - 1; k >= 0; k--) {
          uint32_t g = rg[k];
          double a = ra[k], Ti = rT[k];
          const double* c = &rgb[3 * g];
          double da = 0.0;
          for (int ch = 0; ch < 3; ch++) {
            g2d[9 * (int64_t)g + 6 + ch] += a * Ti * dC[ch];
            da += Ti * (c[ch] - Bk[ch]) * dC[ch];
          }
          for (int ch = 0; ch < 3; ch++) Bk[ch] = a * c[ch] + (1.0 - a) * Bk[ch];
          if (rc[k]) continue; /* alpha clamped at 0.99: no derivative through o or P */
          double dx = uv[2 * g] - (double)x, dy = uv[2 * g + 1] - (double)y;
          double A = conic[3 * g], B = conic[3 * g + 1], Cc = conic[3 * g + 2];
          double P = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
          double G = exp(P);
          double dP = da * a; /* d alpha / dP = o exp(P) = alpha when not clamped */
          g2d[9 * (int64_t)g + 5] += da * G;
          g2d[9 * (int64_t)g + 0] += dP * (-A * dx - B * dy);
          g2d[9 * (int64_t)g + 1] += dP * (-Cc * dy - B * dx);
          g2d[9 * (int64_t)g + 2] += dP * (-0.5 * dx * dx);
          g2d[9 * (int64_t)g + 3] += dP * (-dx * dy);
          g2d[9 * (int64_t)g + 4] += dP * (-0.5 * dy * dy);
        }
      }
  }
  free(rg); free(ra); free(rT); free(rc);
}

/* ---------------------------------------------------------------------------------------- */
/* Adjoint of the projection (chain rule through App. A.1), accumulated over views.          */
/* ---------------------------------------------------------------------------------------- */
static void project_one_bwd(const proj_t* P, const double* sh, int deg, int64_t stride, int64_t g,
                            const orc_cam* cam, const double* gd /*[9]*/, double* dmean /*3*/,
                            double* dquat /*4*/, double* dlogs /*3*/, double* dlogit,
                            double* dsh /*[3K]*/) {
  double du = gd[0], dv = gd[1], dA = gd[2], dB = gd[3], dCc = gd[4], dop = gd[5];
  const double* drgb = gd + 6;
  double W[9];
  for (int i = 0; i < 9; i++) W[i] = (double)cam->R[i];
  double fx = (double)cam->fx, fy = (double)cam->fy;
  double tx = P->t[0], ty = P->t[1], tz = P->t[2];
  double dt[3] = {0.0, 0.0, 0.0};
  /* opacity = sigmoid(logit) */
  *dlogit += dop * P->o * (1.0 - P->o);
  /* colour: rgb = max(0, sum_k sh_k Y_k(dhat) + 0.5) */
  double Y[16], dYx[16], dYy[16], dYz[16];
  sh_basis(deg, P->dhat[0], P->dhat[1], P->dhat[2], Y, dYx, dYy, dYz);
  int K = (deg + 1) * (deg + 1);
  double ddir[3] = {0.0, 0.0, 0.0};
  for (int ch = 0; ch < 3; ch++) {
    if (P->rgb_pre[ch] < 0.0) continue;
    double d = drgb[ch];
    for (int k = 0; k < K; k++) {
      double coef = sh[(int64_t)(k * 3 + ch) * stride + g];
      dsh[k * 3 + ch] += d * Y[k];
      ddir[0] += d * coef * dYx[k];
      ddir[1] += d * coef * dYy[k];
      ddir[2] += d * coef * dYz[k];
    }
  }
  if (P->dn > 0.0) {
    double dd = P->dhat[0] * ddir[0] + P->dhat[1] * ddir[1] + P->dhat[2] * ddir[2];
    for (int i = 0; i < 3; i++) dmean[i] += (ddir[i] - P->dhat[i] * dd) / P->dn;
  }
  /* conic (A,B,C) = (c, -b, a)/det with det = a c - b^2 */
  double a = P->a, b = P->b, c = P->c, det = P->det, det2 = det * det;
  double da = (-c * c * dA + b * c * dB + (det - a * c) * dCc) / det2;
  double db = (2.0 * b * c * dA + (-det - 2.0 * b * b) * dB + 2.0 * a * b * dCc) / det2;
  double dc = ((det - a * c) * dA + a * b * dB - a * a * dCc) / det2;
  /* Sigma_2D = T Sigma T^T (+ constant): G2 symmetric with off-diagonals db/2 */
  double G2[4] = {da, 0.5 * db, 0.5 * db, dc};
  double dSig[9], dT[6];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 2; k++)
        for (int l = 0; l < 2; l++) acc += P->T[k * 3 + i] * G2[k * 2 + l] * P->T[l * 3 + j];
      dSig[i * 3 + j] = acc;
    }
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 2; k++)
        for (int l = 0; l < 3; l++) acc += G2[i * 2 + k] * P->T[k * 3 + l] * P->Sig[l * 3 + j];
      dT[i * 3 + j] = 2.0 * acc;
    }
  /* T = J W  ->  dJ = dT W^T */
  double dJ[6];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += dT[i * 3 + k] * W[j * 3 + k];
      dJ[i * 3 + j] = acc;
    }
  double tz2 = tz * tz, tz3 = tz2 * tz;
  dt[2] += dJ[0] * (-fx / tz2) + dJ[4] * (-fy / tz2);
  double dtxc = dJ[2] * (-fx / tz2), dtyc = dJ[5] * (-fy / tz2);
  dt[2] += dJ[2] * (2.0 * fx * P->txc / tz3) + dJ[5] * (2.0 * fy * P->tyc / tz3);
  if (!P->clipx) dt[0] += dtxc;
  else dt[2] += dtxc * (tx / tz > 0.0 ? P->limx : -P->limx);
  if (!P->clipy) dt[1] += dtyc;
  else dt[2] += dtyc * (ty / tz > 0.0 ? P->limy : -P->limy);
  /* mean2d */
  dt[0] += du * fx / tz;
  dt[1] += dv * fy / tz;
  dt[2] += du * (-fx * tx / tz2) + dv * (-fy * ty / tz2);
  /* t = W mu + t_v */
  for (int i = 0; i < 3; i++) dmean[i] += W[0 * 3 + i] * dt[0] + W[1 * 3 + i] * dt[1] + W[2 * 3 + i] * dt[2];
  /* Sigma = M M^T, M = R diag(s) */
  double dM[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0.0;
      for (int k = 0; k < 3; k++) acc += dSig[i * 3 + k] * P->M[k * 3 + j];
      dM[i * 3 + j] = 2.0 * acc;
    }
  double dR[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) dR[i * 3 + j] = dM[i * 3 + j] * P->s[j];
  for (int j = 0; j < 3; j++) {
    double ds = 0.0;
    for (int i = 0; i < 3; i++) ds += dM[i * 3 + j] * P->Rq[i * 3 + j];
    dlogs[j] += ds * P->s[j];
  }
  /* R(qhat) partials */
  double w = P->qhat[0], x = P->qhat[1], y = P->qhat[2], z = P->qhat[3];
  double dw = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
  dy += dR[0] * (-4.0 * y); dz += dR[0] * (-4.0 * z);
  dw += dR[1] * (-2.0 * z); dx += dR[1] * (2.0 * y); dy += dR[1] * (2.0 * x); dz += dR[1] * (-2.0 * w);
  dw += dR[2] * (2.0 * y); dx += dR[2] * (2.0 * z); dy += dR[2] * (2.0 * w); dz += dR[2] * (2.0 * x);
  dw += dR[3] * (2.0 * z); dx += dR[3] * (2.0 * y); dy += dR[3] * (2.0 * x); dz += dR[3] * (2.0 * w);
  dx += dR[4] * (-4.0 * x); dz += dR[4] * (-4.0 * z);
  dw += dR[5] * (-2.0 * x); dx += dR[5] * (-2.0 * w); dy += dR[5] * (2.0 * z); dz += dR[5] * (2.0 * y);
  dw += dR[6] * (-2.0 * y); dx += dR[6] * (2.0 * z); dy += dR[6] * (-2.0 * w); dz += dR[6] * (2.0 * x);
  dw += dR[7] * (2.0 * x); dx += dR[7] * (2.0 * w); dy += dR[7] * (2.0 * z); dz += dR[7] * (2.0 * y);
  dx += dR[8] * (-4.0 * x); dy += dR[8] * (-4.0 * y);
  double dqh[4] = {dw, dx, dy, dz};
  double dot = w * dw + x * dx + y * dy + z * dz;
  for (int i = 0; i < 4; i++) dquat[i] += (dqh[i] - P->qhat[i] * dot) / P->qn;
}

/* Chain per-view 2D gradients g2d[n][9] back to parameters for one view; accumulates (+=)
 * into dmean[3][n], dquat[4][n], dlogs[3][n], dlogit[n], dsh[3K][n], and adds the norm of
 * the (u,v) gradient of every visible Gaussian to gradnorm[n] and 1 to count[n]. */
void orc_project_bwd(int32_t n, const double* mean, const double* quat, const double* log_scale,
                     const double* logit, const double* sh, int32_t deg, int64_t stride,
                     const orc_cam* cam, int32_t tile_w, int32_t tile_h, const double* g2d,
                     const int32_t* only /* optional mask [n] or NULL */, double* dmean,
                     double* dquat, double* dlogs, double* dlogit, double* dsh,
                     double* gradnorm, int32_t* count) {
  proj_t P;
  int K = (deg + 1) * (deg + 1);
  for (int64_t g = 0; g < n; g++) {
    if (only && !only[g]) continue;
    project_one(mean, quat, log_scale, logit, sh, deg, stride, g, cam, tile_w, tile_h, &P);
    if (!P.visible) continue;
    double dm[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dl[3] = {0, 0, 0}, dlg = 0.0, ds[48];
    for (int k = 0; k < 3 * K; k++) ds[k] = 0.0;
    project_one_bwd(&P, sh, deg, stride, g, cam, &g2d[9 * g], dm, dq, dl, &dlg, ds);
    for (int i = 0; i < 3; i++) dmean[i * (int64_t)n + g] += dm[i];
    for (int i = 0; i < 4; i++) dquat[i * (int64_t)n + g] += dq[i];
    for (int i = 0; i < 3; i++) dlogs[i * (int64_t)n + g] += dl[i];
    dlogit[g] += dlg;
    for (int k = 0; k < 3 * K; k++) dsh[k * (int64_t)n + g] += ds[k];
    gradnorm[g] += sqrt(g2d[9 * g] * g2d[9 * g] + g2d[9 * g + 1] * g2d[9 * g + 1]);
    count[g] += 1;
  }
}

/* ---------------------------------------------------------------------------------------- */
/* Dynamics-aware shift (Sec. 3.3): p' = p + mu_n, q' = norm(q) x norm(sigma_n).            */
/* ---------------------------------------------------------------------------------------- */
static void qmul(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

void orc_shift_fwd(int32_t n, int64_t stride, const double* mean, const double* quat,
                   int32_t n_dyn, const int32_t* dyn_idx, const double* dpos /*[3][n_dyn]*/,
                   const double* drot /*[4][n_dyn]*/, double* out_mean /*[3][n]*/,
                   double* out_quat /*[4][n]*/) {
  for (int64_t g = 0; g < n; g++) {
    for (int i = 0; i < 3; i++) out_mean[i * (int64_t)n + g] = mean[i * stride + g];
    for (int i = 0; i < 4; i++) out_quat[i * (int64_t)n + g] = quat[i * stride + g];
  }
  for (int64_t j = 0; j < n_dyn; j++) {
    int64_t g = dyn_idx[j];
    double q[4], s[4], qn = 0.0, sn = 0.0, o[4];
    for (int i = 0; i < 4; i++) {
      q[i] = quat[i * stride + g];
      s[i] = drot[i * (int64_t)n_dyn + j];
      qn += q[i] * q[i];
      sn += s[i] * s[i];
    }
    qn = sqrt(qn); sn = sqrt(sn);
    for (int i = 0; i < 4; i++) { q[i] /= qn; s[i] /= sn; }
    qmul(q, s, o);
    for (int i = 0; i < 3; i++)
      out_mean[i * (int64_t)n + g] = mean[i * stride + g] + dpos[i * (int64_t)n_dyn + j];
    for (int i = 0; i < 4; i++) out_quat[i * (int64_t)n + g] = o[i];
  }
}

/* Adjoint: d_dpos[:,j] += dmean'[:,g], d_drot[:,j] += d/dsigma of norm(q) x norm(sigma). */
void orc_shift_adj(int32_t n, int64_t stride, const double* quat, int32_t n_dyn,
                   const int32_t* dyn_idx, const double* drot, const double* dmean /*[3][n]*/,
                   const double* dquat /*[4][n]*/, double* d_dpos, double* d_drot) {
  for (int64_t j = 0; j < n_dyn; j++) {
    int64_t g = dyn_idx[j];
    double q[4], s[4], qn = 0.0, sn = 0.0, dq[4];
    for (int i = 0; i < 4; i++) {
      q[i] = quat[i * stride + g];
      s[i] = drot[i * (int64_t)n_dyn + j];
      qn += q[i] * q[i];
      sn += s[i] * s[i];
      dq[i] = dquat[i * (int64_t)n + g];
    }
    qn = sqrt(qn); sn = sqrt(sn);
    for (int i = 0; i < 4; i++) { q[i] /= qn; s[i] /= sn; }
    for (int i = 0; i < 3; i++) d_dpos[i * (int64_t)n_dyn + j] += dmean[i * (int64_t)n + g];
    /* q' = L(q) s with L(q) the left-multiplication matrix; d s_hat = L(q)^T dq' */
    double L[16] = {q[0], -q[1], -q[2], -q[3],
                    q[1], q[0], -q[3], q[2],
                    q[2], q[3], q[0], -q[1],
                    q[3], -q[2], q[1], q[0]};
    double dsh[4];
    for (int c = 0; c < 4; c++) {
      double acc = 0.0;
      for (int r = 0; r < 4; r++) acc += L[r * 4 + c] * dq[r];
      dsh[c] = acc;
    }
    double dot = s[0] * dsh[0] + s[1] * dsh[1] + s[2] * dsh[2] + s[3] * dsh[3];
    for (int i = 0; i < 4; i++) d_drot[i * (int64_t)n_dyn + j] += (dsh[i] - s[i] * dot) / sn;
  }
}

/* ---------------------------------------------------------------------------------------- */
/* Adam (bias-corrected, 1-based step), elementwise in double.                               */
/* ---------------------------------------------------------------------------------------- */
void orc_adam(int64_t n, double* p, const double* g, double* m, double* v, double lr,
              double beta1, double beta2, double eps, int32_t step) {
  double bc1 = 1.0 - pow(beta1, (double)step), bc2 = 1.0 - pow(beta2, (double)step);
  for (int64_t i = 0; i < n; i++) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = m[i] / bc1, vh = v[i] / bc2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ---------------------------------------------------------------------------------------- */
/* L1 fidelity term of the loss (Eqs. 2/3 with lambda = 0) and the error map E (Sec. 3.4):  */
/* L = (1/V) sum_v mean_{c,p} |render - target|; dL/drender = sign(diff) / (3 H W V);      */
/* E(p) = mean over channels of |render - target|.                                          */
/* ---------------------------------------------------------------------------------------- */
double orc_l1(int32_t n_views, int64_t hw, const float* render, const float* target,
              double* dl, double* err) {
  double loss = 0.0;
  double sc = 1.0 / (3.0 * (double)hw * (double)n_views);
  for (int64_t v = 0; v < n_views; v++) {
    for (int64_t p = 0; p < hw; p++) {
      double e = 0.0;
      for (int c = 0; c < 3; c++) {
        int64_t i = (v * 3 + c) * hw + p;
        double d = (double)render[i] - (double)target[i];
        dl[i] = d > 0.0 ? sc : (d < 0.0 ? -sc : 0.0);
        e += fabs(d);
        loss += fabs(d) * sc;
      }
      err[v * hw + p] = e / 3.0;
    }
  }
  return loss;
}

/* ---------------------------------------------------------------------------------------- */
/* Error-guided densification (Sec. 3.4, Alg. 1, Eq. 4).                                    */
/* ---------------------------------------------------------------------------------------- */

/* Alg. 1: [P,1] T with T the full 4x4 projection (row-vector convention), divide by the    */
/* homogeneous coordinate, x_n = Round(0.5((x_norm+1) W - 1)), y_n with y_norm and H.        */
/* Round(z) = floor(z + 0.5).  Returns 0 if the point is not in front of the camera.        */
static int alg1_pixel(const orc_cam* cam, const double* P, int32_t* xn, int32_t* yn) {
  double R[9], t[3];
  for (int i = 0; i < 9; i++) R[i] = (double)cam->R[i];
  for (int i = 0; i < 3; i++) t[i] = (double)cam->t[i];
  double W = (double)cam->width, H = (double)cam->height;
  double sx = (2.0 * (double)cam->fx) / W, sy = (2.0 * (double)cam->fy) / H;
  double kx = (2.0 * (double)cam->cx + 1.0) / W - 1.0;
  double ky = (2.0 * (double)cam->cy + 1.0) / H - 1.0;
  double T[4][4];
  for (int i = 0; i < 3; i++) {
    T[i][0] = sx * R[0 * 3 + i] + kx * R[2 * 3 + i];
    T[i][1] = sy * R[1 * 3 + i] + ky * R[2 * 3 + i];
    T[i][2] = R[2 * 3 + i];
    T[i][3] = R[2 * 3 + i];
  }
  T[3][0] = sx * t[0] + kx * t[2];
  T[3][1] = sy * t[1] + ky * t[2];
  T[3][2] = t[2];
  T[3][3] = t[2];
  double hom[4];
  for (int c = 0; c < 4; c++) hom[c] = ((P[0] * T[0][c] + P[1] * T[1][c]) + P[2] * T[2][c]) + T[3][c];
  if (!(hom[3] > 0.0)) return 0;
  double xnorm = hom[0] / hom[3], ynorm = hom[1] / hom[3];
  double xf = floor(0.5 * ((xnorm + 1.0) * W - 1.0) + 0.5);
  double yf = floor(0.5 * ((ynorm + 1.0) * H - 1.0) + 0.5);
  if (xf < 0.0 || yf < 0.0 || xf >= W || yf >= H) return 0;
  *xn = (int32_t)xf;
  *yn = (int32_t)yf;
  return 1;
}

void orc_alg1(int32_t n, int64_t stride, const double* mean, const orc_cam* cam, int32_t* xy,
              int32_t* ok) {
  for (int64_t g = 0; g < n; g++) {
    double P[3] = {mean[g], mean[stride + g], mean[2 * stride + g]};
    int32_t x = -1, y = -1;
    ok[g] = alg1_pixel(cam, P, &x, &y);
    xy[2 * g] = x;
    xy[2 * g + 1] = y;
  }
}

/* Selection: returns |S| and writes S ranked by (score desc, index asc) into sel[],
 * score[g] = max over views with an on-image Alg. 1 pixel of E^c there (0 if none).
 * The historical gradient is gbar = sum/count in float (0 if count == 0); the decisions
 * gbar > tau and E > gamma are taken in float, as the kernel takes them. */
typedef struct { float score; int32_t g; } sel_item;
static int sel_cmp(const void* a, const void* b) {
  const sel_item* x = (const sel_item*)a;
  const sel_item* y = (const sel_item*)b;
  if (x->score > y->score) return -1;
  if (x->score < y->score) return 1;
  return (x->g > y->g) - (x->g < y->g);
}

int32_t orc_densify_select(int32_t n_base, int64_t stride, const double* mean, int32_t n_views,
                           const orc_cam* cams, const float* err /*[V][H][W]*/,
                           const float* gradnorm_sum, const int32_t* grad_count,
                           float gamma_err, float tau_pos, float tau_err, int32_t* sel,
                           float* score_out, int32_t* in_err_out) {
  sel_item* items = (sel_item*)malloc(sizeof(sel_item) * (n_base > 0 ? n_base : 1));
  int32_t ns = 0;
  int64_t off = 0;
  for (int64_t g = 0; g < n_base; g++) {
    double P[3] = {mean[g], mean[stride + g], mean[2 * stride + g]};
    int in_err = 0;
    float score = 0.0f;
    off = 0;
    for (int c = 0; c < n_views; c++) {
      int32_t x, y;
      int64_t hw = (int64_t)cams[c].width * cams[c].height;
      if (alg1_pixel(&cams[c], P, &x, &y)) {
        float e = err[off + (int64_t)y * cams[c].width + x];
        if (e > gamma_err) in_err = 1;
        if (e > score) score = e;
      }
      off += hw;
    }
    float gbar = grad_count[g] > 0 ? gradnorm_sum[g] / (float)grad_count[g] : 0.0f;
    int in_s = (gbar > tau_pos) || (in_err && gbar > tau_err);
    if (score_out) score_out[g] = score;
    if (in_err_out) in_err_out[g] = in_err;
    if (in_s) { items[ns].score = score; items[ns].g = (int32_t)g; ns++; }
  }
  qsort(items, ns, sizeof(sel_item), sel_cmp);
  for (int i = 0; i < ns; i++) sel[i] = items[i].g;
  free(items);
  return ns;
}

/* SplitMix64 (Steele, Lea, Flood 2014): output i of the stream seeded with s is
 * mix(s + (i+1) * 0x9E3779B97F4A7C15). */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static double unif53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Standard normals of child j: Box-Muller on draws 4j..4j+3 of the stream. */
void orc_child_normals(uint64_t seed, int64_t j, double* z /*[3]*/) {
  double u0 = 1.0 - unif53(orc_splitmix64(seed, 4 * j + 0));
  double u1 = unif53(orc_splitmix64(seed, 4 * j + 1));
  double u2 = 1.0 - unif53(orc_splitmix64(seed, 4 * j + 2));
  double u3 = unif53(orc_splitmix64(seed, 4 * j + 3));
  const double TWO_PI = 6.28318530717958647692;
  double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  z[0] = r0 * cos(TWO_PI * u1);
  z[1] = r0 * sin(TWO_PI * u1);
  z[2] = r1 * cos(TWO_PI * u3);
}

/* Spawn densification: child j copies parent sel[j mod ns]; its mean moves by R diag(s) z,
 * its log-scale drops by ln 1.6.  Writes children into rows [n, n + n_app) of the planes
 * (stride = capacity).  Returns n_app = 0 if ns == 0 else min(k_max, capacity - n). */
int32_t orc_spawn(int32_t n, int32_t capacity, int64_t stride, float* mean, float* quat,
                  float* log_scale, float* logit, float* sh, int32_t n_sh_planes,
                  const int32_t* sel, int32_t ns, int32_t k_max, uint64_t seed, double* child_mean) {
  if (ns <= 0) return 0;
  int32_t n_app = capacity - n < k_max ? capacity - n : k_max;
  if (n_app < 0) n_app = 0;
  const double LN16 = log(1.6);
  for (int64_t j = 0; j < n_app; j++) {
    int64_t p = sel[j % ns], c = n + j;
    double q[4], qn = 0.0, s[3], R[9], z[3];
    for (int i = 0; i < 4; i++) { q[i] = quat[i * stride + p]; qn += q[i] * q[i]; }
    qn = sqrt(qn);
    for (int i = 0; i < 4; i++) q[i] /= qn;
    quat_to_rot(q, R);
    for (int i = 0; i < 3; i++) s[i] = exp(log_scale[i * stride + p]);
    orc_child_normals(seed, j, z);
    for (int i = 0; i < 3; i++) {
      double off = R[i * 3 + 0] * s[0] * z[0] + R[i * 3 + 1] * s[1] * z[1] + R[i * 3 + 2] * s[2] * z[2];
      double m = mean[i * stride + p] + off;
      if (child_mean) child_mean[i * (int64_t)k_max + j] = m; /* [3][k_max] */
      mean[i * stride + c] = (float)m;
    }
    for (int i = 0; i < 4; i++) quat[i * stride + c] = quat[i * stride + p];
    for (int i = 0; i < 3; i++) log_scale[i * stride + c] = (float)((double)log_scale[i * stride + p] - LN16);
    logit[c] = logit[p];
    for (int k = 0; k < n_sh_planes; k++) sh[k * stride + c] = sh[k * stride + p];
  }
  return n_app;
}
