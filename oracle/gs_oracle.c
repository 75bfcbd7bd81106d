/*
 * FP64 CPU oracle for the per-frame Gaussian-splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark have an independent, obviously-correct
 * reference.  It shares no code, header, table or constant generator with the
 * HIP library.
 *
 * What it follows.  AirGS (arXiv 2512.20943) trains and streams a dynamic
 * scene as anchor Gaussians plus per-frame attribute deltas:
 *   - Gaussian primitive {mu, alpha, c, SH, R, S}: Sec. II (Background);
 *   - frame = anchor + accumulated deltas: Eq. (2), Eq. (5), Eq. (12);
 *   - one texel per Gaussian, same location in every attribute image:
 *     Eq. (3) and Sec. III-C;
 *   - pruned deltas d'_t = p(...): Eq. (11), Sec. III-C;
 *   - L1 photometric term: Eq. (1).
 * The paper cites the 3DGS differentiable splatting renderer (Sec. II) but
 * does not define it, so the rasterizer below is written out from standard
 * mathematics: EWA splatting (Zwicker et al. 2001), real orthonormal
 * spherical harmonics, Hamilton quaternion algebra, front-to-back alpha
 * compositing and Adam (Kingma & Ba 2015).  Every constant the paper leaves
 * open (near plane 0.2, dilation 0.3 px^2, radius 3 sqrt(lambda_max) with
 * eigenvalue floor 0.1, alpha cap 0.99, skip below 1/255, stop below
 * transmittance 1e-4, 16x16 tiles, guard band 1.3) is a stated reading.
 *
 * Precision.  All arithmetic is IEEE FP64, built with -ffp-contract=off.
 * The two places where a result is stored at parameter precision are named:
 * the applied frame is rounded to FP32 (it is a set of FP32 parameters), and
 * the depth key is the FP32 rounding of camera-space z.
 *
 * Pins (tests/test_oracle_*.py): rotation orthonormality and the textbook
 * z-rotation; analytic J W Sigma W^T J^T; SH orthonormality by quadrature and
 * the addition theorem; a centred Gaussian compositing to opacity x colour;
 * two Gaussians on one ray; prod(1 - alpha) = final T; the alpha = 0.8 stack
 * stopping after 5; brute-force per-pixel depth sort = tiled result; central
 * finite differences of the whole forward in FP64; apply identities
 * (additive composition, R(dq (x) q) = R(dq) R(q), masked texels bit-exact);
 * closed forms for L1 and the first Adam step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TILE 16
#define OR_NEAR 0.2
#define OR_DILATE 0.3
#define OR_GUARD 1.3
#define OR_ALPHA_MAX 0.99
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_T_STOP 1e-4

/* flag bits of a projected (view, Gaussian) record */
#define OR_F_CLAMP_R 1u
#define OR_F_CLAMP_G 2u
#define OR_F_CLAMP_B 4u
#define OR_F_CLAMP_U 8u
#define OR_F_CLAMP_V 16u
#define OR_F_VISIBLE 32u

/* ------------------------------------------------------------------------ */
/* Camera: world->camera x_c = R mu + t (OpenCV frame: x right, y down, z     */
/* forward), pinhole intrinsics fx, fy, cx, cy, image width/height.  Passed   */
/* as separate arrays: R (V,9) row-major, t (V,3), f (V,4) = fx,fy,cx,cy,     */
/* wh (V,2).                                                                 */
/* ------------------------------------------------------------------------ */

static int tiles_x(int w) { return (w + OR_TILE - 1) / OR_TILE; }

static float round_to_f32(double x) { return (float)x; }

static uint32_t f32_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* ------------------------------------------------------------------------ */
/* Quaternion algebra (Hamilton product, (w, x, y, z) order).                 */
/* ------------------------------------------------------------------------ */

/* out = a (x) b */
static void quat_mul(const double a[4], const double b[4], double out[4]) {
  out[0] = ((a[0] * b[0] - a[1] * b[1]) - a[2] * b[2]) - a[3] * b[3];
  out[1] = ((a[0] * b[1] + a[1] * b[0]) + a[2] * b[3]) - a[3] * b[2];
  out[2] = ((a[0] * b[2] - a[1] * b[3]) + a[2] * b[0]) + a[3] * b[1];
  out[3] = ((a[0] * b[3] + a[1] * b[2]) - a[2] * b[1]) + a[3] * b[0];
}

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(double w, double x, double y, double z, double R[9]) {
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void or_quat_to_rot(const double* q, double* R) {
  double n = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  quat_to_rot(q[0] / n, q[1] / n, q[2] / n, q[3] / n, R);
}

void or_quat_mul(const double* a, const double* b, double* out) { quat_mul(a, b, out); }

/* ------------------------------------------------------------------------ */
/* Real orthonormal spherical harmonics on the unit vector (x, y, z),         */
/* coefficient index l*l + l + m, m = -l..l.                                 */
/* ------------------------------------------------------------------------ */

#define OR_PI 3.14159265358979323846

static void sh_basis(int deg, double x, double y, double z, double* Y) {
  const double c00 = 0.5 * sqrt(1.0 / OR_PI);
  const double c1 = sqrt(3.0 / (4.0 * OR_PI));
  Y[0] = c00;
  if (deg < 1) return;
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (deg < 2) return;
  {
    const double a = 0.5 * sqrt(15.0 / OR_PI);
    const double b = 0.25 * sqrt(5.0 / OR_PI);
    const double c = 0.25 * sqrt(15.0 / OR_PI);
    Y[4] = a * x * y;
    Y[5] = a * y * z;
    Y[6] = b * (3.0 * z * z - 1.0);
    Y[7] = a * x * z;
    Y[8] = c * (x * x - y * y);
  }
  if (deg < 3) return;
  {
    const double a = 0.25 * sqrt(35.0 / (2.0 * OR_PI));
    const double b = 0.5 * sqrt(105.0 / OR_PI);
    const double c = 0.25 * sqrt(21.0 / (2.0 * OR_PI));
    const double d = 0.25 * sqrt(7.0 / OR_PI);
    const double e = 0.25 * sqrt(105.0 / OR_PI);
    Y[9] = a * y * (3.0 * x * x - y * y);
    Y[10] = b * x * y * z;
    Y[11] = c * y * (5.0 * z * z - 1.0);
    Y[12] = d * z * (5.0 * z * z - 3.0);
    Y[13] = c * x * (5.0 * z * z - 1.0);
    Y[14] = e * z * (x * x - y * y);
    Y[15] = a * x * (x * x - 3.0 * y * y);
  }
}

/* Gradient of each basis polynomial w.r.t. (x, y, z): dY[k*3 + axis]. */
static void sh_basis_grad(int deg, double x, double y, double z, double* dY) {
  int K = (deg + 1) * (deg + 1);
  for (int i = 0; i < 3 * K; ++i) dY[i] = 0.0;
  if (deg < 1) return;
  {
    const double c1 = sqrt(3.0 / (4.0 * OR_PI));
    dY[1 * 3 + 1] = c1;
    dY[2 * 3 + 2] = c1;
    dY[3 * 3 + 0] = c1;
  }
  if (deg < 2) return;
  {
    const double a = 0.5 * sqrt(15.0 / OR_PI);
    const double b = 0.25 * sqrt(5.0 / OR_PI);
    const double c = 0.25 * sqrt(15.0 / OR_PI);
    dY[4 * 3 + 0] = a * y;
    dY[4 * 3 + 1] = a * x;
    dY[5 * 3 + 1] = a * z;
    dY[5 * 3 + 2] = a * y;
    dY[6 * 3 + 2] = b * 6.0 * z;
    dY[7 * 3 + 0] = a * z;
    dY[7 * 3 + 2] = a * x;
    dY[8 * 3 + 0] = c * 2.0 * x;
    dY[8 * 3 + 1] = -c * 2.0 * y;
  }
  if (deg < 3) return;
  {
    const double a = 0.25 * sqrt(35.0 / (2.0 * OR_PI));
    const double b = 0.5 * sqrt(105.0 / OR_PI);
    const double c = 0.25 * sqrt(21.0 / (2.0 * OR_PI));
    const double d = 0.25 * sqrt(7.0 / OR_PI);
    const double e = 0.25 * sqrt(105.0 / OR_PI);
    /* y (3x^2 - y^2) */
    dY[9 * 3 + 0] = a * 6.0 * x * y;
    dY[9 * 3 + 1] = a * (3.0 * x * x - 3.0 * y * y);
    /* x y z */
    dY[10 * 3 + 0] = b * y * z;
    dY[10 * 3 + 1] = b * x * z;
    dY[10 * 3 + 2] = b * x * y;
    /* y (5z^2 - 1) */
    dY[11 * 3 + 1] = c * (5.0 * z * z - 1.0);
    dY[11 * 3 + 2] = c * 10.0 * y * z;
    /* z (5z^2 - 3) */
    dY[12 * 3 + 2] = d * (15.0 * z * z - 3.0);
    /* x (5z^2 - 1) */
    dY[13 * 3 + 0] = c * (5.0 * z * z - 1.0);
    dY[13 * 3 + 2] = c * 10.0 * x * z;
    /* z (x^2 - y^2) */
    dY[14 * 3 + 0] = e * 2.0 * x * z;
    dY[14 * 3 + 1] = -e * 2.0 * y * z;
    dY[14 * 3 + 2] = e * (x * x - y * y);
    /* x (x^2 - 3y^2) */
    dY[15 * 3 + 0] = a * (3.0 * x * x - 3.0 * y * y);
    dY[15 * 3 + 1] = -a * 6.0 * x * y;
  }
}

void or_sh_basis(int deg, const double* dir, double* Y) { sh_basis(deg, dir[0], dir[1], dir[2], Y); }

/* ------------------------------------------------------------------------ */
/* Step 1: apply a frame update.  Eq. (2)/(5)/(12): the frame is the anchor   */
/* plus the accumulated (pruned) delta; attribute images hold one texel per   */
/* Gaussian (Eq. (3)).  Channels 0-2 add to the mean, 3-6 are a quaternion    */
/* delta composed on the left, 7 adds to the opacity logit.  mask = 1 keeps   */
/* the texel's update, 0 drops it (pruning, Eq. (11)).  Gaussian i lives at   */
/* texel (i / gw, i % gw).  Result rounded to FP32 parameter storage.         */
/* ------------------------------------------------------------------------ */
void or_apply(int n, int ld, const float* mean, const float* quat, const float* opac,
              const float* delta, const uint8_t* mask, int gw, int gh,
              float* mean_out, float* quat_out, float* opac_out) {
  const size_t plane = (size_t)gw * (size_t)gh;
  for (int i = 0; i < n; ++i) {
    if (mask[i]) {
      for (int k = 0; k < 3; ++k)
        mean_out[(size_t)k * ld + i] =
            round_to_f32((double)mean[(size_t)k * ld + i] + (double)delta[(size_t)k * plane + i]);
      double dq[4], q[4], r[4];
      for (int k = 0; k < 4; ++k) {
        dq[k] = (double)delta[(size_t)(3 + k) * plane + i];
        q[k] = (double)quat[(size_t)k * ld + i];
      }
      quat_mul(dq, q, r);
      for (int k = 0; k < 4; ++k) quat_out[(size_t)k * ld + i] = round_to_f32(r[k]);
      opac_out[i] = round_to_f32((double)opac[i] + (double)delta[(size_t)7 * plane + i]);
    } else {
      for (int k = 0; k < 3; ++k) mean_out[(size_t)k * ld + i] = mean[(size_t)k * ld + i];
      for (int k = 0; k < 4; ++k) quat_out[(size_t)k * ld + i] = quat[(size_t)k * ld + i];
      opac_out[i] = opac[i];
    }
  }
  (void)gh;
}

/* ------------------------------------------------------------------------ */
/* Steps 2-6: projection of one (view, Gaussian).                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  double xc[3];      /* camera-space centre */
  double Rq[9];      /* rotation of the normalised quaternion */
  double qhat[4];    /* normalised quaternion */
  double qnorm;
  double sigma[3];   /* exp(log-scale) */
  double M[9];       /* R_q diag(sigma) */
  double Sigma[9];   /* 3D covariance */
  double V[9];       /* W Sigma W^T */
  double J[6];       /* 2x3 EWA Jacobian */
  double u, v;       /* (possibly clamped) x/z, y/z */
  int clamp_u, clamp_v;
  double a, b, c;    /* raw 2D covariance */
  double ap, cp;     /* dilated diagonal */
  double det;
  double conic[3];
  double p[2];
  int radius;
  int rect[4];
  int tiles;
  double dir[3];     /* unit view direction, world space */
  double dist;       /* |mu - c_v| */
  double raw[3];     /* SH colour before the clamp */
  double rgb[3];
  double alpha_hat;  /* sigmoid(opacity logit) */
  double depth;
  int visible;
} or_proj;

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Full projection of Gaussian (mean m, log-scale s, quaternion q, logit o,
 * SH coefficients sh[k*3 + ch]) into camera (R, t, f, wh).  Returns 0 when
 * the Gaussian is culled (the record is then only partly filled). */
static int project_one(const double m[3], const double s[3], const double q[4], double o,
                       const double* sh, int deg, const double* R, const double* t,
                       const double* f, const int* wh, or_proj* P) {
  const int W = wh[0], H = wh[1];
  const double fx = f[0], fy = f[1], cx = f[2], cy = f[3];
  memset(P, 0, sizeof(*P));
  P->alpha_hat = sigmoid(o);
  /* step 2: camera space, near cull */
  for (int k = 0; k < 3; ++k)
    P->xc[k] = ((R[3 * k + 0] * m[0] + R[3 * k + 1] * m[1]) + R[3 * k + 2] * m[2]) + t[k];
  const double z = P->xc[2];
  P->depth = z;
  if (!(z > OR_NEAR)) return 0;
  /* step 3: 3D covariance */
  P->qnorm = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  if (!(P->qnorm >= 1e-8)) return 0;
  for (int k = 0; k < 4; ++k) P->qhat[k] = q[k] / P->qnorm;
  quat_to_rot(P->qhat[0], P->qhat[1], P->qhat[2], P->qhat[3], P->Rq);
  for (int k = 0; k < 3; ++k) P->sigma[k] = exp(s[k]);
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) P->M[3 * r + cc] = P->Rq[3 * r + cc] * P->sigma[cc];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc)
      P->Sigma[3 * r + cc] = (P->M[3 * r + 0] * P->M[3 * cc + 0] + P->M[3 * r + 1] * P->M[3 * cc + 1]) +
                             P->M[3 * r + 2] * P->M[3 * cc + 2];
  /* V = W Sigma W^T with W the camera rotation */
  double T1[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc)
      T1[3 * r + cc] = (R[3 * r + 0] * P->Sigma[0 * 3 + cc] + R[3 * r + 1] * P->Sigma[1 * 3 + cc]) +
                       R[3 * r + 2] * P->Sigma[2 * 3 + cc];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc)
      P->V[3 * r + cc] = (T1[3 * r + 0] * R[3 * cc + 0] + T1[3 * r + 1] * R[3 * cc + 1]) +
                         T1[3 * r + 2] * R[3 * cc + 2];
  /* step 4: EWA Jacobian with guard band */
  const double limx = OR_GUARD * ((0.5 * (double)W) / fx);
  const double limy = OR_GUARD * ((0.5 * (double)H) / fy);
  double u = P->xc[0] / z, v = P->xc[1] / z;
  if (u < -limx) { u = -limx; P->clamp_u = 1; }
  if (u > limx) { u = limx; P->clamp_u = 1; }
  if (v < -limy) { v = -limy; P->clamp_v = 1; }
  if (v > limy) { v = limy; P->clamp_v = 1; }
  P->u = u;
  P->v = v;
  P->J[0] = fx / z; P->J[1] = 0.0; P->J[2] = -(fx * u) / z;
  P->J[3] = 0.0;    P->J[4] = fy / z; P->J[5] = -(fy * v) / z;
  double T2[6], cov[4];
  for (int r = 0; r < 2; ++r)
    for (int cc = 0; cc < 3; ++cc)
      T2[3 * r + cc] = (P->J[3 * r + 0] * P->V[0 * 3 + cc] + P->J[3 * r + 1] * P->V[1 * 3 + cc]) +
                       P->J[3 * r + 2] * P->V[2 * 3 + cc];
  for (int r = 0; r < 2; ++r)
    for (int cc = 0; cc < 2; ++cc)
      cov[2 * r + cc] = (T2[3 * r + 0] * P->J[3 * cc + 0] + T2[3 * r + 1] * P->J[3 * cc + 1]) +
                        T2[3 * r + 2] * P->J[3 * cc + 2];
  P->a = cov[0];
  P->b = cov[1];
  P->c = cov[3];
  P->ap = P->a + OR_DILATE;
  P->cp = P->c + OR_DILATE;
  P->det = P->ap * P->cp - P->b * P->b;
  if (!(P->det > 0.0)) return 0;
  const double inv = 1.0 / P->det;
  P->conic[0] = P->cp * inv;
  P->conic[1] = -P->b * inv;
  P->conic[2] = P->ap * inv;
  P->p[0] = (fx * P->xc[0]) / z + cx;
  P->p[1] = (fy * P->xc[1]) / z + cy;
  /* step 5: radius and tile rectangle */
  const double mid = 0.5 * (P->ap + P->cp);
  double disc = mid * mid - P->det;
  if (disc < 0.1) disc = 0.1;
  const double lam = mid + sqrt(disc);
  P->radius = (int)ceil(3.0 * sqrt(lam));
  const int TX = tiles_x(W), TY = tiles_x(H);
  const double r = (double)P->radius;
  double b0 = floor((P->p[0] - r) / (double)OR_TILE);
  double b1 = floor((P->p[0] + r) / (double)OR_TILE) + 1.0;
  double b2 = floor((P->p[1] - r) / (double)OR_TILE);
  double b3 = floor((P->p[1] + r) / (double)OR_TILE) + 1.0;
  b0 = b0 < 0.0 ? 0.0 : (b0 > TX ? TX : b0);
  b1 = b1 < 0.0 ? 0.0 : (b1 > TX ? TX : b1);
  b2 = b2 < 0.0 ? 0.0 : (b2 > TY ? TY : b2);
  b3 = b3 < 0.0 ? 0.0 : (b3 > TY ? TY : b3);
  P->rect[0] = (int)b0;
  P->rect[1] = (int)b2;
  P->rect[2] = (int)b1;
  P->rect[3] = (int)b3;
  P->tiles = (P->rect[2] - P->rect[0]) * (P->rect[3] - P->rect[1]);
  if (P->tiles <= 0) {
    P->tiles = 0;
    return 0;
  }
  /* step 6: SH colour along the world-space view direction */
  double cvec[3];
  for (int k = 0; k < 3; ++k)
    cvec[k] = -((R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1]) + R[2 * 3 + k] * t[2]);
  double d[3] = {m[0] - cvec[0], m[1] - cvec[1], m[2] - cvec[2]};
  P->dist = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) P->dir[k] = d[k] / P->dist;
  double Y[16];
  sh_basis(deg, P->dir[0], P->dir[1], P->dir[2], Y);
  const int K = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
    for (int k = 0; k < K; ++k) acc += Y[k] * sh[k * 3 + ch];
    P->raw[ch] = acc;
    P->rgb[ch] = acc > 0.0 ? acc : 0.0;
  }
  P->visible = 1;
  return 1;
}

/* Gather Gaussian i's parameters from planar FP32 storage. */
static void gather_params(int i, int ld, int deg, const float* mean, const float* lsc,
                          const float* quat, const float* opac, const float* sh, double m[3],
                          double s[3], double q[4], double* o, double* shv) {
  const int K = (deg + 1) * (deg + 1);
  for (int k = 0; k < 3; ++k) {
    m[k] = mean[(size_t)k * ld + i];
    s[k] = lsc[(size_t)k * ld + i];
  }
  for (int k = 0; k < 4; ++k) q[k] = quat[(size_t)k * ld + i];
  *o = opac[i];
  for (int k = 0; k < K; ++k)
    for (int ch = 0; ch < 3; ++ch) shv[k * 3 + ch] = sh[((size_t)k * 3 + ch) * ld + i];
}

/*
 * Projection of n Gaussians into V views.  Outputs (index v*n + i):
 *   mean2d (.,2), conic (.,3) = (A, B, C) with power = -(A dx^2 + C dy^2)/2 - B dx dy,
 *   rgb (.,3), alpha_hat (.), depth (.), depth_bits (.) = bits of FP32(z),
 *   rect (.,4) = tx0, ty0, tx1, ty1 (exclusive upper), tiles (.), radius (.),
 *   flags (.) (clamp bits, visible bit).
 */
void or_project(int n, int ld, int deg, const float* mean, const float* lsc, const float* quat,
                const float* opac, const float* sh, int V, const double* camR,
                const double* camt, const double* camf, const int* camwh, double* mean2d,
                double* conic, double* rgb, double* alpha_hat, double* depth,
                uint32_t* depth_bits, int* rect, int* tiles, int* radius, uint8_t* flags) {
  for (int v = 0; v < V; ++v) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double m[3], s[3], q[4], o, shv[48];
      or_proj P;
      gather_params(i, ld, deg, mean, lsc, quat, opac, sh, m, s, q, &o, shv);
      int vis = project_one(m, s, q, o, shv, deg, camR + 9 * v, camt + 3 * v, camf + 4 * v,
                            camwh + 2 * v, &P);
      const size_t j = (size_t)v * n + i;
      mean2d[2 * j] = P.p[0];
      mean2d[2 * j + 1] = P.p[1];
      for (int k = 0; k < 3; ++k) {
        conic[3 * j + k] = P.conic[k];
        rgb[3 * j + k] = P.rgb[k];
      }
      alpha_hat[j] = P.alpha_hat;
      depth[j] = P.depth;
      depth_bits[j] = f32_bits(round_to_f32(P.depth));
      uint8_t fl = 0;
      if (vis) {
        for (int k = 0; k < 4; ++k) rect[4 * j + k] = P.rect[k];
        tiles[j] = P.tiles;
        radius[j] = P.radius;
        fl |= OR_F_VISIBLE;
        if (P.raw[0] <= 0.0) fl |= OR_F_CLAMP_R;
        if (P.raw[1] <= 0.0) fl |= OR_F_CLAMP_G;
        if (P.raw[2] <= 0.0) fl |= OR_F_CLAMP_B;
        if (P.clamp_u) fl |= OR_F_CLAMP_U;
        if (P.clamp_v) fl |= OR_F_CLAMP_V;
      } else {
        for (int k = 0; k < 4; ++k) rect[4 * j + k] = 0;
        tiles[j] = 0;
        radius[j] = 0;
      }
      flags[j] = fl;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Step 5b (optional): tile sets narrower than the rectangle.                 */
/*                                                                            */
/* Step 8 skips a Gaussian at every pixel where its alpha stays below 1/255, */
/* so listing it in a tile none of whose pixels reach that level changes no   */
/* image, transmittance or gradient; only the list positions (n_contrib)      */
/* count a shorter list.  With q(d) = A dx^2 + 2 B dx dy + C dy^2 the conic's */
/* quadratic form (power = -q/2), alpha >= 1/255 needs q <= qm,               */
/* qm = 2 ln(255 alpha_hat); the sets below use the widened ellipse           */
/*   E = { d : q(d) <= thr },  thr = qm + 2e-4 |qm| + 1e-3,                    */
/* whose margin covers an FP32 evaluation of alpha.  D = AC - B^2 > 0.        */
/*   mode 1: the rectangle of step 5 cut to the tiles that meet E's bounding  */
/*           box, x in px +- sqrt(thr C / D), y in py +- sqrt(thr A / D);     */
/*           no tile at all when thr <= 0 (alpha_hat below about 1/255).     */
/*   mode 2: mode 1, then a rectangle of at most OR_SPAN_ROWS tile rows and   */
/*           OR_SPAN_COLS tile columns keeps, in tile row ty, only the        */
/*           columns tx whose pixel centres x in [16 tx, 16 tx + 15] come     */
/*           within OR_SPAN_SLACK px of E's x-extent over the band            */
/*           y in [16 ty - 0.5, 16 ty + 15.5] (a row whose band misses E's    */
/*           y-range by more than the slack keeps none).                      */
/* Every pixel with q <= thr lies in a kept tile (its row's band holds it and */
/* its x lies in the chord of E at its y).  E's chord at offset y is           */
/* x in ((-B y - h) / A, (-B y + h) / A), h = sqrt(A thr - D y^2); its right   */
/* end is concave in y with maximum sqrt(thr C / D) at y = -B sqrt(thr C/D)/C,*/
/* and the left end mirrors it, so over a band the extreme is either that     */
/* point or the chord at one of the band's ends (clamped into E's y-range).   */
/* Records that keep no tile are culled.  spans (V*n, OR_SPAN_ROWS, 2) hold  */
/* absolute [first, end) columns per row of the rectangle; OR_F_SPANS in      */
/* flags marks the records that use them.                                     */
/* ------------------------------------------------------------------------ */
#define OR_SPAN_ROWS 4
#define OR_SPAN_COLS 15
#define OR_SPAN_SLACK 1e-3
#define OR_F_SPANS 64u

static double clamp_d(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ends of E's chord at offset y (clamped into E's y-range [-ey, ey]) */
static void chord_ends(double A, double B, double D, double thr, double ey, double y, double* xl,
                       double* xr, double* yc) {
  const double yy = clamp_d(y, -ey, ey);
  double hh = A * thr - D * yy * yy;
  if (hh < 0.0) hh = 0.0;
  const double h = sqrt(hh);
  *xr = (-B * yy + h) / A;
  *xl = (-B * yy - h) / A;
  *yc = yy;
}

void or_tile_sets(int V, int n, const int* camwh, const double* mean2d, const double* conic,
                  const double* alpha_hat, int mode, int* rect, int* tiles, int* spans,
                  uint8_t* flags) {
  for (int v = 0; v < V; ++v) {
    const double TX = (double)tiles_x(camwh[2 * v]), TY = (double)tiles_x(camwh[2 * v + 1]);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      const size_t j = (size_t)v * n + i;
      int* sp = spans + (size_t)2 * OR_SPAN_ROWS * j;
      for (int k = 0; k < 2 * OR_SPAN_ROWS; ++k) sp[k] = 0;
      if (mode <= 0 || tiles[j] <= 0) continue;
      const double px = mean2d[2 * j], py = mean2d[2 * j + 1];
      const double A = conic[3 * j], B = conic[3 * j + 1], C = conic[3 * j + 2];
      const double D = A * C - B * B;
      const double qm = 2.0 * (log(255.0) + log(alpha_hat[j]));
      const double thr = qm + 2e-4 * fabs(qm) + 1e-3;
      int* r = rect + 4 * j;
      double x0 = r[0], y0 = r[1], x1 = r[2], y1 = r[3];
      double ex = 0.0, ey = 0.0;
      if (thr > 0.0) {
        ex = sqrt(thr * C / D);
        ey = sqrt(thr * A / D);
        x0 = fmax(x0, clamp_d(floor((px - ex) / (double)OR_TILE), 0.0, TX));
        x1 = fmin(x1, clamp_d(floor((px + ex) / (double)OR_TILE) + 1.0, 0.0, TX));
        y0 = fmax(y0, clamp_d(floor((py - ey) / (double)OR_TILE), 0.0, TY));
        y1 = fmin(y1, clamp_d(floor((py + ey) / (double)OR_TILE) + 1.0, 0.0, TY));
      } else {
        x1 = x0;
      }
      int cnt = 0;
      if (x1 > x0 && y1 > y0) {
        cnt = (int)((x1 - x0) * (y1 - y0));
        if (mode >= 2 && y1 - y0 <= OR_SPAN_ROWS && x1 - x0 <= OR_SPAN_COLS) {
          const double ys = -B * ex / C; /* offset of E's rightmost point */
          cnt = 0;
          for (int row = 0; row < (int)(y1 - y0); ++row) {
            const double ty = y0 + row;
            const double lo = ((double)OR_TILE * ty - 0.5) - py;
            const double hi = ((double)OR_TILE * ty + 15.5) - py;
            if (lo > ey + OR_SPAN_SLACK || hi < -ey - OR_SPAN_SLACK) continue;
            double l0, r0, c0, l1, r1, c1;
            chord_ends(A, B, D, thr, ey, lo, &l0, &r0, &c0);
            chord_ends(A, B, D, thr, ey, hi, &l1, &r1, &c1);
            const double xmax = (ys >= c0 && ys <= c1) ? ex : fmax(r0, r1);
            const double xmin = (-ys >= c0 && -ys <= c1) ? -ex : fmin(l0, l1);
            const double a =
                fmax(x0, ceil((((px + xmin) - OR_SPAN_SLACK) - (double)(OR_TILE - 1)) /
                              (double)OR_TILE));
            const double b = fmin(x1, floor(((px + xmax) + OR_SPAN_SLACK) / (double)OR_TILE) + 1.0);
            if (b > a) {
              sp[2 * row] = (int)a;
              sp[2 * row + 1] = (int)b;
              cnt += (int)(b - a);
            }
          }
          flags[j] |= OR_F_SPANS;
        }
      }
      if (cnt <= 0) {
        r[0] = r[1] = r[2] = r[3] = 0;
        tiles[j] = 0;
        flags[j] = 0;
        for (int k = 0; k < 2 * OR_SPAN_ROWS; ++k) sp[k] = 0;
        continue;
      }
      r[0] = (int)x0;
      r[1] = (int)y0;
      r[2] = (int)x1;
      r[3] = (int)y1;
      tiles[j] = cnt;
    }
  }
}

/* Column range [*a, *b) of tile row ty in record j's tile set. */
static void row_columns(const int* r, const int* sp, int spanned, int ty, int* a, int* b) {
  if (spanned) {
    *a = sp[2 * (ty - r[1])];
    *b = sp[2 * (ty - r[1]) + 1];
  } else {
    *a = r[0];
    *b = r[2];
  }
}

/* ------------------------------------------------------------------------ */
/* Step 7: binning and depth-keyed ordering.  Every (Gaussian, tile) pair of  */
/* a visible Gaussian's tile set (its rectangle, or per-row spans of step 5b) */
/* is one instance, key = (segment << 32) |                                   */
/* depth bits, segment = seg_base[v] + ty*TX_v + tx.  The defining order is   */
/* ascending (key, Gaussian id); a comparison sort on that pair gives it.      */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t key;
  uint32_t val;
} or_inst;

static int inst_cmp(const void* pa, const void* pb) {
  const or_inst* a = (const or_inst*)pa;
  const or_inst* b = (const or_inst*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->val != b->val) return a->val < b->val ? -1 : 1;
  return 0;
}

/* Count of instances for the given rectangles. */
int64_t or_count_instances(int V, int n, const int* tiles) {
  int64_t M = 0;
  for (size_t j = 0; j < (size_t)V * n; ++j) M += tiles[j];
  return M;
}

/* seg_base (V) = first segment of each view; TXv (V) = tiles per row.
 * keys/vals have room for M = or_count_instances(...); ranges (n_seg, 2). */
void or_bin_sort(int V, int n, const uint32_t* depth_bits, const int* rect, const int* tiles,
                 const int* spans, const uint8_t* flags, const int64_t* seg_base, const int* TXv,
                 int64_t n_seg, uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
  int64_t M = or_count_instances(V, n, tiles);
  or_inst* a = (or_inst*)malloc(sizeof(or_inst) * (size_t)(M > 0 ? M : 1));
  int64_t w = 0;
  for (int v = 0; v < V; ++v)
    for (int i = 0; i < n; ++i) {
      const size_t j = (size_t)v * n + i;
      if (tiles[j] <= 0) continue;
      const int* r = rect + 4 * j;
      const int spanned = spans && flags && (flags[j] & OR_F_SPANS);
      for (int ty = r[1]; ty < r[3]; ++ty) {
        int c0, c1;
        row_columns(r, spans ? spans + (size_t)2 * OR_SPAN_ROWS * j : NULL, spanned, ty, &c0, &c1);
        for (int tx = c0; tx < c1; ++tx) {
          uint64_t seg = (uint64_t)(seg_base[v] + (int64_t)ty * TXv[v] + tx);
          a[w].key = (seg << 32) | (uint64_t)depth_bits[j];
          a[w].val = (uint32_t)i;
          ++w;
        }
      }
    }
  qsort(a, (size_t)M, sizeof(or_inst), inst_cmp);
  for (int64_t s = 0; s < n_seg; ++s) {
    ranges[2 * s] = 0;
    ranges[2 * s + 1] = 0;
  }
  for (int64_t k = 0; k < M; ++k) {
    keys[k] = a[k].key;
    vals[k] = a[k].val;
    uint64_t seg = a[k].key >> 32;
    if (k == 0 || (a[k - 1].key >> 32) != seg) ranges[2 * seg] = (uint32_t)k;
    if (k == M - 1 || (a[k + 1].key >> 32) != seg) ranges[2 * seg + 1] = (uint32_t)(k + 1);
  }
  free(a);
}

/* ------------------------------------------------------------------------ */
/* Step 8: front-to-back compositing of one pixel over an ordered list.       */
/* near[0] is set when any decision lies within a relative margin of its      */
/* threshold (those pixels can legitimately differ between FP32 and FP64).    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const double* mean2d;
  const double* conic;
  const double* rgb;
  const double* alpha_hat;
} or_splats;

/* Margins of the near-threshold report.  An FP32 evaluation of alpha carries
 * a relative error of order OR_ERR_ALPHA (power, exp and log rounding); the
 * relative error of T after compositing grows with sum alpha/(1-alpha) over
 * the composited entries, so the stop test is reported near its threshold
 * when |T(1-alpha) - 1e-4| is within that propagated bound. */
#define OR_NEAR_REL 2e-4
#define OR_ERR_ALPHA 2e-5

static void composite_pixel(const or_splats* S, const uint32_t* list, int len, double px,
                            double py, const double bg[3], double out_c[3], double* out_T,
                            int* out_n, int* near_thr, int64_t* usage) {
  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  double cond = 0.0; /* sum of alpha/(1-alpha) over composited entries */
  int last = 0;
  for (int j = 0; j < len; ++j) {
    const uint32_t g = list[j];
    const double dx = S->mean2d[2 * g] - px;
    const double dy = S->mean2d[2 * g + 1] - py;
    const double A = S->conic[3 * g], B = S->conic[3 * g + 1], Cc = S->conic[3 * g + 2];
    const double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    if (power > 0.0) continue;
    const double ea = S->alpha_hat[g] * exp(power);
    if (fabs(ea - OR_ALPHA_MIN) <= OR_NEAR_REL * OR_ALPHA_MIN) *near_thr = 1;
    if (fabs(ea - OR_ALPHA_MAX) <= OR_NEAR_REL * OR_ALPHA_MAX) *near_thr = 1;
    const double alpha = ea < OR_ALPHA_MAX ? ea : OR_ALPHA_MAX;
    if (alpha < OR_ALPHA_MIN) continue;
    const double Tn = T * (1.0 - alpha);
    const double a_cond = alpha / (1.0 - alpha);
    const double rel = OR_ERR_ALPHA * (cond + a_cond) + 1e-6 * (double)(last + 1);
    if (fabs(Tn - OR_T_STOP) <= rel * OR_T_STOP) *near_thr = 1;
    if (Tn < OR_T_STOP) break;
    for (int ch = 0; ch < 3; ++ch) C[ch] += S->rgb[3 * g + ch] * alpha * T;
    T = Tn;
    cond += a_cond;
    last = j + 1;
    if (usage) {
#pragma omp atomic
      usage[g] += 1;
    }
  }
  for (int ch = 0; ch < 3; ++ch) out_c[ch] = C[ch] + T * bg[ch];
  *out_T = T;
  *out_n = last;
}

/*
 * Tiled forward render.  Per view v (index base v*n into the projected
 * arrays), every pixel of tile s composites the list vals[ranges[2s] ..
 * ranges[2s+1]).  image (V,3,H,W), final_T (V,H,W), n_contrib (V,H,W),
 * near_thr (V,H,W).  All views share W, H here (wh of view 0).
 */
void or_render_fwd(int V, int n, const double* mean2d, const double* conic, const double* rgb,
                   const double* alpha_hat, const int64_t* seg_base, const int* camwh,
                   const uint32_t* vals, const uint32_t* ranges, const double* bg,
                   double* image, double* final_T, int* n_contrib, uint8_t* near_thr,
                   int64_t* usage, int64_t* near_involved) {
  for (int v = 0; v < V; ++v) {
    const int W = camwh[2 * v], H = camwh[2 * v + 1];
    const int TX = tiles_x(W), TY = tiles_x(H);
    or_splats S = {mean2d + (size_t)2 * v * n, conic + (size_t)3 * v * n,
                   rgb + (size_t)3 * v * n, alpha_hat + (size_t)v * n};
    const size_t pix = (size_t)W * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (int tile = 0; tile < TX * TY; ++tile) {
      const int64_t s = seg_base[v] + tile;
      const uint32_t b = ranges[2 * s], e = ranges[2 * s + 1];
      const int tx = tile % TX, ty = tile / TX;
      for (int yy = 0; yy < OR_TILE; ++yy)
        for (int xx = 0; xx < OR_TILE; ++xx) {
          const int x = tx * OR_TILE + xx, y = ty * OR_TILE + yy;
          if (x >= W || y >= H) continue;
          double c[3], T;
          int nc, nt = 0;
          composite_pixel(&S, vals + b, (int)(e - b), (double)x, (double)y, bg + 3 * v, c, &T,
                          &nc, &nt, usage);
          /* usage: per Gaussian, the number of (view, pixel) pairs that
           * composite it; near_involved: pixels near a threshold whose list
           * holds it (where an FP32 walk may composite it or not) */
          if (nt && near_involved)
            for (uint32_t k = b; k < e; ++k) {
#pragma omp atomic
              near_involved[vals[k]] += 1;
            }
          const size_t p = (size_t)y * W + x;
          for (int ch = 0; ch < 3; ++ch) image[(size_t)v * 3 * pix + ch * pix + p] = c[ch];
          final_T[(size_t)v * pix + p] = T;
          n_contrib[(size_t)v * pix + p] = nc;
          near_thr[(size_t)v * pix + p] = (uint8_t)nt;
        }
    }
  }
}

/* Brute-force render of one view straight from the plain definition: for
 * every pixel, the contributing set is every visible Gaussian whose tile set
 * (rectangle, or per-row spans) contains the pixel's tile, ordered by (FP32
 * depth, id). */
typedef struct {
  uint32_t d;
  uint32_t id;
} or_did;

static int did_cmp(const void* pa, const void* pb) {
  const or_did* a = (const or_did*)pa;
  const or_did* b = (const or_did*)pb;
  if (a->d != b->d) return a->d < b->d ? -1 : 1;
  return a->id < b->id ? -1 : (a->id > b->id);
}

void or_render_brute(int n, const double* mean2d, const double* conic, const double* rgb,
                     const double* alpha_hat, const uint32_t* depth_bits, const int* rect,
                     const int* tiles, const int* spans, const uint8_t* flags, int W, int H,
                     const double* bg, double* image, double* final_T, int* n_contrib) {
  or_splats S = {mean2d, conic, rgb, alpha_hat};
  or_did* lst = (or_did*)malloc(sizeof(or_did) * (size_t)(n > 0 ? n : 1));
  uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  const size_t pix = (size_t)W * H;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int tx = x / OR_TILE, ty = y / OR_TILE;
      int len = 0;
      for (int i = 0; i < n; ++i) {
        if (tiles[i] <= 0) continue;
        const int* r = rect + 4 * i;
        if (ty < r[1] || ty >= r[3]) continue;
        int c0, c1;
        row_columns(r, spans ? spans + (size_t)2 * OR_SPAN_ROWS * i : NULL,
                    spans && flags && (flags[i] & OR_F_SPANS), ty, &c0, &c1);
        if (tx >= c0 && tx < c1) {
          lst[len].d = depth_bits[i];
          lst[len].id = (uint32_t)i;
          ++len;
        }
      }
      qsort(lst, (size_t)len, sizeof(or_did), did_cmp);
      for (int k = 0; k < len; ++k) ids[k] = lst[k].id;
      double c[3], T;
      int nc, nt = 0;
      composite_pixel(&S, ids, len, (double)x, (double)y, bg, c, &T, &nc, &nt, NULL);
      const size_t p = (size_t)y * W + x;
      for (int ch = 0; ch < 3; ++ch) image[ch * pix + p] = c[ch];
      final_T[p] = T;
      n_contrib[p] = nc;
    }
  free(lst);
  free(ids);
}

/* ------------------------------------------------------------------------ */
/* Step 9: L1 loss, mean over V*3*H*W values, and its gradient              */
/* sign(I - I*)/count with sign(0) = 0 (Eq. (1), L1 term).                   */
/* ------------------------------------------------------------------------ */
double or_l1(int64_t count, const double* img, const double* target, double* grad) {
  double acc = 0.0;
  for (int64_t k = 0; k < count; ++k) {
    const double d = img[k] - target[k];
    acc += fabs(d);
    if (grad) grad[k] = d > 0.0 ? 1.0 / (double)count : (d < 0.0 ? -1.0 / (double)count : 0.0);
  }
  return acc / (double)count;
}

/* ------------------------------------------------------------------------ */
/* Backward of compositing, per pixel, exact derivative of step 8.           */
/* Gradients go to per-(view, Gaussian) accumulators g2d (.,9):              */
/*   0,1: mean2d   2,3,4: conic A, B, C   5: alpha_hat   6,7,8: rgb          */
/* ------------------------------------------------------------------------ */
static void composite_pixel_bwd(const or_splats* S, const uint32_t* list, int len, double px,
                                double py, const double bg[3], const double gI[3], double* g2d) {
  /* forward again, remembering what was composited */
  int* idx = (int*)malloc(sizeof(int) * (size_t)(len > 0 ? len : 1));
  double* al = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
  double* Tk = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
  double* ex = (double*)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
  int* capped = (int*)malloc(sizeof(int) * (size_t)(len > 0 ? len : 1));
  int cnt = 0;
  double T = 1.0;
  for (int j = 0; j < len; ++j) {
    const uint32_t g = list[j];
    const double dx = S->mean2d[2 * g] - px;
    const double dy = S->mean2d[2 * g + 1] - py;
    const double A = S->conic[3 * g], B = S->conic[3 * g + 1], Cc = S->conic[3 * g + 2];
    const double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    if (power > 0.0) continue;
    const double e = exp(power);
    const double ea = S->alpha_hat[g] * e;
    const double alpha = ea < OR_ALPHA_MAX ? ea : OR_ALPHA_MAX;
    if (alpha < OR_ALPHA_MIN) continue;
    const double Tn = T * (1.0 - alpha);
    if (Tn < OR_T_STOP) break;
    idx[cnt] = j;
    al[cnt] = alpha;
    Tk[cnt] = T;
    ex[cnt] = e;
    capped[cnt] = !(ea < OR_ALPHA_MAX);
    ++cnt;
    T = Tn;
  }
  /* back to front: B_n = bg, B_{k-1} = alpha_k c_k + (1 - alpha_k) B_k */
  double Bk[3] = {bg[0], bg[1], bg[2]};
  for (int k = cnt - 1; k >= 0; --k) {
    const uint32_t g = list[idx[k]];
    const double* c = S->rgb + 3 * g;
    double galpha = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      galpha += gI[ch] * Tk[k] * (c[ch] - Bk[ch]);
      g2d[9 * (size_t)g + 6 + ch] += gI[ch] * al[k] * Tk[k];
    }
    if (!capped[k]) {
      const double dx = S->mean2d[2 * g] - px;
      const double dy = S->mean2d[2 * g + 1] - py;
      const double A = S->conic[3 * g], B = S->conic[3 * g + 1], Cc = S->conic[3 * g + 2];
      const double gpow = galpha * al[k];
      g2d[9 * (size_t)g + 5] += galpha * ex[k];
      g2d[9 * (size_t)g + 0] += -gpow * (A * dx + B * dy);
      g2d[9 * (size_t)g + 1] += -gpow * (B * dx + Cc * dy);
      g2d[9 * (size_t)g + 2] += -0.5 * gpow * dx * dx;
      g2d[9 * (size_t)g + 3] += -gpow * dx * dy;
      g2d[9 * (size_t)g + 4] += -0.5 * gpow * dy * dy;
    }
    for (int ch = 0; ch < 3; ++ch) Bk[ch] = al[k] * c[ch] + (1.0 - al[k]) * Bk[ch];
  }
  free(idx);
  free(al);
  free(Tk);
  free(ex);
  free(capped);
}

/* Tiled backward of compositing for V views; g2d (V*n, 9) is accumulated. */
void or_render_bwd(int V, int n, const double* mean2d, const double* conic, const double* rgb,
                   const double* alpha_hat, const int64_t* seg_base, const int* camwh,
                   const uint32_t* vals, const uint32_t* ranges, const double* bg,
                   const double* dL_dimage, double* g2d) {
  for (int v = 0; v < V; ++v) {
    const int W = camwh[2 * v], H = camwh[2 * v + 1];
    const int TX = tiles_x(W), TY = tiles_x(H);
    or_splats S = {mean2d + (size_t)2 * v * n, conic + (size_t)3 * v * n,
                   rgb + (size_t)3 * v * n, alpha_hat + (size_t)v * n};
    const size_t pix = (size_t)W * H;
    double* gv = g2d + (size_t)9 * v * n;
#pragma omp parallel
    {
      double* loc = (double*)calloc((size_t)9 * n, sizeof(double));
#pragma omp for schedule(dynamic, 4)
      for (int tile = 0; tile < TX * TY; ++tile) {
        const int64_t s = seg_base[v] + tile;
        const uint32_t b = ranges[2 * s], e = ranges[2 * s + 1];
        const int tx = tile % TX, ty = tile / TX;
        for (int yy = 0; yy < OR_TILE; ++yy)
          for (int xx = 0; xx < OR_TILE; ++xx) {
            const int x = tx * OR_TILE + xx, y = ty * OR_TILE + yy;
            if (x >= W || y >= H) continue;
            const size_t p = (size_t)y * W + x;
            double gI[3];
            for (int ch = 0; ch < 3; ++ch) gI[ch] = dL_dimage[(size_t)v * 3 * pix + ch * pix + p];
            /* a pixel with zero image gradient contributes nothing */
            if (gI[0] == 0.0 && gI[1] == 0.0 && gI[2] == 0.0) continue;
            composite_pixel_bwd(&S, vals + b, (int)(e - b), (double)x, (double)y, bg + 3 * v, gI,
                                loc);
          }
      }
#pragma omp critical
      {
        for (size_t k = 0; k < (size_t)9 * n; ++k) gv[k] += loc[k];
      }
      free(loc);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Chain rule from the per-(view, Gaussian) 2D gradients to the parameters.  */
/* Gradients are summed over views and ADDED to the outputs (planar, like     */
/* the parameters): g_mean (3,ld), g_lsc (3,ld), g_quat (4,ld), g_opac (ld),  */
/* g_sh (K,3,ld).                                                            */
/* ------------------------------------------------------------------------ */
void or_project_bwd(int n, int ld, int deg, const float* mean, const float* lsc,
                    const float* quat, const float* opac, const float* sh, int V,
                    const double* camR, const double* camt, const double* camf,
                    const int* camwh, const double* g2d, double* g_mean, double* g_lsc,
                    double* g_quat, double* g_opac, double* g_sh) {
  const int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    double m[3], s[3], q[4], o, shv[48];
    gather_params(i, ld, deg, mean, lsc, quat, opac, sh, m, s, q, &o, shv);
    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, galpha_hat = 0.0;
    double gsh[48];
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.0;
    for (int v = 0; v < V; ++v) {
      or_proj P;
      const double* R = camR + 9 * v;
      const double* f = camf + 4 * v;
      if (!project_one(m, s, q, o, shv, deg, R, camt + 3 * v, f, camwh + 2 * v, &P)) continue;
      const double* g = g2d + (size_t)9 * ((size_t)v * n + i);
      const double fx = f[0], fy = f[1];
      const double z = P.xc[2];
      galpha_hat += g[5];
      /* colour -> SH coefficients and view direction */
      double Y[16], dY[48];
      sh_basis(deg, P.dir[0], P.dir[1], P.dir[2], Y);
      sh_basis_grad(deg, P.dir[0], P.dir[1], P.dir[2], dY);
      double gdir[3] = {0, 0, 0};
      for (int ch = 0; ch < 3; ++ch) {
        if (!(P.raw[ch] > 0.0)) continue;
        const double gc = g[6 + ch];
        for (int k = 0; k < K; ++k) {
          gsh[k * 3 + ch] += Y[k] * gc;
          for (int ax = 0; ax < 3; ++ax) gdir[ax] += gc * shv[k * 3 + ch] * dY[k * 3 + ax];
        }
      }
      const double dd = (gdir[0] * P.dir[0] + gdir[1] * P.dir[1]) + gdir[2] * P.dir[2];
      for (int ax = 0; ax < 3; ++ax) gm[ax] += (gdir[ax] - dd * P.dir[ax]) / P.dist;
      /* mean2d -> camera space */
      double gx[3] = {0, 0, 0};
      gx[0] += g[0] * fx / z;
      gx[1] += g[1] * fy / z;
      gx[2] -= (g[0] * fx * P.xc[0] + g[1] * fy * P.xc[1]) / (z * z);
      /* conic -> 2D covariance: G_S = -Q G_Q Q */
      const double A = P.conic[0], B = P.conic[1], C = P.conic[2];
      const double Q[4] = {A, B, B, C};
      const double GQ[4] = {g[2], 0.5 * g[3], 0.5 * g[3], g[4]};
      double QG[4], GS[4];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) QG[2 * r + c] = Q[2 * r] * GQ[c] + Q[2 * r + 1] * GQ[2 + c];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) GS[2 * r + c] = -(QG[2 * r] * Q[c] + QG[2 * r + 1] * Q[2 + c]);
      /* cov2D = J V J^T: G_V = J^T G_S J, G_J = 2 G_S J V */
      double GV[9], GJ[6], GSJ[6];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) GSJ[3 * r + c] = GS[2 * r] * P.J[c] + GS[2 * r + 1] * P.J[3 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GV[3 * r + c] = P.J[r] * GSJ[c] + P.J[3 + r] * GSJ[3 + c];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += GSJ[3 * r + k] * P.V[3 * k + c];
          GJ[3 * r + c] = 2.0 * acc;
        }
      /* J entries: J00 = fx/z, J02 = -fx u/z, J11 = fy/z, J12 = -fy v/z */
      gx[2] += GJ[0] * (-fx / (z * z)) + GJ[4] * (-fy / (z * z));
      if (P.clamp_u) {
        gx[2] += GJ[2] * (fx * P.u / (z * z));
      } else {
        gx[0] += GJ[2] * (-fx / (z * z));
        gx[2] += GJ[2] * (2.0 * fx * P.xc[0] / (z * z * z));
      }
      if (P.clamp_v) {
        gx[2] += GJ[5] * (fy * P.v / (z * z));
      } else {
        gx[1] += GJ[5] * (-fy / (z * z));
        gx[2] += GJ[5] * (2.0 * fy * P.xc[1] / (z * z * z));
      }
      for (int ax = 0; ax < 3; ++ax) gm[ax] += (R[0 * 3 + ax] * gx[0] + R[1 * 3 + ax] * gx[1]) + R[2 * 3 + ax] * gx[2];
      /* V = W Sigma W^T: G_Sigma = W^T G_V W */
      double GSig[9], tmp[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += R[3 * k + r] * GV[3 * k + c];
          tmp[3 * r + c] = acc;
        }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += tmp[3 * r + k] * R[3 * k + c];
          GSig[3 * r + c] = acc;
        }
      /* Sigma = M M^T: G_M = (G_Sigma + G_Sigma^T) M */
      double GM[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += (GSig[3 * r + k] + GSig[3 * k + r]) * P.M[3 * k + c];
          GM[3 * r + c] = acc;
        }
      /* M = R_q diag(sigma) */
      double GR[9];
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r) {
          acc += P.Rq[3 * r + c] * GM[3 * r + c];
          GR[3 * r + c] = GM[3 * r + c] * P.sigma[c];
        }
        gs[c] += acc * P.sigma[c];
      }
      /* R_q(qhat) -> qhat -> q */
      const double w = P.qhat[0], x = P.qhat[1], y = P.qhat[2], zq = P.qhat[3];
      double gh[4];
      gh[0] = 2.0 * (-zq * GR[1] + y * GR[2] + zq * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
      gh[1] = 2.0 * (y * GR[1] + zq * GR[2] + y * GR[3] - 2.0 * x * GR[4] - w * GR[5] + zq * GR[6] +
                     w * GR[7] - 2.0 * x * GR[8]);
      gh[2] = 2.0 * (-2.0 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + zq * GR[5] - w * GR[6] +
                     zq * GR[7] - 2.0 * y * GR[8]);
      gh[3] = 2.0 * (-2.0 * zq * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.0 * zq * GR[4] +
                     y * GR[5] + x * GR[6] + y * GR[7]);
      const double dq = gh[0] * P.qhat[0] + gh[1] * P.qhat[1] + gh[2] * P.qhat[2] + gh[3] * P.qhat[3];
      for (int k = 0; k < 4; ++k) gq[k] += (gh[k] - dq * P.qhat[k]) / P.qnorm;
    }
    const double ah = sigmoid(o);
    for (int k = 0; k < 3; ++k) {
      g_mean[(size_t)k * ld + i] += gm[k];
      g_lsc[(size_t)k * ld + i] += gs[k];
    }
    for (int k = 0; k < 4; ++k) g_quat[(size_t)k * ld + i] += gq[k];
    g_opac[i] += galpha_hat * ah * (1.0 - ah);
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) g_sh[((size_t)k * 3 + ch) * ld + i] += gsh[k * 3 + ch];
  }
}

/* Backward of step 1 to the delta images (8, gh, gw).  Padding texels and
 * masked texels receive 0.  quat is the ANCHOR quaternion (FP32 storage). */
void or_apply_bwd(int n, int ld, const float* quat, const uint8_t* mask, int gw, int gh,
                  const double* g_mean, const double* g_quat, const double* g_opac,
                  double* g_delta) {
  const size_t plane = (size_t)gw * (size_t)gh;
  for (size_t k = 0; k < 8 * plane; ++k) g_delta[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!mask[i]) continue;
    for (int k = 0; k < 3; ++k) g_delta[(size_t)k * plane + i] = g_mean[(size_t)k * ld + i];
    /* (dq (x) q) = Rr(q) dq, so g_dq = Rr(q)^T g_q' */
    const double bw = quat[i], bx = quat[(size_t)ld + i], by = quat[(size_t)2 * ld + i],
                 bz = quat[(size_t)3 * ld + i];
    const double Rr[16] = {bw, -bx, -by, -bz, bx, bw, bz, -by, by, -bz, bw, bx, bz, by, -bx, bw};
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int r = 0; r < 4; ++r) acc += Rr[4 * r + c] * g_quat[(size_t)r * ld + i];
      g_delta[(size_t)(3 + c) * plane + i] = acc;
    }
    g_delta[(size_t)7 * plane + i] = g_opac[i];
  }
}

/* Adam (Kingma & Ba 2015, Algorithm 1) with bias correction; step t >= 1.
 * theta, m, v updated in place (FP64 copies of the FP32 state). */
void or_adam(int64_t count, double* theta, const double* grad, double* m, double* v, int t,
             double lr, double beta1, double beta2, double eps) {
  const double bc1 = 1.0 - pow(beta1, (double)t);
  const double bc2 = 1.0 - pow(beta2, (double)t);
  for (int64_t k = 0; k < count; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * grad[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * grad[k] * grad[k];
    const double mh = m[k] / bc1;
    const double vh = v[k] / bc2;
    theta[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Whole forward to an L1 loss, used by the finite-difference driver.         */
/* Writes a 64-bit structure signature (hash of culling, rectangles, clamp    */
/* flags and every pixel's composited-entry list) so that a caller can drop   */
/* FD components whose stencil crosses a discontinuity.                       */
/* ------------------------------------------------------------------------ */
static uint64_t mix64(uint64_t h, uint64_t x) {
  h ^= x + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  return h;
}

double or_forward_loss(int n, int ld, int deg, const float* mean, const float* lsc,
                       const float* quat, const float* opac, const float* sh,
                       const double* mean_d, const double* lsc_d, const double* quat_d,
                       const double* opac_d, const double* sh_d, int V, const double* camR,
                       const double* camt, const double* camf, const int* camwh,
                       const double* bg, const double* target, uint64_t* signature) {
  /* parameters: if the *_d pointer is given the FP64 value is used, else the
   * FP32 one (FD steps must not be rounded to FP32). */
  const int K = (deg + 1) * (deg + 1);
  double loss = 0.0;
  int64_t count = 0;
  uint64_t h = 1469598103934665603ULL;
  for (int v = 0; v < V; ++v) {
    const int W = camwh[2 * v], H = camwh[2 * v + 1];
    const int TX = tiles_x(W), TY = tiles_x(H);
    double* m2 = (double*)calloc((size_t)2 * n, sizeof(double));
    double* co = (double*)calloc((size_t)3 * n, sizeof(double));
    double* rg = (double*)calloc((size_t)3 * n, sizeof(double));
    double* ah = (double*)calloc((size_t)n, sizeof(double));
    uint32_t* db = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    int* rc = (int*)calloc((size_t)4 * n, sizeof(int));
    int* tl = (int*)calloc((size_t)n, sizeof(int));
    for (int i = 0; i < n; ++i) {
      double m[3], s[3], q[4], o, shv[48];
      for (int k = 0; k < 3; ++k) {
        m[k] = mean_d ? mean_d[(size_t)k * ld + i] : mean[(size_t)k * ld + i];
        s[k] = lsc_d ? lsc_d[(size_t)k * ld + i] : lsc[(size_t)k * ld + i];
      }
      for (int k = 0; k < 4; ++k) q[k] = quat_d ? quat_d[(size_t)k * ld + i] : quat[(size_t)k * ld + i];
      o = opac_d ? opac_d[i] : opac[i];
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) {
          const size_t a = ((size_t)k * 3 + ch) * ld + i;
          shv[k * 3 + ch] = sh_d ? sh_d[a] : sh[a];
        }
      or_proj P;
      int vis = project_one(m, s, q, o, shv, deg, camR + 9 * v, camt + 3 * v, camf + 4 * v,
                            camwh + 2 * v, &P);
      h = mix64(h, (uint64_t)vis);
      if (!vis) continue;
      m2[2 * i] = P.p[0];
      m2[2 * i + 1] = P.p[1];
      for (int k = 0; k < 3; ++k) {
        co[3 * i + k] = P.conic[k];
        rg[3 * i + k] = P.rgb[k];
      }
      ah[i] = P.alpha_hat;
      db[i] = f32_bits(round_to_f32(P.depth));
      for (int k = 0; k < 4; ++k) {
        rc[4 * i + k] = P.rect[k];
        h = mix64(h, (uint64_t)(uint32_t)P.rect[k]);
      }
      tl[i] = P.tiles;
      h = mix64(h, (uint64_t)((P.raw[0] > 0) | ((P.raw[1] > 0) << 1) | ((P.raw[2] > 0) << 2) |
                              (P.clamp_u << 3) | (P.clamp_v << 4)));
    }
    int64_t M = or_count_instances(1, n, tl);
    const int64_t nseg = (int64_t)TX * TY;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(M > 0 ? M : 1));
    uint32_t* vals = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(M > 0 ? M : 1));
    uint32_t* ranges = (uint32_t*)malloc(sizeof(uint32_t) * 2 * (size_t)nseg);
    const int64_t sb = 0;
    or_bin_sort(1, n, db, rc, tl, NULL, NULL, &sb, &TX, nseg, keys, vals, ranges);
    or_splats S = {m2, co, rg, ah};
    const size_t pix = (size_t)W * H;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const int64_t sg = (int64_t)(y / OR_TILE) * TX + x / OR_TILE;
        const uint32_t b = ranges[2 * sg], e = ranges[2 * sg + 1];
        /* list of composited entries for the signature */
        double T = 1.0, C[3] = {0, 0, 0};
        for (uint32_t j = b; j < e; ++j) {
          const uint32_t g = vals[j];
          const double dx = S.mean2d[2 * g] - x, dy = S.mean2d[2 * g + 1] - y;
          const double A = S.conic[3 * g], B = S.conic[3 * g + 1], Cc = S.conic[3 * g + 2];
          const double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
          if (power > 0.0) continue;
          const double ea = S.alpha_hat[g] * exp(power);
          const double alpha = ea < OR_ALPHA_MAX ? ea : OR_ALPHA_MAX;
          h = mix64(h, (uint64_t)(ea < OR_ALPHA_MAX));
          if (alpha < OR_ALPHA_MIN) continue;
          const double Tn = T * (1.0 - alpha);
          if (Tn < OR_T_STOP) {
            h = mix64(h, 0xdeadULL);
            break;
          }
          h = mix64(h, (uint64_t)g + 1);
          for (int ch = 0; ch < 3; ++ch) C[ch] += S.rgb[3 * g + ch] * alpha * T;
          T = Tn;
        }
        for (int ch = 0; ch < 3; ++ch) {
          const double val = C[ch] + T * bg[3 * v + ch];
          const double d = val - target[(size_t)v * 3 * pix + ch * pix + (size_t)y * W + x];
          loss += fabs(d);
          h = mix64(h, (uint64_t)(d > 0) + 2 * (uint64_t)(d < 0));
          ++count;
        }
      }
    free(keys);
    free(vals);
    free(ranges);
    free(m2);
    free(co);
    free(rg);
    free(ah);
    free(db);
    free(rc);
    free(tl);
  }
  if (signature) *signature = h;
  return count ? loss / (double)count : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Photometric loss of Eq. (1): L = (1 - lambda) L1 + lambda (1 - SSIM).      */
/* SSIM per channel with an 11x11 Gaussian window (sigma 1.5, weights         */
/* normalised to sum 1), zero padding outside the image, C1 = 0.01^2,        */
/* C2 = 0.03^2; SSIM = mean of the per-pixel index over (V, 3, H, W).         */
/* ------------------------------------------------------------------------ */
#define OR_SSIM_R 5

static void ssim_window(double w[2 * OR_SSIM_R + 1]) {
  double s = 0.0;
  for (int i = -OR_SSIM_R; i <= OR_SSIM_R; ++i) {
    w[i + OR_SSIM_R] = exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
    s += w[i + OR_SSIM_R];
  }
  for (int i = 0; i <= 2 * OR_SSIM_R; ++i) w[i] /= s;
}

void or_ssim_window(double* w) { ssim_window(w); }

/* Windowed sum of one plane at (x, y): sum over the 11x11 window of
 * w(i) w(j) f(y + j, x + i), samples outside the image taken as 0. */
static double window_sum(const double* f, int W, int H, int x, int y, const double* w) {
  double acc = 0.0;
  for (int j = -OR_SSIM_R; j <= OR_SSIM_R; ++j) {
    const int yy = y + j;
    if (yy < 0 || yy >= H) continue;
    for (int i = -OR_SSIM_R; i <= OR_SSIM_R; ++i) {
      const int xx = x + i;
      if (xx < 0 || xx >= W) continue;
      acc += w[i + OR_SSIM_R] * w[j + OR_SSIM_R] * f[(size_t)yy * W + xx];
    }
  }
  return acc;
}

/* Loss and gradient for `planes` image planes of H x W (V*3 planes).
 * ssim_map (planes*H*W, nullable) receives the per-pixel index.  Returns
 * (1 - lambda) mean|I - I*| + lambda (1 - mean SSIM); grad gets its exact
 * derivative w.r.t. the image (sign(0) = 0 for the L1 part). */
double or_l1_dssim(int planes, int H, int W, const double* img, const double* tgt,
                   double lambda, double* grad, double* ssim_map) {
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  const size_t pix = (size_t)W * H;
  const double count = (double)planes * (double)pix;
  double w[2 * OR_SSIM_R + 1];
  ssim_window(w);
  double ssim_sum = 0.0, l1_sum = 0.0;
  for (int pl = 0; pl < planes; ++pl) {
    const double* x = img + (size_t)pl * pix;
    const double* y = tgt + (size_t)pl * pix;
    double* xx = (double*)malloc(sizeof(double) * pix);
    double* yy = (double*)malloc(sizeof(double) * pix);
    double* xy = (double*)malloc(sizeof(double) * pix);
    double* A1 = (double*)malloc(sizeof(double) * pix);
    double* A2 = (double*)malloc(sizeof(double) * pix);
    double* A3 = (double*)malloc(sizeof(double) * pix);
    for (size_t p = 0; p < pix; ++p) {
      xx[p] = x[p] * x[p];
      yy[p] = y[p] * y[p];
      xy[p] = x[p] * y[p];
    }
    double plane_sum = 0.0;
#pragma omp parallel for reduction(+ : plane_sum) schedule(static)
    for (int r = 0; r < H; ++r)
      for (int c = 0; c < W; ++c) {
        const double mx = window_sum(x, W, H, c, r, w), my = window_sum(y, W, H, c, r, w);
        const double sxx = window_sum(xx, W, H, c, r, w) - mx * mx;
        const double syy = window_sum(yy, W, H, c, r, w) - my * my;
        const double sxy = window_sum(xy, W, H, c, r, w) - mx * my;
        const double N1 = 2.0 * mx * my + C1, N2 = 2.0 * sxy + C2;
        const double D1 = mx * mx + my * my + C1, D2 = sxx + syy + C2;
        const double S = (N1 * N2) / (D1 * D2);
        const size_t p = (size_t)r * W + c;
        if (ssim_map) ssim_map[(size_t)pl * pix + p] = S;
        plane_sum += S;
        /* partials of S w.r.t. the windowed statistics */
        const double dS_dmx = (2.0 * my * N2) / (D1 * D2) - S * (2.0 * mx) / D1;
        const double dS_dsxx = -S / D2;
        const double dS_dsxy = (2.0 * N1) / (D1 * D2);
        /* sxx = E[x^2] - mx^2 and sxy = E[xy] - mx my, so through mx: */
        A1[p] = dS_dmx - 2.0 * mx * dS_dsxx - my * dS_dsxy;
        A2[p] = dS_dsxx;
        A3[p] = dS_dsxy;
      }
    ssim_sum += plane_sum;
    if (grad) {
      /* adjoint of the windowed sums (the window is symmetric) */
#pragma omp parallel for schedule(static)
      for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
          const size_t p = (size_t)r * W + c;
          const double g_ssim = window_sum(A1, W, H, c, r, w) +
                                2.0 * x[p] * window_sum(A2, W, H, c, r, w) +
                                y[p] * window_sum(A3, W, H, c, r, w);
          const double d = x[p] - y[p];
          const double g_l1 = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
          grad[(size_t)pl * pix + p] = ((1.0 - lambda) * g_l1 - lambda * g_ssim) / count;
        }
    }
    for (size_t p = 0; p < pix; ++p) l1_sum += fabs(x[p] - y[p]);
    free(xx);
    free(yy);
    free(xy);
    free(A1);
    free(A2);
    free(A3);
  }
  return (1.0 - lambda) * l1_sum / count + lambda * (1.0 - ssim_sum / count);
}
