// EWA projection of anisotropic Gaussians with spherical-harmonic colour,
// and its backward pass (the splatting renderer AirGS cites in Sec. II).
//
// A thread takes one Gaussian and a group of consecutive views; a workgroup
// takes 256 consecutive Gaussians and one view group.  All view groups of a
// chunk of Gaussians land on one XCD (workgroups are dealt to the 8 XCDs
// round-robin by index), so the SoA parameters (56 B at SH degree 0, 236 B
// at degree 3) come from HBM once and from that XCD's L2 for the other
// groups, while the view groups multiply the waves in flight; the
// per-(view, Gaussian) records are written coalesced.  The quantities that
// decide integers downstream -- depth key, radius, tile rectangle -- are
// evaluated in FP64 with contraction off and a fixed operation order, so
// that tile lists are reproducible exactly.  Colour is FP32.
#include <algorithm>

#include "gs_internal.h"

namespace gs {
namespace {

// Real orthonormal SH on the unit vector (x, y, z), index l*l + l + m.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;   // xy, yz, xz
constexpr float kY2b = 0.31539156525252005f;  // 3z^2 - 1
constexpr float kY2c = 0.54627421529603959f;  // x^2 - y^2
constexpr float kY3a = 0.59004358992664352f;  // y(3x^2-y^2), x(x^2-3y^2)
constexpr float kY3b = 2.8906114426405538f;   // xyz
constexpr float kY3c = 0.45704579946446572f;  // y(5z^2-1), x(5z^2-1)
constexpr float kY3d = 0.37317633259011540f;  // z(5z^2-3)
constexpr float kY3e = 1.4453057213202769f;   // z(x^2-y^2)
constexpr double kLn255d = 5.541263545158426;  // ln 255

template <int DEG>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y) {
  Y[0] = kY0;
  if constexpr (DEG >= 1) {
    Y[1] = kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = kY1 * x;
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * (x * y);
    Y[5] = kY2a * (y * z);
    Y[6] = kY2b * (3.f * zz - 1.f);
    Y[7] = kY2a * (x * z);
    Y[8] = kY2c * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = kY3a * y * (3.f * xx - yy);
      Y[10] = kY3b * x * y * z;
      Y[11] = kY3c * y * (5.f * zz - 1.f);
      Y[12] = kY3d * z * (5.f * zz - 3.f);
      Y[13] = kY3c * x * (5.f * zz - 1.f);
      Y[14] = kY3e * z * (xx - yy);
      Y[15] = kY3a * x * (xx - 3.f * yy);
    }
  }
}

// g = sum_k w_k * grad(Y_k) for polynomial forms above.
template <int DEG>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float* w,
                                            float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.f;
  if constexpr (DEG >= 1) {
    gy += kY1 * w[1];
    gz += kY1 * w[2];
    gx += kY1 * w[3];
  }
  if constexpr (DEG >= 2) {
    gx += kY2a * (y * w[4] + z * w[7]) + kY2c * 2.f * x * w[8];
    gy += kY2a * (x * w[4] + z * w[5]) - kY2c * 2.f * y * w[8];
    gz += kY2a * (y * w[5] + x * w[7]) + kY2b * 6.f * z * w[6];
    if constexpr (DEG >= 3) {
      const float xx = x * x, yy = y * y, zz = z * z;
      gx += kY3a * 6.f * x * y * w[9] + kY3b * y * z * w[10] +
            kY3c * (5.f * zz - 1.f) * w[13] + kY3e * 2.f * x * z * w[14] +
            kY3a * 3.f * (xx - yy) * w[15];
      gy += kY3a * 3.f * (xx - yy) * w[9] + kY3b * x * z * w[10] +
            kY3c * (5.f * zz - 1.f) * w[11] - kY3e * 2.f * y * z * w[14] -
            kY3a * 6.f * x * y * w[15];
      gz += kY3b * x * y * w[10] + kY3c * 10.f * y * z * w[11] +
            kY3d * (15.f * zz - 3.f) * w[12] + kY3c * 10.f * x * z * w[13] +
            kY3e * (xx - yy) * w[14];
    }
  }
}

__device__ __forceinline__ double clampd(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(
    int n, int ld, const float* __restrict__ mean, const float* __restrict__ lsc,
    const float* __restrict__ quat, const float* __restrict__ opac, const float* __restrict__ sh,
    const gs_camera* __restrict__ cams, int n_views, int groups, int per_group,
    float4* __restrict__ splat, int4* __restrict__ rect, int32_t* __restrict__ tiles,
    uint32_t* __restrict__ depth_bits, uint8_t* __restrict__ flags, bool tight, bool spans) {
#pragma clang fp contract(off)
  constexpr int K = (DEG + 1) * (DEG + 1);
  // workgroup b: XCD b % 8; chunk = 8 (b / (8 groups)) + b % 8, view group
  // (b / 8) % groups
  const int b = blockIdx.x;
  const int chunk = 8 * (b / (8 * groups)) + (b & 7);
  const int vg = (b >> 3) % groups;
  const int i = chunk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v_begin = vg * per_group;
  const int v_end = min(n_views, v_begin + per_group);
  const size_t L = (size_t)ld;
  const double m0 = mean[i], m1 = mean[L + i], m2 = mean[2 * L + i];
  double qw = quat[i], qx = quat[L + i], qy = quat[2 * L + i], qz = quat[3 * L + i];
  const double qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const bool degenerate = !(qn >= 1e-8);
  qw = qw / qn;
  qx = qx / qn;
  qy = qy / qn;
  qz = qz / qn;
  double Rq[9];
  Rq[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
  Rq[1] = 2.0 * (qx * qy - qw * qz);
  Rq[2] = 2.0 * (qx * qz + qw * qy);
  Rq[3] = 2.0 * (qx * qy + qw * qz);
  Rq[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
  Rq[5] = 2.0 * (qy * qz - qw * qx);
  Rq[6] = 2.0 * (qx * qz - qw * qy);
  Rq[7] = 2.0 * (qy * qz + qw * qx);
  Rq[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
  const double s0 = exp((double)lsc[i]), s1 = exp((double)lsc[L + i]),
               s2 = exp((double)lsc[2 * L + i]);
  double M[9];
  for (int r = 0; r < 3; ++r) {
    M[3 * r + 0] = Rq[3 * r + 0] * s0;
    M[3 * r + 1] = Rq[3 * r + 1] * s1;
    M[3 * r + 2] = Rq[3 * r + 2] * s2;
  }
  double S[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[3 * r + c] = (M[3 * r + 0] * M[3 * c + 0] + M[3 * r + 1] * M[3 * c + 1]) +
                     M[3 * r + 2] * M[3 * c + 2];
  const float alpha_hat = 1.f / (1.f + __expf(-opac[i]));
  // threshold of the opacity-aware tile sets: alpha >= 1/255 needs
  // q(d) <= 2 ln(255 opacity) (in FP64 from the logit, one per Gaussian)
  double thr = 0.0;
  if (tight) {
    const double ahd = 1.0 / (1.0 + exp(-(double)opac[i]));
    const double qm = 2.0 * (kLn255d + log(ahd));
    thr = qm + 2e-4 * fabs(qm) + 1e-3;
  }
  float shv[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) shv[k] = sh[(size_t)k * L + i];

  for (int v = v_begin; v < v_end; ++v) {
    const gs_camera& cam = cams[v];
    const double* R = cam.R;
    const size_t j = (size_t)v * L + i;
    const double xc0 = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + cam.t[0];
    const double xc1 = ((R[3] * m0 + R[4] * m1) + R[5] * m2) + cam.t[1];
    const double z = ((R[6] * m0 + R[7] * m1) + R[8] * m2) + cam.t[2];
    depth_bits[j] = __float_as_uint((float)z);
    bool vis = (z > kNear) && !degenerate;
    uint8_t fl = 0;
    double px = 0, py = 0, A = 0, B = 0, C = 0, detq = 0;
    int4 rc = make_int4(0, 0, 0, 0);
    int nt = 0;
    uint32_t span_word = 0;  // per-row tile spans, when span_mode
    bool span_mode = false;
    if (vis) {
      // V = W S W^T, W = camera rotation
      double T1[9], Vm[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          T1[3 * r + c] = (R[3 * r + 0] * S[0 * 3 + c] + R[3 * r + 1] * S[1 * 3 + c]) +
                          R[3 * r + 2] * S[2 * 3 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Vm[3 * r + c] = (T1[3 * r + 0] * R[3 * c + 0] + T1[3 * r + 1] * R[3 * c + 1]) +
                          T1[3 * r + 2] * R[3 * c + 2];
      const double fx = cam.fx, fy = cam.fy;
      const double limx = kGuard * ((0.5 * (double)cam.width) / fx);
      const double limy = kGuard * ((0.5 * (double)cam.height) / fy);
      double u = xc0 / z, w = xc1 / z;
      if (u < -limx || u > limx) fl |= kClampU;
      if (w < -limy || w > limy) fl |= kClampV;
      u = clampd(u, -limx, limx);
      w = clampd(w, -limy, limy);
      const double J[6] = {fx / z, 0.0, -(fx * u) / z, 0.0, fy / z, -(fy * w) / z};
      double T2[6];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
          T2[3 * r + c] = (J[3 * r + 0] * Vm[0 * 3 + c] + J[3 * r + 1] * Vm[1 * 3 + c]) +
                          J[3 * r + 2] * Vm[2 * 3 + c];
      const double a = (T2[0] * J[0] + T2[1] * J[1]) + T2[2] * J[2];
      const double b = (T2[0] * J[3] + T2[1] * J[4]) + T2[2] * J[5];
      const double c = (T2[3] * J[3] + T2[4] * J[4]) + T2[5] * J[5];
      const double ap = a + kDilate, cp = c + kDilate;
      const double det = ap * cp - b * b;
      vis = det > 0.0;
      if (vis) {
        const double inv = 1.0 / det;
        detq = inv;  // A C - B^2 of the conic
        A = cp * inv;
        B = -b * inv;
        C = ap * inv;
        px = (fx * xc0) / z + cam.cx;
        py = (fy * xc1) / z + cam.cy;
        const double mid = 0.5 * (ap + cp);
        double disc = mid * mid - det;
        if (disc < 0.1) disc = 0.1;
        const double lam = mid + sqrt(disc);
        const double rad = ceil(3.0 * sqrt(lam));
        const double TX = (double)tiles_across(cam.width), TY = (double)tiles_across(cam.height);
        double t0 = clampd(floor((px - rad) / (double)kTile), 0.0, TX);
        double t2 = clampd(floor((px + rad) / (double)kTile) + 1.0, 0.0, TX);
        double t1 = clampd(floor((py - rad) / (double)kTile), 0.0, TY);
        double t3 = clampd(floor((py + rad) / (double)kTile) + 1.0, 0.0, TY);
        if (tight) {
          // A tile none of whose pixels reaches alpha >= 1/255 composites
          // nothing of this Gaussian.  alpha >= 1/255 needs q(d) = A dx^2 +
          // 2B dx dy + C dy^2 <= 2 ln(255 opacity); with a margin that covers
          // FP32 evaluation of alpha, the kept tiles are those meeting the
          // ellipse q <= thr (bounding box x +- sqrt(thr C / Dq), y +-
          // sqrt(thr A / Dq), Dq = AC - B^2).  Everything here is IEEE FP64
          // in a fixed operation order, opacity included, so that the tile
          // sets are a deterministic function of the FP64 binning geometry.
          const double Dq = A * C - B * B;
          double ex = 0.0, ey = 0.0;  // half-extents of that ellipse
          if (thr > 0.0) {
            ex = sqrt(thr * C / Dq);
            ey = sqrt(thr * A / Dq);
            t0 = fmax(t0, clampd(floor((px - ex) / (double)kTile), 0.0, TX));
            t2 = fmin(t2, clampd(floor((px + ex) / (double)kTile) + 1.0, 0.0, TX));
            t1 = fmax(t1, clampd(floor((py - ey) / (double)kTile), 0.0, TY));
            t3 = fmin(t3, clampd(floor((py + ey) / (double)kTile) + 1.0, 0.0, TY));
          } else {
            t2 = t0;  // no pixel can reach alpha 1/255
          }
          rc = t2 > t0 && t3 > t1 ? make_int4((int)t0, (int)t1, (int)t2, (int)t3)
                                  : make_int4(0, 0, 0, 0);
          nt = (rc.z - rc.x) * (rc.w - rc.y);
          if (spans && nt > 0 && rc.w - rc.y <= kSpanRows && rc.z - rc.x <= kSpanWidth) {
            // Per tile row, the columns whose pixel centres come within
            // kSpanEps of the ellipse's x-extent over the row's band (pixel
            // centres +- 0.5 px in y, so neighbouring rows share an edge).
            // The chord at offset y spans x in ((-By - h)/A, (-By + h)/A),
            // h = sqrt(A thr - Dq y^2); its right end is concave in y with
            // maximum ex at y = -B ex / C and the left end mirrors it, so
            // over a band the extreme is that point or the chord at a band
            // end (clamped into [-ey, ey]).
            const double ys = -B * ex / C;
            auto chord = [&](double y, double& xl, double& xr) {
              const double yy = clampd(y, -ey, ey);
              double hh = A * thr - Dq * yy * yy;
              if (hh < 0.0) hh = 0.0;
              const double h = sqrt(hh);
              xr = (-B * yy + h) / A;
              xl = (-B * yy - h) / A;
              return yy;
            };
            uint32_t packed = 0;
            int cnt = 0;
            // a row's upper band edge is the next row's lower one (the same
            // FP64 value), so its chord is reused
            bool have = false;
            double pl = 0.0, pr = 0.0, pc = 0.0;
            for (int r = 0; r < rc.w - rc.y; ++r) {
              const double tyd = (double)(rc.y + r);
              const double lo = ((double)kTile * tyd - 0.5) - py;
              const double hi = ((double)kTile * tyd + 15.5) - py;
              if (lo > ey + kSpanEps || hi < -ey - kSpanEps) {
                have = false;
                continue;
              }
              double l0, r0, l1, r1, c0;
              if (have) {
                l0 = pl;
                r0 = pr;
                c0 = pc;
              } else {
                c0 = chord(lo, l0, r0);
              }
              const double c1 = chord(hi, l1, r1);
              pl = l1;
              pr = r1;
              pc = c1;
              have = true;
              const double xmax = (ys >= c0 && ys <= c1) ? ex : fmax(r0, r1);
              const double xmin = (-ys >= c0 && -ys <= c1) ? -ex : fmin(l0, l1);
              const double xs = fmax(
                  t0, ceil((((px + xmin) - kSpanEps) - (double)(kTile - 1)) / (double)kTile));
              const double xe = fmin(t2, floor(((px + xmax) + kSpanEps) / (double)kTile) + 1.0);
              if (xe > xs) {
                const uint32_t a0 = (uint32_t)(xs - t0), a1 = (uint32_t)(xe - t0);
                packed |= (a0 | a1 << 4) << (8 * r);
                cnt += (int)(a1 - a0);
              }
            }
            span_word = packed;
            span_mode = true;
            nt = cnt;
            if (nt == 0) rc = make_int4(0, 0, 0, 0);
          }
        } else {
          rc = t2 > t0 && t3 > t1 ? make_int4((int)t0, (int)t1, (int)t2, (int)t3)
                                  : make_int4(0, 0, 0, 0);
          nt = (rc.z - rc.x) * (rc.w - rc.y);
        }
        vis = nt > 0;
      }
    }
    float4 o0 = make_float4(0.f, 0.f, 0.f, 0.f), o1 = o0, o2 = o0, o3 = o0;
    if (vis) {
      // colour along the world-space direction camera centre -> mean
      const float ccx = (float)-((R[0] * cam.t[0] + R[3] * cam.t[1]) + R[6] * cam.t[2]);
      const float ccy = (float)-((R[1] * cam.t[0] + R[4] * cam.t[1]) + R[7] * cam.t[2]);
      const float ccz = (float)-((R[2] * cam.t[0] + R[5] * cam.t[1]) + R[8] * cam.t[2]);
      float dx = (float)m0 - ccx, dy = (float)m1 - ccy, dz = (float)m2 - ccz;
      const float inv_len = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
      dx *= inv_len;
      dy *= inv_len;
      dz *= inv_len;
      float Y[K];
      sh_eval<DEG>(dx, dy, dz, Y);
      float rgb[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += Y[k] * shv[k * 3 + ch];
        if (!(acc > 0.f)) fl |= (uint8_t)(1u << ch);
        rgb[ch] = acc > 0.f ? acc : 0.f;
      }
      fl |= kVisible;
      o0 = make_float4((float)px, (float)py, (float)A, (float)B);
      o1 = make_float4((float)C, alpha_hat, rgb[0], rgb[1]);
      o2 = make_float4(rgb[2], (float)z, (float)detq, 0.f);
      // tile rectangle for the backward's instance rows (the emission base,
      // component z, is filled in by the binning)
      o3 = make_float4(__uint_as_float((uint32_t)rc.x | ((uint32_t)rc.y << 16)),
                       __uint_as_float((uint32_t)(rc.z - rc.x) | (span_mode ? kSpanFlag : 0u)),
                       0.f, __uint_as_float(span_word));
    } else {
      fl = 0;
      rc = make_int4(0, 0, 0, 0);
      nt = 0;
    }
    splat[kSplatF4 * j + 0] = o0;
    splat[kSplatF4 * j + 1] = o1;
    splat[kSplatF4 * j + 2] = o2;
    splat[kSplatF4 * j + 3] = o3;
    rect[j] = rc;
    tiles[j] = nt;
    flags[j] = fl;
  }
}

// Backward of the projection: screen-space gradients (per view) to the
// Gaussian parameters, summed over views.  FP32.  The covariance gradient is
// accumulated over views and pushed through Sigma = M M^T once.
template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(
    int n, int ld, const float* __restrict__ mean, const float* __restrict__ lsc,
    const float* __restrict__ quat, const float* __restrict__ opac, const float* __restrict__ sh,
    const gs_camera* __restrict__ cams, int n_views, const float4* __restrict__ splat,
    const uint8_t* __restrict__ flags, const float4* __restrict__ g2d, float* __restrict__ g_mean,
    float* __restrict__ g_lsc, float* __restrict__ g_quat, float* __restrict__ g_opac,
    float* __restrict__ g_sh, float* __restrict__ st_norm, uint32_t* __restrict__ st_views) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t L = (size_t)ld;
  const float m0 = mean[i], m1 = mean[L + i], m2 = mean[2 * L + i];
  float qw = quat[i], qx = quat[L + i], qy = quat[2 * L + i], qz = quat[3 * L + i];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (!(qn >= 1e-8f)) {  // culled in every view: zero gradient
    for (int k = 0; k < 3; ++k) g_mean[k * L + i] = g_lsc[k * L + i] = 0.f;
    for (int k = 0; k < 4; ++k) g_quat[k * L + i] = 0.f;
    g_opac[i] = 0.f;
    for (int k = 0; k < K * 3; ++k) g_sh[(size_t)k * L + i] = 0.f;
    return;
  }
  const float iq = 1.f / qn;
  qw *= iq;
  qx *= iq;
  qy *= iq;
  qz *= iq;
  float Rq[9];
  Rq[0] = 1.f - 2.f * (qy * qy + qz * qz);
  Rq[1] = 2.f * (qx * qy - qw * qz);
  Rq[2] = 2.f * (qx * qz + qw * qy);
  Rq[3] = 2.f * (qx * qy + qw * qz);
  Rq[4] = 1.f - 2.f * (qx * qx + qz * qz);
  Rq[5] = 2.f * (qy * qz - qw * qx);
  Rq[6] = 2.f * (qx * qz - qw * qy);
  Rq[7] = 2.f * (qy * qz + qw * qx);
  Rq[8] = 1.f - 2.f * (qx * qx + qy * qy);
  const float sg[3] = {__expf(lsc[i]), __expf(lsc[L + i]), __expf(lsc[2 * L + i])};
  float M[9], S[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sg[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
  float shv[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) shv[k] = sh[(size_t)k * L + i];

  float gm[3] = {0.f, 0.f, 0.f};
  float GSig[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gah = 0.f;
  float gsh[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;

  float st_acc = 0.f;
  uint32_t st_cnt = 0;
  for (int v = 0; v < n_views; ++v) {
    const size_t j = (size_t)v * L + i;
    const uint8_t fl = flags[j];
    if (!(fl & kVisible)) continue;
    const float4 ga = g2d[3 * j + 0], gb = g2d[3 * j + 1], gc = g2d[3 * j + 2];
    const float g_px = ga.x, g_py = ga.y, g_A = ga.z, g_B = ga.w, g_C = gb.x, g_al = gb.y;
    st_acc += sqrtf(g_px * g_px + g_py * g_py);
    ++st_cnt;
    const float g_rgb[3] = {gb.z, gb.w, gc.x};
    if (g_px == 0.f && g_py == 0.f && g_A == 0.f && g_B == 0.f && g_C == 0.f && g_al == 0.f &&
        g_rgb[0] == 0.f && g_rgb[1] == 0.f && g_rgb[2] == 0.f)
      continue;
    const gs_camera& cam = cams[v];
    float R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (float)cam.R[k];
    const float t0 = (float)cam.t[0], t1 = (float)cam.t[1], t2 = (float)cam.t[2];
    const float fx = (float)cam.fx, fy = (float)cam.fy;
    const float x0 = R[0] * m0 + R[1] * m1 + R[2] * m2 + t0;
    const float x1 = R[3] * m0 + R[4] * m1 + R[5] * m2 + t1;
    const float z = R[6] * m0 + R[7] * m1 + R[8] * m2 + t2;
    const float iz = 1.f / z, iz2 = iz * iz;
    gah += g_al;

    // colour -> SH coefficients and view direction
    {
      const float ccx = -(R[0] * t0 + R[3] * t1 + R[6] * t2);
      const float ccy = -(R[1] * t0 + R[4] * t1 + R[7] * t2);
      const float ccz = -(R[2] * t0 + R[5] * t1 + R[8] * t2);
      float dx = m0 - ccx, dy = m1 - ccy, dz = m2 - ccz;
      const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
      const float idist = 1.f / dist;
      dx *= idist;
      dy *= idist;
      dz *= idist;
      float Y[K];
      sh_eval<DEG>(dx, dy, dz, Y);
      float gcol[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gcol[ch] = (fl & (1u << ch)) ? 0.f : g_rgb[ch];
      float w[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        w[k] = gcol[0] * shv[3 * k] + gcol[1] * shv[3 * k + 1] + gcol[2] * shv[3 * k + 2];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gsh[3 * k + ch] += Y[k] * gcol[ch];
      }
      if constexpr (DEG > 0) {
        float gx, gy, gz;
        sh_grad_dot<DEG>(dx, dy, dz, w, gx, gy, gz);
        const float dd = gx * dx + gy * dy + gz * dz;
        gm[0] += (gx - dd * dx) * idist;
        gm[1] += (gy - dd * dy) * idist;
        gm[2] += (gz - dd * dz) * idist;
      }
    }

    // screen mean -> camera space
    float gx0 = g_px * fx * iz, gx1 = g_py * fy * iz;
    float gz = -(g_px * fx * x0 + g_py * fy * x1) * iz2;

    // conic -> 2D covariance: G_S = -Q G_Q Q, G_Q = [[gA, gB/2], [gB/2, gC]]
    const float4 s0 = splat[kSplatF4 * j + 0];
    const float4 s1 = splat[kSplatF4 * j + 1];
    const float A = s0.z, B = s0.w, C = s1.x;
    const float q00 = A * g_A + B * 0.5f * g_B, q01 = A * 0.5f * g_B + B * g_C;
    const float q10 = B * g_A + C * 0.5f * g_B, q11 = B * 0.5f * g_B + C * g_C;
    const float G00 = -(q00 * A + q01 * B), G01 = -(q00 * B + q01 * C);
    const float G10 = -(q10 * A + q11 * B), G11 = -(q10 * B + q11 * C);
    const float Gs01 = 0.5f * (G01 + G10);

    // Jacobian (clamped components carry no gradient through x/z, y/z)
    const float limx = 1.3f * (0.5f * (float)cam.width / fx);
    const float limy = 1.3f * (0.5f * (float)cam.height / fy);
    float u = x0 * iz, wv = x1 * iz;
    u = fminf(fmaxf(u, -limx), limx);
    wv = fminf(fmaxf(wv, -limy), limy);
    const float J00 = fx * iz, J02 = -fx * u * iz, J11 = fy * iz, J12 = -fy * wv * iz;
    // V = W S W^T
    float T1[9], V[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        T1[3 * r + c] = R[3 * r] * S[c] + R[3 * r + 1] * S[3 + c] + R[3 * r + 2] * S[6 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        V[3 * r + c] = T1[3 * r] * R[3 * c] + T1[3 * r + 1] * R[3 * c + 1] + T1[3 * r + 2] * R[3 * c + 2];
    // GSJ = G_S J (2x3), G_S symmetric [[G00, Gs01], [Gs01, G11]]
    const float J[6] = {J00, 0.f, J02, 0.f, J11, J12};
    float GSJ[6];
    for (int c = 0; c < 3; ++c) {
      GSJ[c] = G00 * J[c] + Gs01 * J[3 + c];
      GSJ[3 + c] = Gs01 * J[c] + G11 * J[3 + c];
    }
    // G_V = J^T G_S J
    float GV[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) GV[3 * r + c] = J[r] * GSJ[c] + J[3 + r] * GSJ[3 + c];
    // G_J = 2 G_S J V (only the non-constant entries are used)
    float GJ[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        GJ[3 * r + c] = 2.f * (GSJ[3 * r] * V[c] + GSJ[3 * r + 1] * V[3 + c] + GSJ[3 * r + 2] * V[6 + c]);
    gz += -(GJ[0] * fx + GJ[4] * fy) * iz2;
    if (fl & kClampU) {
      gz += GJ[2] * fx * u * iz2;
    } else {
      gx0 += -GJ[2] * fx * iz2;
      gz += GJ[2] * 2.f * fx * x0 * iz2 * iz;
    }
    if (fl & kClampV) {
      gz += GJ[5] * fy * wv * iz2;
    } else {
      gx1 += -GJ[5] * fy * iz2;
      gz += GJ[5] * 2.f * fy * x1 * iz2 * iz;
    }
    gm[0] += R[0] * gx0 + R[3] * gx1 + R[6] * gz;
    gm[1] += R[1] * gx0 + R[4] * gx1 + R[7] * gz;
    gm[2] += R[2] * gx0 + R[5] * gx1 + R[8] * gz;
    // G_Sigma += W^T G_V W
    float Tm[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Tm[3 * r + c] = R[r] * GV[c] + R[3 + r] * GV[3 + c] + R[6 + r] * GV[6 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        GSig[3 * r + c] += Tm[3 * r] * R[c] + Tm[3 * r + 1] * R[3 + c] + Tm[3 * r + 2] * R[6 + c];
  }

  // Sigma = M M^T -> M = R_q diag(sigma) -> (log-scale, quaternion)
  float GM[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      GM[3 * r + c] = (GSig[3 * r] + GSig[r]) * M[c] + (GSig[3 * r + 1] + GSig[3 + r]) * M[3 + c] +
                      (GSig[3 * r + 2] + GSig[6 + r]) * M[6 + c];
  float gs[3], GR[9];
  for (int c = 0; c < 3; ++c) {
    float acc = 0.f;
    for (int r = 0; r < 3; ++r) {
      acc += Rq[3 * r + c] * GM[3 * r + c];
      GR[3 * r + c] = GM[3 * r + c] * sg[c];
    }
    gs[c] = acc * sg[c];
  }
  float gh[4];
  gh[0] = 2.f * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
  gh[1] = 2.f * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.f * qx * GR[4] - qw * GR[5] + qz * GR[6] +
                 qw * GR[7] - 2.f * qx * GR[8]);
  gh[2] = 2.f * (-2.f * qy * GR[0] + qx * GR[1] + qw * GR[2] + qx * GR[3] + qz * GR[5] - qw * GR[6] +
                 qz * GR[7] - 2.f * qy * GR[8]);
  gh[3] = 2.f * (-2.f * qz * GR[0] - qw * GR[1] + qx * GR[2] + qw * GR[3] - 2.f * qz * GR[4] +
                 qy * GR[5] + qx * GR[6] + qy * GR[7]);
  const float dq = gh[0] * qw + gh[1] * qx + gh[2] * qy + gh[3] * qz;
  const float qh[4] = {qw, qx, qy, qz};
  const float ah = 1.f / (1.f + __expf(-opac[i]));
  g_mean[i] = gm[0];
  g_mean[L + i] = gm[1];
  g_mean[2 * L + i] = gm[2];
  g_lsc[i] = gs[0];
  g_lsc[L + i] = gs[1];
  g_lsc[2 * L + i] = gs[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) g_quat[(size_t)k * L + i] = (gh[k] - dq * qh[k]) * iq;
  g_opac[i] = gah * ah * (1.f - ah);
#pragma unroll
  for (int k = 0; k < K * 3; ++k) g_sh[(size_t)k * L + i] = gsh[k];
  if (st_norm) {  // densification statistics (uniform branch)
    st_norm[i] += st_acc;
    st_views[i] += st_cnt;
  }
}

}  // namespace

void launch_project(const gs_gaussians& g, const gs_camera* cams, int V, const gs_projected& o,
                    hipStream_t s) {
  const int chunks = (g.n + 255) / 256;
  if (chunks == 0 || V <= 0) return;
  // enough view groups for about 16 waves per SIMD (1024 SIMDs), each group
  // at least one view
  const int64_t waves = 4 * (int64_t)chunks;
  int groups = (int)std::min<int64_t>(V, std::max<int64_t>(1, (16384 + waves - 1) / waves));
  const int per_group = (V + groups - 1) / groups;
  groups = (V + per_group - 1) / per_group;
  const int64_t blocks = (int64_t)((chunks + 7) / 8) * 8 * groups;
  StageScope scope(kStProject, s);
  float4* sp = reinterpret_cast<float4*>(o.splat);
  int4* rc = reinterpret_cast<int4*>(o.rect);
#define GS_PROJ(D)                                                                             \
  hipLaunchKernelGGL(k_project<D>, dim3((unsigned)blocks), dim3(256), 0, s, g.n, g.ld, g.mean, \
                     g.log_scale, g.quat, g.opacity, g.sh, cams, V, groups, per_group, sp, rc, \
                     o.tiles_touched, o.depth_bits, o.flags,                                   \
                     (o.options & (GS_PROJECT_TIGHT_RECT | GS_PROJECT_TILE_SPANS)) != 0,      \
                     (o.options & GS_PROJECT_TILE_SPANS) != 0)
  switch (g.sh_degree) {
    case 0: GS_PROJ(0); break;
    case 1: GS_PROJ(1); break;
    case 2: GS_PROJ(2); break;
    default: GS_PROJ(3); break;
  }
#undef GS_PROJ
}

void launch_project_bwd(const gs_gaussians& g, const gs_camera* cams, int V,
                        const gs_projected& p, const float* grad2d, gs_gaussians& gr,
                        float* st_norm, uint32_t* st_views, hipStream_t s) {
  const int blocks = (g.n + 255) / 256;
  if (blocks == 0) return;
  StageScope scope(kStProjectBwd, s);
  const float4* sp = reinterpret_cast<const float4*>(p.splat);
  const float4* g2 = reinterpret_cast<const float4*>(grad2d);
#define GS_PROJ_BWD(D)                                                                        \
  hipLaunchKernelGGL(k_project_bwd<D>, dim3(blocks), dim3(256), 0, s, g.n, g.ld, g.mean,     \
                     g.log_scale, g.quat, g.opacity, g.sh, cams, V, sp, p.flags, g2, gr.mean, \
                     gr.log_scale, gr.quat, gr.opacity, gr.sh, st_norm, st_views)
  switch (g.sh_degree) {
    case 0: GS_PROJ_BWD(0); break;
    case 1: GS_PROJ_BWD(1); break;
    case 2: GS_PROJ_BWD(2); break;
    default: GS_PROJ_BWD(3); break;
  }
#undef GS_PROJ_BWD
}

}  // namespace gs
