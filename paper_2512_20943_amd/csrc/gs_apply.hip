// Frame update: anchor Gaussians plus a decoded, pruned delta image set
// (AirGS Eq. (2), (5), (12): frame = anchor + accumulated delta; Eq. (3):
// attribute images with one texel per Gaussian; Eq. (11): pruning mask).
//
// Elementwise and HBM-bound: 8 delta planes + 1 mask byte + 8 anchor values
// read, 8 frame values written per Gaussian (97 B).  The arithmetic is done
// in FP64 and rounded once to the FP32 parameter storage, so that the frame
// is the correctly rounded result of the update, independent of the order a
// compiler might pick.
#include "gs_internal.h"

namespace gs {
namespace {

#pragma clang fp contract(off)

__global__ __launch_bounds__(256) void k_apply(int n, int ld, size_t plane,
                                               const float* __restrict__ mean,
                                               const float* __restrict__ quat,
                                               const float* __restrict__ opac,
                                               const float* __restrict__ delta,
                                               const uint8_t* __restrict__ mask, float* mean_o,
                                               float* quat_o, float* opac_o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m0 = mean[i], m1 = mean[ld + i], m2 = mean[2 * (size_t)ld + i];
  const float q0 = quat[i], q1 = quat[ld + i], q2 = quat[2 * (size_t)ld + i],
              q3 = quat[3 * (size_t)ld + i];
  const float o = opac[i];
  if (mask[i]) {
    mean_o[i] = (float)((double)m0 + (double)delta[i]);
    mean_o[ld + i] = (float)((double)m1 + (double)delta[plane + i]);
    mean_o[2 * (size_t)ld + i] = (float)((double)m2 + (double)delta[2 * plane + i]);
    // Hamilton product dq (x) q, left operand the delta
    const double aw = delta[3 * plane + i], ax = delta[4 * plane + i],
                 ay = delta[5 * plane + i], az = delta[6 * plane + i];
    const double bw = q0, bx = q1, by = q2, bz = q3;
    const double rw = ((aw * bw - ax * bx) - ay * by) - az * bz;
    const double rx = ((aw * bx + ax * bw) + ay * bz) - az * by;
    const double ry = ((aw * by - ax * bz) + ay * bw) + az * bx;
    const double rz = ((aw * bz + ax * by) - ay * bx) + az * bw;
    quat_o[i] = (float)rw;
    quat_o[ld + i] = (float)rx;
    quat_o[2 * (size_t)ld + i] = (float)ry;
    quat_o[3 * (size_t)ld + i] = (float)rz;
    opac_o[i] = (float)((double)o + (double)delta[7 * plane + i]);
  } else {
    mean_o[i] = m0;
    mean_o[ld + i] = m1;
    mean_o[2 * (size_t)ld + i] = m2;
    quat_o[i] = q0;
    quat_o[ld + i] = q1;
    quat_o[2 * (size_t)ld + i] = q2;
    quat_o[3 * (size_t)ld + i] = q3;
    opac_o[i] = o;
  }
}

// dL/d(delta) from dL/d(frame): identity for the additive channels, the
// transpose of q -> dq (x) q (a linear map of dq) for the quaternion.
__global__ __launch_bounds__(256) void k_apply_bwd(int n, int ld, size_t plane,
                                                   const float* __restrict__ aq,
                                                   const uint8_t* __restrict__ mask,
                                                   const float* __restrict__ gmean,
                                                   const float* __restrict__ gquat,
                                                   const float* __restrict__ gopac,
                                                   float* __restrict__ gdelta) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= plane) return;
  float out[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (t < (size_t)n && mask[t]) {
    out[0] = gmean[t];
    out[1] = gmean[ld + t];
    out[2] = gmean[2 * (size_t)ld + t];
    const float bw = aq[t], bx = aq[ld + t], by = aq[2 * (size_t)ld + t],
                bz = aq[3 * (size_t)ld + t];
    const float g0 = gquat[t], g1 = gquat[ld + t], g2 = gquat[2 * (size_t)ld + t],
                g3 = gquat[3 * (size_t)ld + t];
    out[3] = bw * g0 + bx * g1 + by * g2 + bz * g3;
    out[4] = -bx * g0 + bw * g1 - bz * g2 + by * g3;
    out[5] = -by * g0 + bz * g1 + bw * g2 - bx * g3;
    out[6] = -bz * g0 - by * g1 + bx * g2 + bw * g3;
    out[7] = gopac[t];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) gdelta[c * plane + t] = out[c];
}

}  // namespace

void launch_apply(const gs_gaussians& a, const float* delta, const uint8_t* mask, int gw, int gh,
                  gs_gaussians& f, hipStream_t s) {
  const size_t plane = (size_t)gw * (size_t)gh;
  const int blocks = (a.n + 255) / 256;
  if (blocks == 0) return;
  StageScope scope(kStApply, s);
  hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(256), 0, s, a.n, a.ld, plane, a.mean, a.quat,
                     a.opacity, delta, mask, f.mean, f.quat, f.opacity);
}

void launch_apply_bwd(int n, const gs_frame_update& u, const gs_gaussians& g, float* gdelta,
                      hipStream_t s) {
  const size_t plane = (size_t)u.gw * (size_t)u.gh;
  const int blocks = (int)((plane + 255) / 256);
  if (blocks == 0) return;
  StageScope scope(kStApplyBwd, s);
  hipLaunchKernelGGL(k_apply_bwd, dim3(blocks), dim3(256), 0, s, n, u.ld, plane, u.anchor_quat,
                     u.mask, g.mean, g.quat, g.opacity, gdelta);
}

}  // namespace gs
