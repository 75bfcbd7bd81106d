// Frame update: anchor Gaussians plus a decoded, pruned delta image set
// (AirGS Eq. (2), (5), (12): frame = anchor + accumulated delta; Eq. (3):
// attribute images with one texel per Gaussian; Eq. (11): pruning mask).
//
// Elementwise and HBM-bound: 8 delta planes + 1 mask byte + 8 anchor values
// read, 8 frame values written per Gaussian (97 B).  The backward optionally
// carries the temporal term of Eq. (6)/(7) (8 more delta values read).  The arithmetic is done
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
// transpose of q -> dq (x) q (a linear map of dq) for the quaternion.  With
// TEMPORAL, the temporal term (Eq. (6)/(7)) adds w * sign(delta - e) at every
// texel i < n, e the no-motion update, and its value w * sum |delta - e| is
// reduced per block and added to *tloss.
template <bool TEMPORAL>
__global__ __launch_bounds__(256) void k_apply_bwd(int n, int ld, size_t plane,
                                                   const float* __restrict__ aq,
                                                   const uint8_t* __restrict__ mask,
                                                   const float* __restrict__ gmean,
                                                   const float* __restrict__ gquat,
                                                   const float* __restrict__ gopac,
                                                   float* __restrict__ gdelta, float tw,
                                                   const float* __restrict__ delta,
                                                   double* __restrict__ tloss) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
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
  if constexpr (TEMPORAL) {
    float acc = 0.f;
    if (t < (size_t)n) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float r = delta[c * plane + t] - (c == 3 ? 1.f : 0.f);
        const float sg = r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f);
        out[c] += tw * sg;
        acc += fabsf(r);
      }
    }
    if (tloss) {
      double a = (double)acc;
      for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
      __shared__ double s_red[4];
      if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = a;
      __syncthreads();
      if (threadIdx.x == 0)
        atomicAdd(tloss, (double)tw * ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])));
    }
  }
  if (t >= plane) return;
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
  if (u.temporal_weight != 0.f)
    hipLaunchKernelGGL(k_apply_bwd<true>, dim3(blocks), dim3(256), 0, s, n, u.ld, plane,
                       u.anchor_quat, u.mask, g.mean, g.quat, g.opacity, gdelta,
                       u.temporal_weight, u.delta, u.temporal_loss);
  else
    hipLaunchKernelGGL(k_apply_bwd<false>, dim3(blocks), dim3(256), 0, s, n, u.ld, plane,
                       u.anchor_quat, u.mask, g.mean, g.quat, g.opacity, gdelta, 0.f,
                       (const float*)nullptr, (double*)nullptr);
}

}  // namespace gs
