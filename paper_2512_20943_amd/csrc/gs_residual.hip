// Residual bookkeeping of sent updates and their quantised planes (AirGS
// Sec. III-C, Eq. (11), (12)).
//
// The server keeps the true accumulated delta D_t of the frame and the sum
// D'_(t-1) of what the client has already received.  The update sent for
// frame t is the pruning mask applied to the residual D_t - D'_(t-1), so the
// motion of a pruned Gaussian is not lost but sent with a later frame.  Sent
// updates travel as signed 8- or 16-bit codes with one scale per channel
// (symmetric, so a pruned texel stays exactly zero); both ends add the
// dequantised update to D' so that they hold bit-identical sums, and the
// client applies D'_t to the anchor in the same pass.
//
// Elementwise, HBM-bound, FP32 planes, one IEEE operation per step and
// contraction off so that every step rounds the way it is written.
#include "gs_internal.h"

namespace gs {
namespace {

#pragma clang fp contract(off)

constexpr int kChannels = 8;

// d = mask ? D - P : 0 for texels i < n, 0 elsewhere; per-channel max |d|
// over i < n accumulated as the bits of a non-negative float.
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ D,
                                                  const float* __restrict__ P,
                                                  const uint8_t* __restrict__ mask, int n,
                                                  size_t plane, float* __restrict__ d,
                                                  uint32_t* __restrict__ absmax_bits) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool keep = t < (size_t)n && mask[t] != 0;
  __shared__ uint32_t s_max[4][kChannels];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kChannels; ++c) {
    float v = 0.f;
    if (keep) v = D[c * plane + t] - P[c * plane + t];
    if (t < plane) d[c * plane + t] = v;
    uint32_t m = __float_as_uint(fabsf(v));
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    if (lane == 0) s_max[wave][c] = m;
  }
  __syncthreads();
  if (threadIdx.x < kChannels) {
    const int c = threadIdx.x;
    const uint32_t m = max(max(s_max[0][c], s_max[1][c]), max(s_max[2][c], s_max[3][c]));
    if (m) atomicMax(absmax_bits + c, m);
  }
}

template <typename Q>
__global__ __launch_bounds__(256) void k_quantize(const float* __restrict__ d,
                                                  const float* __restrict__ absmax, float qmax,
                                                  int n, size_t plane, Q* __restrict__ q,
                                                  float* __restrict__ scale_out,
                                                  float* __restrict__ P) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= plane) return;
#pragma unroll
  for (int c = 0; c < kChannels; ++c) {
    const float a = absmax[c];
    const float sc = a > 0.f ? a / qmax : 0.f;
    if (t == 0) scale_out[c] = sc;
    float code = 0.f;
    if (t < (size_t)n && sc > 0.f) code = fminf(fmaxf(rintf(d[c * plane + t] / sc), -qmax), qmax);
    q[c * plane + t] = (Q)code;
    if (P && t < (size_t)n) P[c * plane + t] = P[c * plane + t] + code * sc;
  }
}

// Client side: P += code * scale at texels i < n, then the frame is the
// anchor with P applied (all texels, as the frame-update apply with a full
// mask; FP64 arithmetic rounded once to FP32).
template <typename Q>
__global__ __launch_bounds__(256) void k_apply_quantized(
    int n, int ld, size_t plane, const Q* __restrict__ q, const float* __restrict__ scale,
    float* __restrict__ P, const float* __restrict__ mean, const float* __restrict__ quat,
    const float* __restrict__ opac, float* __restrict__ mean_o, float* __restrict__ quat_o,
    float* __restrict__ opac_o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float u[kChannels];
#pragma unroll
  for (int c = 0; c < kChannels; ++c) {
    const float v = P[c * plane + i] + (float)q[c * plane + i] * scale[c];
    P[c * plane + i] = v;
    u[c] = v;
  }
  mean_o[i] = (float)((double)mean[i] + (double)u[0]);
  mean_o[ld + i] = (float)((double)mean[ld + i] + (double)u[1]);
  mean_o[2 * (size_t)ld + i] = (float)((double)mean[2 * (size_t)ld + i] + (double)u[2]);
  const double aw = u[3], ax = u[4], ay = u[5], az = u[6];
  const double bw = quat[i], bx = quat[ld + i], by = quat[2 * (size_t)ld + i],
               bz = quat[3 * (size_t)ld + i];
  quat_o[i] = (float)(((aw * bw - ax * bx) - ay * by) - az * bz);
  quat_o[ld + i] = (float)(((aw * bx + ax * bw) + ay * bz) - az * by);
  quat_o[2 * (size_t)ld + i] = (float)(((aw * by - ax * bz) + ay * bw) + az * bx);
  quat_o[3 * (size_t)ld + i] = (float)(((aw * bz + ax * by) - ay * bx) + az * bw);
  opac_o[i] = (float)((double)opac[i] + (double)u[7]);
}

}  // namespace

void launch_residual(const float* D, const float* P, const uint8_t* mask, int n, int gw, int gh,
                     float* d, float* absmax, hipStream_t s) {
  const size_t plane = (size_t)gw * (size_t)gh;
  const int blocks = (int)((plane + 255) / 256);
  if (blocks == 0) return;
  StageScope scope(kStResidual, s);
  hipLaunchKernelGGL(k_residual, dim3(blocks), dim3(256), 0, s, D, P, mask, n, plane, d,
                     reinterpret_cast<uint32_t*>(absmax));
}

void launch_quantize(const float* d, const float* absmax, int bits, int n, int gw, int gh,
                     void* q, float* scale, float* P, hipStream_t s) {
  const size_t plane = (size_t)gw * (size_t)gh;
  const int blocks = (int)((plane + 255) / 256);
  if (blocks == 0) return;
  StageScope scope(kStResidual, s);
  const float qmax = (float)((1 << (bits - 1)) - 1);
  if (bits == 8)
    hipLaunchKernelGGL(k_quantize<int8_t>, dim3(blocks), dim3(256), 0, s, d, absmax, qmax, n,
                       plane, static_cast<int8_t*>(q), scale, P);
  else
    hipLaunchKernelGGL(k_quantize<int16_t>, dim3(blocks), dim3(256), 0, s, d, absmax, qmax, n,
                       plane, static_cast<int16_t*>(q), scale, P);
}

void launch_apply_quantized(const gs_gaussians& a, const void* q, int bits, const float* scale,
                            float* P, int gw, int gh, gs_gaussians& f, hipStream_t s) {
  const size_t plane = (size_t)gw * (size_t)gh;
  const int blocks = (a.n + 255) / 256;
  if (blocks == 0) return;
  StageScope scope(kStResidual, s);
  if (bits == 8)
    hipLaunchKernelGGL(k_apply_quantized<int8_t>, dim3(blocks), dim3(256), 0, s, a.n, a.ld, plane,
                       static_cast<const int8_t*>(q), scale, P, a.mean, a.quat, a.opacity, f.mean,
                       f.quat, f.opacity);
  else
    hipLaunchKernelGGL(k_apply_quantized<int16_t>, dim3(blocks), dim3(256), 0, s, a.n, a.ld,
                       plane, static_cast<const int16_t*>(q), scale, P, a.mean, a.quat, a.opacity,
                       f.mean, f.quat, f.opacity);
}

}  // namespace gs
