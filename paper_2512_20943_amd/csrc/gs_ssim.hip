// Photometric loss of AirGS Eq. (1): (1 - lambda) L1 + lambda (1 - SSIM),
// with SSIM over an 11x11 Gaussian window (sigma 1.5), zero padding,
// C1 = 0.01^2, C2 = 0.03^2, averaged over every image value.
//
// Two tiled passes, each a separable 11-tap window over a 32x8 output tile
// whose 42x18 input footprint is staged in LDS:
//   1. windowed statistics of x, y, x^2, y^2, xy -> per-pixel SSIM index and
//      the partials A1 = dS/dmu_x - 2 mu_x dS/dvar_x - mu_y dS/dcov,
//      A2 = dS/dvar_x, A3 = dS/dcov (written to the workspace), loss partials;
//   2. the adjoint window over A1..A3 -> dL/dx = ((1 - lambda) sign(x - y)
//      - lambda (w*A1 + 2 x w*A2 + y w*A3)) / count.
// HBM-bound: 8 B read + 12 B written per value in pass 1, 20 B read + 4 B
// written in pass 2.
#include <cmath>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kR = 5;            // window radius
constexpr int kTW = 32, kTH = 8;  // output tile
constexpr int kIW = kTW + 2 * kR, kIH = kTH + 2 * kR;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
  float w[2 * kR + 1];
};

// Stage a (kIH x kIW) footprint of up to 3 planes with zero padding.
template <int NP>
__device__ __forceinline__ void stage(float (*dst)[kIH][kIW], const float* const* src, int W,
                                      int H, int x0, int y0) {
  for (int t = threadIdx.x; t < kIH * kIW; t += blockDim.x) {
    const int r = t / kIW, c = t - r * kIW;
    const int yy = y0 + r - kR, xx = x0 + c - kR;
    const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
    const size_t p = (size_t)yy * W + xx;
#pragma unroll
    for (int q = 0; q < NP; ++q) dst[q][r][c] = in ? src[q][p] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_ssim_stats(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int W, int H,
                                                   Window win, float lambda, float inv_count,
                                                   float* __restrict__ amaps,
                                                   double* __restrict__ loss) {
  __shared__ float s_in[2][kIH][kIW];
  __shared__ float s_h[5][kIH][kTW];
  __shared__ double s_red[4];
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
  const float* srcs[2] = {img + pl * plane, tgt + pl * plane};
  stage<2>(s_in, srcs, W, H, x0, y0);
  __syncthreads();
  // horizontal window: kIH rows x kTW output columns, 5 statistics
  for (int t = threadIdx.x; t < kIH * kTW; t += blockDim.x) {
    const int r = t / kTW, c = t - r * kTW;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int i = 0; i <= 2 * kR; ++i) {
      const float x = s_in[0][r][c + i], y = s_in[1][r][c + i], w = win.w[i];
      a = fmaf(w, x, a);
      b = fmaf(w, y, b);
      aa = fmaf(w, x * x, aa);
      bb = fmaf(w, y * y, bb);
      ab = fmaf(w, x * y, ab);
    }
    s_h[0][r][c] = a;
    s_h[1][r][c] = b;
    s_h[2][r][c] = aa;
    s_h[3][r][c] = bb;
    s_h[4][r][c] = ab;
  }
  __syncthreads();
  const int c = threadIdx.x % kTW, r = threadIdx.x / kTW;
  const int x = x0 + c, y = y0 + r;
  double part = 0.0;
  if (x < W && y < H) {
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int j = 0; j <= 2 * kR; ++j) {
      const float w = win.w[j];
      mx = fmaf(w, s_h[0][r + j][c], mx);
      my = fmaf(w, s_h[1][r + j][c], my);
      exx = fmaf(w, s_h[2][r + j][c], exx);
      eyy = fmaf(w, s_h[3][r + j][c], eyy);
      exy = fmaf(w, s_h[4][r + j][c], exy);
    }
    const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const float N1 = 2.f * mx * my + kC1, N2 = 2.f * sxy + kC2;
    const float D1 = mx * mx + my * my + kC1, D2 = sxx + syy + kC2;
    const float iD = 1.f / (D1 * D2);
    const float S = N1 * N2 * iD;
    const float dS_dmx = 2.f * my * N2 * iD - S * 2.f * mx / D1;
    const float dS_dsxx = -S / D2;
    const float dS_dsxy = 2.f * N1 * iD;
    const size_t p = (size_t)y * W + x;
    float* a = amaps + (size_t)pl * 3 * plane;
    a[p] = dS_dmx - 2.f * mx * dS_dsxx - my * dS_dsxy;
    a[plane + p] = dS_dsxx;
    a[2 * plane + p] = dS_dsxy;
    const float d = s_in[0][r + kR][c + kR] - s_in[1][r + kR][c + kR];
    part = (double)(1.f - lambda) * fabs((double)d) - (double)lambda * (double)S;
  }
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])) * (double)inv_count;
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) tot += (double)lambda;
    atomicAdd(loss, tot);
  }
}

__global__ __launch_bounds__(256) void k_ssim_grad(const float* __restrict__ img,
                                                  const float* __restrict__ tgt, int W, int H,
                                                  Window win, float lambda, float inv_count,
                                                  const float* __restrict__ amaps,
                                                  float* __restrict__ grad) {
  __shared__ float s_in[3][kIH][kIW];
  __shared__ float s_h[3][kIH][kTW];
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
  const float* a = amaps + (size_t)pl * 3 * plane;
  const float* srcs[3] = {a, a + plane, a + 2 * plane};
  stage<3>(s_in, srcs, W, H, x0, y0);
  __syncthreads();
  for (int t = threadIdx.x; t < kIH * kTW; t += blockDim.x) {
    const int r = t / kTW, c = t - r * kTW;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int i = 0; i <= 2 * kR; ++i) {
      const float w = win.w[i];
      s0 = fmaf(w, s_in[0][r][c + i], s0);
      s1 = fmaf(w, s_in[1][r][c + i], s1);
      s2 = fmaf(w, s_in[2][r][c + i], s2);
    }
    s_h[0][r][c] = s0;
    s_h[1][r][c] = s1;
    s_h[2][r][c] = s2;
  }
  __syncthreads();
  const int c = threadIdx.x % kTW, r = threadIdx.x / kTW;
  const int x = x0 + c, y = y0 + r;
  if (x >= W || y >= H) return;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
  for (int j = 0; j <= 2 * kR; ++j) {
    const float w = win.w[j];
    g0 = fmaf(w, s_h[0][r + j][c], g0);
    g1 = fmaf(w, s_h[1][r + j][c], g1);
    g2 = fmaf(w, s_h[2][r + j][c], g2);
  }
  const size_t p = (size_t)pl * plane + (size_t)y * W + x;
  const float xv = img[p], yv = tgt[p];
  const float d = xv - yv;
  const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
  const float gs = g0 + 2.f * xv * g1 + yv * g2;
  grad[p] = ((1.f - lambda) * sg - lambda * gs) * inv_count;
}

Window make_window() {
  Window win;
  double w[2 * kR + 1], s = 0.0;
  for (int i = -kR; i <= kR; ++i) {
    w[i + kR] = std::exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
    s += w[i + kR];
  }
  for (int i = 0; i <= 2 * kR; ++i) win.w[i] = (float)(w[i] / s);
  return win;
}

}  // namespace

size_t l1_dssim_workspace_bytes(int planes, int H, int W) {
  return (size_t)planes * 3 * (size_t)H * (size_t)W * sizeof(float);
}

void launch_l1_dssim(const float* image, const float* target, int planes, int H, int W,
                     float lambda, float* grad, double* loss, void* ws, hipStream_t s) {
  if (planes <= 0 || H <= 0 || W <= 0) return;
  const Window win = make_window();
  const double count = (double)planes * (double)H * (double)W;
  const float inv = (float)(1.0 / count);
  const dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH, planes);
  float* amaps = static_cast<float*>(ws);
  StageScope scope(kStDssim, s);
  hipLaunchKernelGGL(k_ssim_stats, grid, dim3(256), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, loss);
  hipLaunchKernelGGL(k_ssim_grad, grid, dim3(256), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, grad);
}

}  // namespace gs
