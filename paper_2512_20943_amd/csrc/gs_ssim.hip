// Photometric loss of AirGS Eq. (1): (1 - lambda) L1 + lambda (1 - SSIM),
// with SSIM over an 11x11 Gaussian window (sigma 1.5), zero padding,
// C1 = 0.01^2, C2 = 0.03^2, averaged over every image value.
//
// Two tiled passes, each a separable 11-tap window over a 32x32 output tile
// whose 42x42 input footprint is staged in LDS (horizontal pass: 8 columns
// per thread, vertical pass: 4 rows per thread, sliding in registers):
//   1. windowed statistics of x, y, x^2, y^2, xy -> per-pixel SSIM index and
//      the partials A1 = dS/dmu_x - 2 mu_x dS/dvar_x - mu_y dS/dcov,
//      A2 = dS/dvar_x, A3 = dS/dcov (written to the workspace), one loss
//      partial per tile (summed by one workgroup afterwards);
//   2. the adjoint window over A1..A3 -> dL/dx = ((1 - lambda) sign(x - y)
//      - lambda (w*A1 + 2 x w*A2 + y w*A3)) / count.
// HBM-bound: 8 B read + 12 B written per value in pass 1, 20 B read + 4 B
// written in pass 2.
#include <cmath>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kR = 5;             // window radius
constexpr int kT = 32;            // output tile side
constexpr int kI = kT + 2 * kR;   // staged footprint side (42)
constexpr int kIP = kI + 1;       // padded LDS row stride of the staged input
constexpr int kTP = kT + 1;       // padded LDS row stride of the horizontal sums
constexpr int kSeg = 8;           // columns per thread in the horizontal pass
constexpr int kRows = 4;          // output rows per thread in the vertical pass
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
  float w[2 * kR + 1];
};

// Stage a kI x kI footprint of NP planes with zero padding.  Every thread
// issues all of its global loads before its first LDS store, so the loads of
// one workgroup are in flight together.
template <int NP>
__device__ __forceinline__ void stage(float (*dst)[kI][kIP], const float* const* src, int W, int H,
                                      int x0, int y0) {
  constexpr int kPer = (kI * kI + 255) / 256;
  float v[NP][kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int t = threadIdx.x + u * 256;
    const int r = t / kI, c = t - r * kI;
    const int yy = y0 + r - kR, xx = x0 + c - kR;
    const bool in = t < kI * kI && yy >= 0 && yy < H && xx >= 0 && xx < W;
    const size_t p = in ? (size_t)yy * W + xx : 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) v[q][u] = in ? src[q][p] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int t = threadIdx.x + u * 256;
    if (t < kI * kI) {
      const int r = t / kI, c = t - r * kI;
#pragma unroll
      for (int q = 0; q < NP; ++q) dst[q][r][c] = v[q][u];
    }
  }
}

// Horizontal window over the kI staged rows, kSeg consecutive output
// columns per work item (kI rows x kT/kSeg segments), sliding in registers.
// F maps the NP staged planes at one position to NS statistics.
template <int NP, int NS, typename F>
__device__ __forceinline__ void hpass(const float (*in)[kI][kIP], float (*out)[kI][kTP],
                                      const Window& win, F stat) {
  constexpr int kItems = kI * (kT / kSeg);
  for (int t = threadIdx.x; t < kItems; t += blockDim.x) {
    // consecutive threads take consecutive rows (with the padded strides
    // their LDS accesses fall into different banks)
    const int seg = t / kI, r = t - seg * kI, c0 = seg * kSeg;
    float acc[kSeg][NS];
#pragma unroll
    for (int o = 0; o < kSeg; ++o)
#pragma unroll
      for (int q = 0; q < NS; ++q) acc[o][q] = 0.f;
#pragma unroll
    for (int i = 0; i < kSeg + 2 * kR; ++i) {
      float v[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) v[p] = in[p][r][c0 + i];
      float st[NS];
      stat(v, st);
#pragma unroll
      for (int o = 0; o < kSeg; ++o) {
        const int tap = i - o;
        if (tap >= 0 && tap <= 2 * kR) {
#pragma unroll
          for (int q = 0; q < NS; ++q) acc[o][q] = fmaf(win.w[tap], st[q], acc[o][q]);
        }
      }
    }
#pragma unroll
    for (int o = 0; o < kSeg; ++o)
#pragma unroll
      for (int q = 0; q < NS; ++q) out[q][r][c0 + o] = acc[o][q];
  }
}

// Vertical window: thread (c, g) produces rows 4g..4g+3 of column c.
template <int NS>
__device__ __forceinline__ void vpass(const float (*h)[kI][kTP], const Window& win, int c, int g,
                                      float (*res)[NS]) {
#pragma unroll
  for (int o = 0; o < kRows; ++o)
#pragma unroll
    for (int q = 0; q < NS; ++q) res[o][q] = 0.f;
#pragma unroll
  for (int j = 0; j < kRows + 2 * kR; ++j) {
    float v[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] = h[q][kRows * g + j][c];
#pragma unroll
    for (int o = 0; o < kRows; ++o) {
      const int tap = j - o;
      if (tap >= 0 && tap <= 2 * kR) {
#pragma unroll
        for (int q = 0; q < NS; ++q) res[o][q] = fmaf(win.w[tap], v[q], res[o][q]);
      }
    }
  }
}

struct StatsShared {
  float in[2][kI][kIP];
  float h[5][kI][kTP];
  double red[4];
};

__global__ __launch_bounds__(256) void k_ssim_stats(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int W, int H,
                                                   Window win, float lambda, float inv_count,
                                                   float* __restrict__ amaps,
                                                   double* __restrict__ partial) {
  __shared__ StatsShared sh;
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z;
  const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
  const float* srcs[2] = {img + pl * plane, tgt + pl * plane};
  stage<2>(sh.in, srcs, W, H, x0, y0);
  __syncthreads();
  hpass<2, 5>(sh.in, sh.h, win, [](const float* v, float* st) {
    st[0] = v[0];
    st[1] = v[1];
    st[2] = v[0] * v[0];
    st[3] = v[1] * v[1];
    st[4] = v[0] * v[1];
  });
  __syncthreads();
  const int c = threadIdx.x % kT, g = threadIdx.x / kT;
  float res[kRows][5];
  vpass<5>(sh.h, win, c, g, res);
  double part = 0.0;
  float* a = amaps + (size_t)pl * 3 * plane;
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int x = x0 + c, y = y0 + kRows * g + o;
    if (x < W && y < H) {
      const float mx = res[o][0], my = res[o][1];
      const float sxx = res[o][2] - mx * mx, syy = res[o][3] - my * my, sxy = res[o][4] - mx * my;
      const float N1 = 2.f * mx * my + kC1, N2 = 2.f * sxy + kC2;
      const float D1 = mx * mx + my * my + kC1, D2 = sxx + syy + kC2;
      const float iD = 1.f / (D1 * D2);
      const float S = N1 * N2 * iD;
      const float dS_dmx = 2.f * my * N2 * iD - S * 2.f * mx / D1;
      const float dS_dsxx = -S / D2;
      const float dS_dsxy = 2.f * N1 * iD;
      const size_t p = (size_t)y * W + x;
      a[p] = dS_dmx - 2.f * mx * dS_dsxx - my * dS_dsxy;
      a[plane + p] = dS_dsxx;
      a[2 * plane + p] = dS_dsxy;
      const int ly = kRows * g + o + kR, lx = c + kR;
      const float d = sh.in[0][ly][lx] - sh.in[1][ly][lx];
      part += (double)(1.f - lambda) * fabs((double)d) - (double)lambda * (double)S;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[b] = ((sh.red[0] + sh.red[1]) + (sh.red[2] + sh.red[3])) * (double)inv_count;
  }
}

// One workgroup adds the per-tile partials (fixed order per thread, then a
// tree), plus lambda for the constant of 1 - SSIM, into *loss.
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ partial,
                                                       size_t nb, float lambda,
                                                       double* __restrict__ loss) {
  __shared__ double s[16];
  // eight independent sums per thread (fixed order, eight loads in flight)
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  size_t i = threadIdx.x;
  for (; i + 7 * 1024 < nb; i += 8 * 1024) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += partial[i + u * 1024];
  }
  for (int u = 0; i < nb; i += 1024, ++u) a[u] += partial[i];
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += s[w];
    atomicAdd(loss, t + (double)lambda);
  }
}

struct GradShared {
  float in[3][kI][kIP];
  float h[3][kI][kTP];
};

__global__ __launch_bounds__(256) void k_ssim_grad(const float* __restrict__ img,
                                                  const float* __restrict__ tgt, int W, int H,
                                                  Window win, float lambda, float inv_count,
                                                  const float* __restrict__ amaps,
                                                  float* __restrict__ grad) {
  __shared__ GradShared sh;
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z;
  const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
  const float* a = amaps + (size_t)pl * 3 * plane;
  const float* srcs[3] = {a, a + plane, a + 2 * plane};
  stage<3>(sh.in, srcs, W, H, x0, y0);
  __syncthreads();
  hpass<3, 3>(sh.in, sh.h, win, [](const float* v, float* st) {
    st[0] = v[0];
    st[1] = v[1];
    st[2] = v[2];
  });
  __syncthreads();
  const int c = threadIdx.x % kT, g = threadIdx.x / kT;
  float res[kRows][3];
  vpass<3>(sh.h, win, c, g, res);
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int x = x0 + c, y = y0 + kRows * g + o;
    if (x < W && y < H) {
      const size_t p = (size_t)pl * plane + (size_t)y * W + x;
      const float xv = img[p], yv = tgt[p];
      const float d = xv - yv;
      const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      const float gs = res[o][0] + 2.f * xv * res[o][1] + yv * res[o][2];
      grad[p] = ((1.f - lambda) * sg - lambda * gs) * inv_count;
    }
  }
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

inline size_t tiles_of(int planes, int H, int W) {
  return (size_t)planes * (size_t)((H + kT - 1) / kT) * (size_t)((W + kT - 1) / kT);
}

size_t l1_dssim_workspace_bytes(int planes, int H, int W) {
  return (size_t)planes * 3 * (size_t)H * (size_t)W * sizeof(float) +
         tiles_of(planes, H, W) * sizeof(double);
}

void launch_l1_dssim(const float* image, const float* target, int planes, int H, int W,
                     float lambda, float* grad, double* loss, void* ws, hipStream_t s) {
  if (planes <= 0 || H <= 0 || W <= 0) return;
  const Window win = make_window();
  const double count = (double)planes * (double)H * (double)W;
  const float inv = (float)(1.0 / count);
  const dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT, planes);
  float* amaps = static_cast<float*>(ws);
  double* partial =
      reinterpret_cast<double*>(static_cast<char*>(ws) + (size_t)planes * 3 * H * W * sizeof(float));
  StageScope scope(kStDssim, s);
  hipLaunchKernelGGL(k_ssim_stats, grid, dim3(256), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, (const double*)partial,
                     tiles_of(planes, H, W), lambda, loss);
  hipLaunchKernelGGL(k_ssim_grad, grid, dim3(256), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, grad);
}

}  // namespace gs
