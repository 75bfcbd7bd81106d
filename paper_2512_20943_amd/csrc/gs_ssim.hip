// Photometric loss of AirGS Eq. (1): (1 - lambda) L1 + lambda (1 - SSIM),
// with SSIM over an 11x11 Gaussian window (sigma 1.5), zero padding,
// C1 = 0.01^2, C2 = 0.03^2, averaged over every image value.
//
// Two streaming passes.  A workgroup owns a strip of kSW output columns (one
// per thread) and a band of kBand output rows; it walks the band's input
// rows top to bottom, staging each row of the strip plus its kR-column
// margins in LDS (two row buffers, the next row's loads in flight while the
// current one is summed), takes each thread's horizontal 11-tap sums, and
// keeps the last 11 rows of those sums in registers, so that every row
// after the first 2 kR yields one output row of vertical sums:
//   1. windowed statistics of x, y, x^2, y^2, xy -> per-pixel SSIM index and
//      the partials A1 = dS/dmu_x - 2 mu_x dS/dvar_x - mu_y dS/dcov,
//      A2 = dS/dvar_x, A3 = dS/dcov (written to the workspace), one loss
//      partial per workgroup (summed by one workgroup afterwards);
//   2. the adjoint window over A1..A3 -> dL/dx = ((1 - lambda) sign(x - y)
//      - lambda (w*A1 + 2 x w*A2 + y w*A3)) / count.
// HBM-bound: 8 B read + 12 B written per value in pass 1, 20 B read + 4 B
// written in pass 2 (plus the margins: (kSW + 2 kR) / kSW columns and
// (kBand + 2 kR) / kBand rows of input).
#include <cmath>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kR = 5;               // window radius
constexpr int kTaps = 2 * kR + 1;
constexpr int kSW = 128;            // strip width: output columns, one per thread
constexpr int kBand = 64;           // output rows per workgroup
constexpr int kSI = kSW + 2 * kR;   // staged columns of one input row
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
  float w[kTaps];
};

// One input row of the strip in registers: column x0 - kR + t, and for
// t < 2 kR also column x0 - kR + kSW + t; zero outside the image.
template <int NP>
struct RowRegs {
  float a[NP], b[NP];
};

template <int NP>
__device__ __forceinline__ void load_row(RowRegs<NP>& r, const float* const* src, int W, int H,
                                         int x0, int y) {
  const int t = threadIdx.x;
  const int xa = x0 - kR + t, xb = xa + kSW;
  const bool row_in = y >= 0 && y < H;
  const size_t base = (size_t)(row_in ? y : 0) * (size_t)W;
  const bool a_in = row_in && xa >= 0 && xa < W;
  const bool b_in = row_in && t < 2 * kR && xb < W;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    r.a[q] = a_in ? src[q][base + xa] : 0.f;
    r.b[q] = b_in ? src[q][base + xb] : 0.f;
  }
}

template <int NP>
__device__ __forceinline__ void store_row(float (*buf)[kSI], const RowRegs<NP>& r) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    buf[q][t] = r.a[q];
    if (t < 2 * kR) buf[q][kSW + t] = r.b[q];
  }
}

// The band walk shared by both passes.  For input row i of the band
// (image row y0 - kR + i), Horiz(in, hs) forms the thread's NS horizontal
// sums from the staged row (in[q][t + k], k = 0 .. 2 kR, is tap k of plane
// q); once 2 kR + 1 rows are in, Out(y, vs) receives the vertical sums of
// output row y = y0 + i - 2 kR.  Centre(i, in) sees every staged row, and
// Ahead(i) runs right after the loads of row i + 1 are issued, so that the
// caller can issue its own loads for the next output row with them.  The
// next row's loads are in flight while a row is summed; the ring slot of
// row i is i mod 11, and the rows are unrolled by 11 so that every slot
// index is static.
template <int NP, int NS, typename Horiz, typename Out, typename Centre, typename Ahead>
__device__ __forceinline__ void walk_band(const float* const* src, int W, int H, int x0, int y0,
                                          const Window& win, float (*buf)[NP][kSI], Horiz horiz,
                                          Out out, Centre centre, Ahead ahead) {
  const int rows = min(kBand, H - y0) + 2 * kR;  // same for the whole workgroup
  float ring[kTaps][NS];
  RowRegs<NP> nx;
  load_row<NP>(nx, src, W, H, x0, y0 - kR);
  store_row<NP>(buf[0], nx);
  __syncthreads();
  for (int i0 = 0; i0 < rows; i0 += kTaps) {
#pragma unroll
    for (int u = 0; u < kTaps; ++u) {
      const int i = i0 + u;
      if (i < rows) {
        // the next row's loads go out before this row is summed
        if (i + 1 < rows) load_row<NP>(nx, src, W, H, x0, y0 - kR + i + 1);
        ahead(i);
        const float (*in)[kSI] = buf[i & 1];
        horiz(in, ring[u]);
        centre(i, in);
        if (i >= 2 * kR) {
          float vs[NS];
#pragma unroll
          for (int q = 0; q < NS; ++q) vs[q] = 0.f;
#pragma unroll
          for (int k = 0; k < kTaps; ++k) {
            // row i - 2 kR + k sits in slot (u + 1 + k) mod 11
#pragma unroll
            for (int q = 0; q < NS; ++q)
              vs[q] = fmaf(win.w[k], ring[(u + 1 + k) % kTaps][q], vs[q]);
          }
          out(y0 + i - 2 * kR, vs);
        }
        if (i + 1 < rows) store_row<NP>(buf[(i + 1) & 1], nx);
        __syncthreads();
      }
    }
  }
}

__global__ __launch_bounds__(kSW) void k_ssim_stats(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int W, int H,
                                                   Window win, float lambda, float inv_count,
                                                   float* __restrict__ amaps,
                                                   double* __restrict__ partial) {
  __shared__ float buf[2][2][kSI];
  __shared__ double red[kSW / 64];
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z, t = threadIdx.x;
  const int x0 = blockIdx.x * kSW, y0 = blockIdx.y * kBand;
  const int x = x0 + t;
  const float* srcs[2] = {img + pl * plane, tgt + pl * plane};
  float* a = amaps + (size_t)pl * 3 * plane;
  double part = 0.0;
  const int rows = min(kBand, H - y0) + 2 * kR;
  walk_band<2, 5>(
      srcs, W, H, x0, y0, win, buf,
      [&](const float (*in)[kSI], float* hs) {
#pragma unroll
        for (int q = 0; q < 5; ++q) hs[q] = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) {
          // the weighted values once, then each sum one instruction: seven
          // per tap instead of three products and five multiply-adds
          const float xv = in[0][t + k], yv = in[1][t + k], w = win.w[k];
          const float wx = w * xv, wy = w * yv;
          hs[0] += wx;
          hs[1] += wy;
          hs[2] = fmaf(wx, xv, hs[2]);
          hs[3] = fmaf(wy, yv, hs[3]);
          hs[4] = fmaf(wx, yv, hs[4]);
        }
      },
      [&](int y, const float* st) {
        if (x >= W) return;
        const float mx = st[0], my = st[1];
        const float sxx = st[2] - mx * mx, syy = st[3] - my * my, sxy = st[4] - mx * my;
        const float N1 = 2.f * mx * my + kC1, N2 = 2.f * sxy + kC2;
        const float D1 = mx * mx + my * my + kC1, D2 = sxx + syy + kC2;
        // hardware reciprocals (1 ulp); D1 and D2 are at least C1 and C2
        const float iD1 = __builtin_amdgcn_rcpf(D1), iD2 = __builtin_amdgcn_rcpf(D2);
        const float iD = iD1 * iD2;
        const float S = N1 * N2 * iD;
        const float dS_dmx = 2.f * my * N2 * iD - S * 2.f * mx * iD1;
        const float dS_dsxx = -S * iD2;
        const float dS_dsxy = 2.f * N1 * iD;
        const size_t p = (size_t)y * W + x;
        a[p] = dS_dmx - 2.f * mx * dS_dsxx - my * dS_dsxy;
        a[plane + p] = dS_dsxx;
        a[2 * plane + p] = dS_dsxy;
        part -= (double)lambda * (double)S;
      },
      [&](int i, const float (*in)[kSI]) {
        // the L1 term of the band's own rows
        if (i >= kR && i < rows - kR && x < W)
          part += (double)(1.f - lambda) * fabs((double)(in[0][t + kR] - in[1][t + kR]));
      },
      [](int) {});
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((t & 63) == 0) red[t >> 6] = part;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSW / 64; ++w) s += red[w];
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[b] = s * (double)inv_count;
  }
}

// One workgroup adds the per-workgroup partials (fixed order per thread,
// then a tree), plus lambda for the constant of 1 - SSIM, into *loss.
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

__global__ __launch_bounds__(kSW) void k_ssim_grad(const float* __restrict__ img,
                                                  const float* __restrict__ tgt, int W, int H,
                                                  Window win, float lambda, float inv_count,
                                                  const float* __restrict__ amaps,
                                                  float* __restrict__ grad) {
  __shared__ float buf[2][3][kSI];
  const size_t plane = (size_t)W * H;
  const int pl = blockIdx.z, t = threadIdx.x;
  const int x0 = blockIdx.x * kSW, y0 = blockIdx.y * kBand;
  const int x = x0 + t;
  const float* a = amaps + (size_t)pl * 3 * plane;
  const float* srcs[3] = {a, a + plane, a + 2 * plane};
  const int rows = min(kBand, H - y0) + 2 * kR;
  // x and y at this thread's pixel of the next output row, loaded a row
  // ahead of their use
  float xa = 0.f, ya = 0.f, xc = 0.f, yc = 0.f;
  walk_band<3, 3>(
      srcs, W, H, x0, y0, win, buf,
      [&](const float (*in)[kSI], float* hs) {
#pragma unroll
        for (int q = 0; q < 3; ++q) hs[q] = 0.f;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) {
          const float w = win.w[k];
#pragma unroll
          for (int q = 0; q < 3; ++q) hs[q] = fmaf(w, in[q][t + k], hs[q]);
        }
      },
      [&](int y, const float* r) {
        const float xv = xc, yv = yc;
        if (x >= W) return;
        const size_t p = (size_t)pl * plane + (size_t)y * W + x;
        const float d = xv - yv;
        const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        const float gs = r[0] + 2.f * xv * r[1] + yv * r[2];
        grad[p] = ((1.f - lambda) * sg - lambda * gs) * inv_count;
      },
      [](int, const float (*)[kSI]) {},
      [&](int i) {
        // the pixel of output row y0 + i - 2 kR was loaded last round; row
        // i + 1 (if it yields output) is loaded now
        xc = xa;
        yc = ya;
        if (i + 1 >= 2 * kR && i + 1 < rows && x < W) {
          const size_t p = (size_t)pl * plane + (size_t)(y0 + i + 1 - 2 * kR) * W + x;
          xa = img[p];
          ya = tgt[p];
        }
      });
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
  return (size_t)planes * (size_t)((H + kBand - 1) / kBand) * (size_t)((W + kSW - 1) / kSW);
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
  const dim3 grid((W + kSW - 1) / kSW, (H + kBand - 1) / kBand, planes);
  float* amaps = static_cast<float*>(ws);
  double* partial =
      reinterpret_cast<double*>(static_cast<char*>(ws) + (size_t)planes * 3 * H * W * sizeof(float));
  StageScope scope(kStDssim, s);
  hipLaunchKernelGGL(k_ssim_stats, grid, dim3(kSW), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, (const double*)partial,
                     tiles_of(planes, H, W), lambda, loss);
  hipLaunchKernelGGL(k_ssim_grad, grid, dim3(kSW), 0, s, image, target, W, H, win, lambda, inv,
                     amaps, grad);
}

}  // namespace gs
