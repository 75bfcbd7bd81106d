// Tile compositing: forward and backward (the splatting renderer AirGS cites
// in Sec. II; every training view and every delivered view runs it).
//
// One 256-thread workgroup per 16x16 tile; wave w (of 4) owns the 8x8
// quadrant (w & 1, w >> 1), so the 64 lanes of a wave are a compact pixel
// block.  The tile's instance list is walked in batches of 256 records
// gathered into LDS.  While staging a record, its loader thread also tests
// the Gaussian's alpha >= 1/255 ellipse against each quadrant's pixel box
// (with a conservative margin): a wave skips, uniformly, every record whose
// ellipse misses its quadrant, which is exact because every such pair would
// be skipped per pixel anyway.  Transmittance saturation ends a wave with a
// ballot and the block with a barrier count.
//
// The backward walks each pixel's list back to front from its last
// contributor, recovering T_k = T_{k+1} / (1 - alpha_k); alpha is recomputed
// by the same device function as in the forward, so every skip and stop
// decision is bit-identical.  Per-pair gradients are summed across the wave
// with DPP row shifts and row broadcasts, across the 4 waves in LDS, and
// leave the workgroup as one set of global float atomics per (tile,
// Gaussian).
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kBlock = 256;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn255 = 5.541263545158426f;

// Screen-space record as staged in LDS:
//   a = (px, py, nA, r1), b = (n2, log2 opacity, r, g), c = (b, A, B, C)
// with power = nA (dx + r1 dy)^2 + n2 dy^2, nA = -A/2, r1 = B/A,
// n2 = -(AC - B^2) / (2A): the conic quadratic form written as a sum of two
// non-positive squares, so FP32 evaluation has no cancellation.
struct Rec {
  float4 a, b, c;
};

__device__ __forceinline__ Rec make_rec(float4 s0, float4 s1, float4 s2) {
  // s0 = (px, py, A, B), s1 = (C, opacity, r, g), s2 = (b, depth, detQ, 0)
  Rec r;
  const float A = s0.z, B = s0.w, C = s1.x, dq = s2.z;
  const float iA = 1.f / A;
  r.a = make_float4(s0.x, s0.y, -0.5f * A, B * iA);
  r.b = make_float4(-0.5f * dq * iA, __log2f(s1.y), s1.z, s1.w);
  r.c = make_float4(s2.x, A, B, C);
  return r;
}

__device__ __forceinline__ float eval_power(const float4& a, float n2, float dx, float dy) {
  const float t = fmaf(a.w, dy, dx);
  return fmaf(a.z * t, t, n2 * (dy * dy));
}

// ea = opacity * exp(power) evaluated as exp2(power log2e + log2 opacity).
__device__ __forceinline__ float eval_ea(float power, float l2o) {
  return __builtin_amdgcn_exp2f(fmaf(power, kLog2e, l2o));
}

// Minimum over the box [u0,u1] x [v0,v1] of q(u,v) = A u^2 + 2B uv + C v^2,
// written as A (u + r1 v)^2 + (detQ/A) v^2 = C (v + r2 u)^2 + (detQ/C) u^2.
__device__ __forceinline__ float box_min_q(float A, float C, float r1, float r2, float dA,
                                           float dC, float u0, float u1, float v0, float v1) {
  if (u0 <= 0.f && u1 >= 0.f && v0 <= 0.f && v1 >= 0.f) return 0.f;
  float m = 3.0e38f;
  {
    const float u = u0, v = fminf(fmaxf(-r2 * u, v0), v1), t = v + r2 * u;
    m = fminf(m, C * t * t + dC * u * u);
  }
  {
    const float u = u1, v = fminf(fmaxf(-r2 * u, v0), v1), t = v + r2 * u;
    m = fminf(m, C * t * t + dC * u * u);
  }
  {
    const float v = v0, u = fminf(fmaxf(-r1 * v, u0), u1), t = u + r1 * v;
    m = fminf(m, A * t * t + dA * v * v);
  }
  {
    const float v = v1, u = fminf(fmaxf(-r1 * v, u0), u1), t = u + r1 * v;
    m = fminf(m, A * t * t + dA * v * v);
  }
  return m;
}

// Bit w set when some pixel of quadrant w could reach alpha >= 1/255.
__device__ __forceinline__ uint32_t quadrant_mask(float4 s0, float4 s1, float4 s2, float ox,
                                                  float oy) {
  const float A = s0.z, B = s0.w, C = s1.x, dq = s2.z, op = s1.y;
  // alpha >= 1/255  <=>  q <= 2 ln(255 opacity)
  const float qmax = 2.f * (kLn255 + __logf(op));
  const float thr = qmax + 2e-4f * fabsf(qmax) + 1e-3f;
  if (!(thr > 0.f)) return 0u;
  const float r1 = B / A, r2 = B / C, dA = dq / A, dC = dq / C;
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float u0 = ox + (float)((w & 1) * 8) - s0.x;
    const float v0 = oy + (float)((w >> 1) * 8) - s0.y;
    if (box_min_q(A, C, r1, r2, dA, dC, u0, u0 + 7.f, v0, v0 + 7.f) <= thr) m |= 1u << w;
  }
  return m;
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float dpp_take(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, BOUND));
}

// Sum over the 64 lanes, valid in lane 63.  Must be called with all lanes
// active.
__device__ __forceinline__ float wave_sum_lane63(float v) {
  v += dpp_take<0x111, 0xF, true>(v);  // row_shr:1
  v += dpp_take<0x112, 0xF, true>(v);  // row_shr:2
  v += dpp_take<0x114, 0xF, true>(v);  // row_shr:4
  v += dpp_take<0x118, 0xF, true>(v);  // row_shr:8
  v += dpp_take<0x142, 0xA, false>(v); // row_bcast:15 into rows 1, 3
  v += dpp_take<0x143, 0xC, false>(v); // row_bcast:31 into rows 2, 3
  return v;
}

__global__ __launch_bounds__(kBlock) void k_render_fwd(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib) {
  __shared__ float4 s_a[kBlock];
  __shared__ float4 s_b[kBlock];
  __shared__ float s_c[kBlock];
  __shared__ uint32_t s_m[kBlock];

  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int y = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = x < W && y < H;
  const float fx = (float)x, fy = (float)y;
  const uint2 rg = ranges[seg];
  const float4* sv = splat + 3 * (size_t)v * ld;

  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  int last = 0;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const uint32_t e = b0 + threadIdx.x;
    if (e < rg.y) {
      const uint32_t g = vals[e];
      const float4 q0 = sv[3 * (size_t)g], q1 = sv[3 * (size_t)g + 1], q2 = sv[3 * (size_t)g + 2];
      const Rec r = make_rec(q0, q1, q2);
      s_a[threadIdx.x] = r.a;
      s_b[threadIdx.x] = r.b;
      s_c[threadIdx.x] = r.c.x;
      s_m[threadIdx.x] = quadrant_mask(q0, q1, q2, (float)(tx * kTile), (float)(ty * kTile));
    }
    __syncthreads();
    const int nb = (int)((rg.y - b0) < (uint32_t)kBlock ? (rg.y - b0) : (uint32_t)kBlock);
    if (__builtin_amdgcn_ballot_w64(!done) == 0) continue;
    for (int k = 0; k < nb; ++k) {
      const uint32_t m = __builtin_amdgcn_readfirstlane(s_m[k]);
      if (!((m >> wave) & 1u)) continue;
      if (!done) {
        const float4 a = s_a[k];
        const float4 b = s_b[k];
        const float dx = a.x - fx, dy = a.y - fy;
        const float power = eval_power(a, b.x, dx, dy);
        if (!(power > 0.f)) {
          const float alpha = fminf(kAlphaMax, eval_ea(power, b.y));
          if (alpha >= kAlphaMin) {
            const float Tn = T * (1.f - alpha);
            if (Tn < kTStop) {
              done = true;
            } else {
              const float w = alpha * T;
              c0 = fmaf(b.z, w, c0);
              c1 = fmaf(b.w, w, c1);
              c2 = fmaf(s_c[k], w, c2);
              T = Tn;
              last = (int)(b0 - rg.x) + k + 1;
            }
          }
        }
      }
      if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    }
  }
  if (inside) {
    const size_t pix = (size_t)W * H, p = (size_t)y * W + x;
    float* im = image + 3 * pix * v;
    im[p] = c0 + T * bg0;
    im[pix + p] = c1 + T * bg1;
    im[2 * pix + p] = c2 + T * bg2;
    final_T[pix * v + p] = T;
    n_contrib[pix * v + p] = last;
  }
}

__global__ __launch_bounds__(kBlock) void k_render_bwd(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, const float* __restrict__ final_T, const int32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, float* __restrict__ grad2d) {
  __shared__ float4 s_a[kBlock];
  __shared__ float4 s_b[kBlock];
  __shared__ float4 s_c[kBlock];
  __shared__ uint32_t s_m[kBlock];
  __shared__ uint32_t s_g[kBlock];
  __shared__ float s_acc[kBlock][9];
  __shared__ int s_max[4];

  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int y = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = x < W && y < H;
  const float fx = (float)x, fy = (float)y;
  const uint2 rg = ranges[seg];
  const float4* sv = splat + 3 * (size_t)v * ld;
  const size_t pix = (size_t)W * H, p = (size_t)y * W + x;

  float T = 1.f, gI0 = 0.f, gI1 = 0.f, gI2 = 0.f;
  int nc = 0;
  if (inside) {
    T = final_T[pix * v + p];
    nc = n_contrib[pix * v + p];
    const float* gi = dL_dimage + 3 * pix * v;
    gI0 = gi[p];
    gI1 = gi[pix + p];
    gI2 = gi[2 * pix + p];
  }
  // longest walk in the wave and in the block
  int wmax = nc;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off, 64));
  if (lane == 0) s_max[wave] = wmax;
  __syncthreads();
  const int bmax = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
  float B0 = bg0, B1 = bg1, B2 = bg2;  // colour behind the current entry

  for (int hi = bmax; hi > 0; hi -= kBlock) {
    const int lo = hi > kBlock ? hi - kBlock : 0;
    __syncthreads();
    {
      const int k = (int)threadIdx.x;
      if (lo + k < hi) {
        const uint32_t g = vals[rg.x + (uint32_t)(lo + k)];
        const float4 q0 = sv[3 * (size_t)g], q1 = sv[3 * (size_t)g + 1], q2 = sv[3 * (size_t)g + 2];
        const Rec r = make_rec(q0, q1, q2);
        s_a[k] = r.a;
        s_b[k] = r.b;
        s_c[k] = r.c;
        s_g[k] = g;
        s_m[k] = quadrant_mask(q0, q1, q2, (float)(tx * kTile), (float)(ty * kTile));
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) s_acc[k][c] = 0.f;
    }
    __syncthreads();
    for (int k = hi - lo - 1; k >= 0; --k) {
      const int j = lo + k;  // position in the tile list
      if (j >= wmax) continue;
      const uint32_t m = __builtin_amdgcn_readfirstlane(s_m[k]);
      if (!((m >> wave) & 1u)) continue;
      float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bool contrib = false;
      if (j < nc) {
        const float4 a = s_a[k];
        const float4 b = s_b[k];
        const float dx = a.x - fx, dy = a.y - fy;
        const float power = eval_power(a, b.x, dx, dy);
        if (!(power > 0.f)) {
          const float ea = eval_ea(power, b.y);
          const float alpha = fminf(kAlphaMax, ea);
          if (alpha >= kAlphaMin) {
            contrib = true;
            const float4 c = s_c[k];
            T = __fdividef(T, 1.f - alpha);
            const float w = alpha * T;
            g[6] = gI0 * w;
            g[7] = gI1 * w;
            g[8] = gI2 * w;
            const float da = T * (gI0 * (b.z - B0) + gI1 * (b.w - B1) + gI2 * (c.x - B2));
            if (ea < kAlphaMax) {
              const float gp = da * alpha;
              g[5] = da * __builtin_amdgcn_exp2f(power * kLog2e);
              g[0] = -gp * (c.y * dx + c.z * dy);
              g[1] = -gp * (c.z * dx + c.w * dy);
              g[2] = -0.5f * gp * dx * dx;
              g[3] = -gp * dx * dy;
              g[4] = -0.5f * gp * dy * dy;
            }
            B0 = alpha * b.z + (1.f - alpha) * B0;
            B1 = alpha * b.w + (1.f - alpha) * B1;
            B2 = alpha * c.x + (1.f - alpha) * B2;
          }
        }
      }
      if (__builtin_amdgcn_ballot_w64(contrib) == 0) continue;
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float s = wave_sum_lane63(g[c]);
        if (lane == 63 && s != 0.f) atomicAdd(&s_acc[k][c], s);
      }
    }
    __syncthreads();
    {
      const int k = (int)threadIdx.x;
      if (lo + k < hi) {
        float* dst = grad2d + ((size_t)v * ld + s_g[k]) * kGrad2dFloats;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const float s = s_acc[k][c];
          if (s != 0.f) atomicAdd(dst + c, s);
        }
      }
    }
  }
}

}  // namespace

void launch_render_fwd(const gs_projected& proj, const gs_tile_lists& lists, int V, int W, int H,
                       const float bg[3], float* image, float* final_T, int32_t* n_contrib,
                       hipStream_t s) {
  const int TX = tiles_across(W), TY = tiles_across(H);
  const int tpv = TX * TY;
  const int blocks = tpv * V;
  if (blocks == 0) return;
  StageScope scope(kStRenderFwd, s);
  hipLaunchKernelGGL(k_render_fwd, dim3(blocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                     reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                     bg[2], image, final_T, n_contrib);
}

void launch_render_bwd(const gs_projected& proj, const gs_tile_lists& lists, int V, int W, int H,
                       const float bg[3], const float* final_T, const int32_t* n_contrib,
                       const float* dL_dimage, float* grad2d, hipStream_t s) {
  const int TX = tiles_across(W), TY = tiles_across(H);
  const int tpv = TX * TY;
  const int blocks = tpv * V;
  if (blocks == 0) return;
  StageScope scope(kStRenderBwd, s);
  hipLaunchKernelGGL(k_render_bwd, dim3(blocks), dim3(kBlock), 0, s,
                     reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                     reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                     bg[2], final_T, n_contrib, dL_dimage, grad2d);
}

}  // namespace gs
