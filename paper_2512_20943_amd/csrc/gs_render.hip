// Tile compositing: forward and backward (the splatting renderer AirGS cites
// in Sec. II; every training view and every delivered view runs it).
//
// One 64-lane wave (one workgroup) per 16x16 tile.  Lane l owns pixel
// (l & 7, l >> 3) of each of the tile's four 8x8 quadrants ("slots"), so a
// slot is a compact 64-pixel block.  The tile's instance list is walked in
// batches staged in LDS (the forward one record per lane, the backward one
// per two lanes).  While staging a record, its lane also tests the
// Gaussian's alpha >= 1/255 ellipse against each quadrant's pixel box (exact
// box minimum of the quadratic form, with a conservative margin); the
// results are kept as one wave ballot per quadrant, and the wave walks the
// set bits, skipping, uniformly, every slot whose quadrant the ellipse
// misses, which is exact because every such pair would be skipped per pixel
// anyway.  A slot whose 64 pixels have all stopped is dropped with a ballot;
// the tile ends when all four have.
//
// The backward walks each pixel's list back to front from its last
// contributor, recovering T_k = T_{k+1} / (1 - alpha_k); alpha is recomputed
// by the same device functions as in the forward, so every skip and stop
// decision is bit-identical.  Per entry it accumulates, per lane, the colour
// gradients and five moments of dL/dpower in the exponent's coordinates (the
// mean and conic gradients are linear in them with per-entry coefficients),
// sums the nine values over each 16-lane row with DPP exchanges that leave
// one row sum per lane (22 instructions, one LDS store), adds the four row
// sums when the batch is flushed, and writes one 9-float gradient row per
// (tile, Gaussian) at the instance's index in the binning's emission order.
// A second kernel sums
// each (view, Gaussian)'s rows, which that order keeps contiguous: no
// floating-point atomics, and the result does not depend on scheduling.
#include "gs_internal.h"

namespace gs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn255 = 5.541263545158426f;

// Screen-space record as staged in LDS:
//   a = (px, py, nA, r1), b = (n2, log2 opacity, r, g), c = (b, 1/opacity, B, C)
// with power log2(e) = nA (dx + r1 dy)^2 + n2 dy^2, nA = -log2(e) A/2,
// r1 = B/A, n2 = -log2(e) (AC - B^2) / (2A): the conic quadratic form written
// as a sum of two non-positive squares (A > 0 and AC - B^2 > 0 for every
// projected conic), in base-2 units, so FP32 evaluation has no cancellation
// and never exceeds 0.
struct Rec {
  float4 a, b, c;
};

__device__ __forceinline__ Rec make_rec(float4 s0, float4 s1, float4 s2) {
  // s0 = (px, py, A, B), s1 = (C, opacity, r, g), s2 = (b, depth, detQ, 0)
  Rec r;
  const float A = s0.z, B = s0.w, C = s1.x, dq = s2.z;
  const float iA = __builtin_amdgcn_rcpf(A);  // hardware reciprocal (1 ulp)
  r.a = make_float4(s0.x, s0.y, (-0.5f * kLog2e) * A, B * iA);
  r.b = make_float4((-0.5f * kLog2e) * dq * iA, __log2f(s1.y), s1.z, s1.w);
  r.c = make_float4(s2.x, __builtin_amdgcn_rcpf(s1.y), B, C);
  return r;
}

// ea = opacity * exp(power) = exp2(nA (dx + r1 dy)^2 + q), where
// q = n2 dy^2 + log2(opacity) depends on the pixel row only.  Both squares
// carry non-positive coefficients, so the exponent never exceeds
// log2(opacity): power > 0 cannot occur in this form and is not tested.
__device__ __forceinline__ float row_q(const float4& b, float dy) {
  return fmaf(b.x, dy * dy, b.y);
}

__device__ __forceinline__ float eval_ea(const float4& a, float q, float dx, float dy) {
  const float t = fmaf(a.w, dy, dx);
  return __builtin_amdgcn_exp2f(fmaf(a.z * t, t, q));
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
  // hardware reciprocals: their error is far inside the threshold's margin
  const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
  const float r1 = B * iA, r2 = B * iC, dA = dq * iA, dC = dq * iC;
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float u0 = ox + (float)((w & 1) * 8) - s0.x;
    const float v0 = oy + (float)((w >> 1) * 8) - s0.y;
    if (box_min_q(A, C, r1, r2, dA, dC, u0, u0 + 7.f, v0, v0 + 7.f) <= thr) m |= 1u << w;
  }
  return m;
}

// Bits 0 and 1 set when some pixel of the quadrant at (ox, oyq), resp.
// (ox + 8, oyq), could reach alpha >= 1/255: the quadrant_mask test for one
// row of quadrants (oyq = oy or oy + 8).
__device__ __forceinline__ uint32_t quadrant_row_mask(float4 s0, float4 s1, float4 s2, float ox,
                                                      float oyq) {
  const float A = s0.z, B = s0.w, C = s1.x, dq = s2.z, op = s1.y;
  const float qmax = 2.f * (kLn255 + __logf(op));
  const float thr = qmax + 2e-4f * fabsf(qmax) + 1e-3f;
  if (!(thr > 0.f)) return 0u;
  const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
  const float r1 = B * iA, r2 = B * iC, dA = dq * iA, dC = dq * iC;
  const float v0 = oyq - s0.y;
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const float u0 = ox + (float)(w * 8) - s0.x;
    if (box_min_q(A, C, r1, r2, dA, dC, u0, u0 + 7.f, v0, v0 + 7.f) <= thr) m |= 1u << w;
  }
  return m;
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float dpp_take(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, BOUND));
}

// Row sums of nine values, scattered over the row: each step pairs every lane
// with one in the other half of its group (row mirror, half-row mirror, then
// quad swaps by 2 and by 1); the lower half keeps one value of each pair and
// the upper half the other, so a step halves the values a lane carries.
// Afterwards, with b_k bit k of (lane & 15), a lane holds its row's sum of
// value 4 b1 + 2 b2 + b3 when b0 = 0, and of value 8 when b0 = 1.  Must be
// called with all lanes active; u_k = (lane & (1 << k)) != 0.
constexpr int kDppMirror = 0x140, kDppHalfMirror = 0x141, kDppSwap2 = 0x4E, kDppSwap1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float pair_step(float lo, float hi, bool upper) {
  const float keep = upper ? hi : lo, send = upper ? lo : hi;
  return keep + dpp_take<CTRL, 0xF, true>(send);
}

template <int CTRL>
__device__ __forceinline__ float single_step(float v) {
  return v + dpp_take<CTRL, 0xF, true>(v);
}

// pair_step for the two steps whose halves are whole DPP banks (four-lane
// groups): every lane first adds hi across the pair, then the lanes of the
// lower half (bank mask) overwrite that with the sum of lo while the others
// keep it; two instructions per pair instead of two selects and an add.  The
// wait states before and after cover a DPP read of a register a vector
// instruction has just written (lo here, the results in the next step).
__device__ __forceinline__ void pair_steps_mirror(const float (&x)[9], float (&y)[5]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = single_step<kDppMirror>(x[2 * i + 1]);
  y[4] = single_step<kDppMirror>(x[8]);
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %4, %4 row_mirror row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %1, %5, %5 row_mirror row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %2, %6, %6 row_mirror row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %3, %7, %7 row_mirror row_mask:0xf bank_mask:0x3\n\t"
      "s_nop 1"
      : "+v"(y[0]), "+v"(y[1]), "+v"(y[2]), "+v"(y[3])
      : "v"(x[0]), "v"(x[2]), "v"(x[4]), "v"(x[6]));
}

__device__ __forceinline__ void pair_steps_half_mirror(const float (&y)[5], float (&z)[3]) {
  z[0] = single_step<kDppHalfMirror>(y[1]);
  z[1] = single_step<kDppHalfMirror>(y[3]);
  z[2] = single_step<kDppHalfMirror>(y[4]);
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "v_add_f32_dpp %1, %3, %3 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "s_nop 1"
      : "+v"(z[0]), "+v"(z[1])
      : "v"(y[0]), "v"(y[2]));
}

__device__ __forceinline__ float row_sums9(const float (&x)[9], bool u1, bool u0) {
  // lanes 0-7 of a row are the lower half of the mirror step (banks 0, 1),
  // lanes 0-3 and 8-11 that of the half-row mirror step (banks 0, 2)
  float y[5], z[3];
  pair_steps_mirror(x, y);
  pair_steps_half_mirror(y, z);
  const float w0 = pair_step<kDppSwap2>(z[0], z[1], u1), w1 = single_step<kDppSwap2>(z[2]);
  return pair_step<kDppSwap1>(w0, w1, u0);
}

// ---------------------------------------------------------------- forward
// One 64-lane wave per 16x16 tile.  Lane l owns pixel (l & 7, l >> 3) of
// each of the four 8x8 quadrants ("slot" w = quadrant w), so a record's
// quadrant mask selects slots uniformly across the wave.
constexpr int kFwdBatch = 64;   // records staged per batch (1 per lane)
// records staged per backward batch (at most 32, two lanes per record): 30
// ran 1-2 % faster than 32 on the 20-view frame, 28 about as fast as 30,
// 24 as fast as 32 and 20 slower
constexpr int kBwdBatch = 30;
static_assert(kBwdBatch <= 32, "the backward stages one batch with two lanes per entry");

// c holds the record's blue in .x only: a float4 stride puts it at the
// same offset from a[k] as b[k], so one address register serves all three
struct FwdShared {
  float4 a[kFwdBatch];
  float4 b[kFwdBatch];
  float4 c[kFwdBatch];
};
static_assert(kFwdBatch == 64, "the forward stages one record per lane");

// Extra staging for per-Gaussian usage counts (composited pixels).
struct UsageShared {
  uint32_t g[kFwdBatch];
  uint32_t u[kFwdBatch];
};

// Bit w set while some pixel of slot w still composites (T > 0).
// One pixel slot of the forward: transmittance (its sign is the "still
// compositing" flag), colour sums and the last composited list position.
// Each slot is its own variable, not an element of an array: indexing an
// array by the unrolled slot number lets the compiler keep the four slots
// in one vector register tuple, whose merge points cost register copies on
// every list entry.
struct FwdSlot {
  float T, c0, c1, c2;
  int last;
};

template <int W>
using SlotId = std::integral_constant<int, W>;

__device__ __forceinline__ uint32_t live_bit(const FwdSlot& s, int w) {
  return __builtin_amdgcn_ballot_w64(s.T > 0.f) != 0 ? 1u << w : 0u;
}

// The L1 term of Eq. (1) evaluated where the forward writes its pixels:
// target and grad point at the view's (3, H, W) planes, partial at the
// tile's slot for the sum of |image - target| over its pixels.
struct L1Out {
  const float* target;
  float* grad;
  float inv_count;
  double* partial;
};

// Composites one tile; all 64 lanes of the workgroup call it.  image points
// at the view's (3, H, W) planes (with L1 it may be null: not written);
// final_T / n_contrib at its (H, W) planes or are null.
// With USAGE, the number of the tile's pixels that composite each entry is
// added to usage[Gaussian id].  With L1, dL/dimage = sign(image - target) /
// count is written and the tile's sum of |image - target| stored.  With
// COUNT, the tile's work tallies (entries staged and visited, slot
// evaluations, pairs with T > 0 and alpha >= 1/255) are added to cnt[0..3].
template <bool USAGE, bool L1 = false, bool COUNT = false>
__device__ __forceinline__ void render_tile_fwd(FwdShared& sh, UsageShared* us,
                                                const float4* __restrict__ sv,
                                                const uint32_t* __restrict__ vals, uint2 rg,
                                                int tx, int ty, int W, int H, float bg0,
                                                float bg1, float bg2, float* __restrict__ image,
                                                float* __restrict__ final_T,
                                                int32_t* __restrict__ n_contrib,
                                                uint32_t* __restrict__ usage,
                                                const L1Out* l1 = nullptr,
                                                unsigned long long* cnt = nullptr) {
  const int lane = threadIdx.x;
  uint32_t wk_staged = 0, wk_visits = 0, wk_slots = 0;
  unsigned long long wk_used = 0;
  // slot w's pixel is (x0 + 8 (w & 1), y0 + 8 (w >> 1))
  const int x0 = tx * kTile + (lane & 7), y0 = ty * kTile + (lane >> 3);
  const float fx0 = (float)x0, fy0 = (float)y0;
  // T > 0 while a slot's pixel composites; a pixel that has stopped holds
  // its final transmittance negated (and one outside the image holds -1), so
  // the sign is the per-lane "done" flag without a register of its own
  auto init = [&](int w) {
    FwdSlot st;
    st.T = (x0 + 8 * (w & 1) < W && y0 + 8 * (w >> 1) < H) ? 1.f : -1.f;
    st.c0 = st.c1 = st.c2 = 0.f;
    st.last = 0;
    return st;
  };
  FwdSlot s0 = init(0), s1 = init(1), s2 = init(2), s3 = init(3);
  uint32_t live = live_bit(s0, 0) | live_bit(s1, 1) | live_bit(s2, 2) | live_bit(s3, 3);
  const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
  for (uint32_t b0 = rg.x; b0 < rg.y && live != 0; b0 += kFwdBatch) {
    __syncthreads();
    uint32_t qmask = 0;
    {
      const int k = lane;
      const uint32_t e = b0 + (uint32_t)k;
      if (e < rg.y) {
        const uint32_t g = vals[e];
        const float4 q0 = sv[kSplatF4 * (size_t)g], q1 = sv[kSplatF4 * (size_t)g + 1],
                     q2 = sv[kSplatF4 * (size_t)g + 2];
        const Rec rr = make_rec(q0, q1, q2);
        sh.a[k] = rr.a;
        sh.b[k] = rr.b;
        sh.c[k].x = rr.c.x;
        qmask = quadrant_mask(q0, q1, q2, ox, oy);
        if constexpr (USAGE) {
          us->g[k] = g;
          us->u[k] = 0u;
        }
      }
    }
    // bit k of qm[w]: entry b0 + k is evaluated in slot w (cleared for a
    // slot once none of its pixels composites any more)
    unsigned long long qm[4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
      qm[w] = (live >> w) & 1u ? __builtin_amdgcn_ballot_w64((qmask >> w) & 1u) : 0ull;
    __syncthreads();
    if constexpr (COUNT) {
      const uint32_t left = rg.y - b0;
      wk_staged += left < (uint32_t)kFwdBatch ? left : (uint32_t)kFwdBatch;
    }
    // entries front to back, only those evaluated in a live slot
    for (unsigned long long todo = qm[0] | qm[1] | qm[2] | qm[3]; todo != 0;) {
      const int k = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const unsigned long long bit = 1ull << k;
      const uint32_t m = ((qm[0] & bit) ? 1u : 0u) | ((qm[1] & bit) ? 2u : 0u) |
                         ((qm[2] & bit) ? 4u : 0u) | ((qm[3] & bit) ? 8u : 0u);
      if constexpr (COUNT) ++wk_visits;
      uint32_t used = 0;
      const float4 a = sh.a[k];
      const float4 b = sh.b[k];
      const float cb = sh.c[k].x;
      const int pos = (int)(b0 - rg.x) + k + 1;
      int posv;  // pos in a vector register, read by the per-slot selects
      asm("v_mov_b32 %0, %1" : "=v"(posv) : "s"(pos));
      const float dxl = a.x - fx0, dyt = a.y - fy0;
      auto slot = [&](auto wid, FwdSlot& st) {
        constexpr int w = decltype(wid)::value;
        if (m & (1u << w)) {
          // per-lane decisions as selects: no divergent branches in the slot
          const float dx = (w & 1) ? dxl - 8.f : dxl;
          const float dy = (w >> 1) ? dyt - 8.f : dyt;
          const float alpha = fminf(kAlphaMax, eval_ea(a, row_q(b, dy), dx, dy));
          const float Tk = st.T;
          const bool use = Tk > 0.f && alpha >= kAlphaMin;
          const float Tn = Tk * (1.f - alpha);
          const bool stop = use && Tn < kTStop;
          const bool comp = use && !stop;
          const float wt = comp ? alpha * Tk : 0.f;
          st.c0 = fmaf(b.z, wt, st.c0);
          st.c1 = fmaf(b.w, wt, st.c1);
          st.c2 = fmaf(cb, wt, st.c2);
          // a stopping pixel keeps its transmittance, negated
          st.T = comp ? Tn : (stop ? -Tk : Tk);
          st.last = comp ? posv : st.last;
          if constexpr (USAGE) used += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(comp));
          if constexpr (COUNT) {
            ++wk_slots;
            wk_used += (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(use));
          }
          if (__builtin_amdgcn_ballot_w64(stop) != 0) {  // once per pixel
            if (__builtin_amdgcn_ballot_w64(st.T > 0.f) == 0) {
              live &= ~(1u << w);
              qm[w] = 0;
            }
          }
        }
      };
      slot(SlotId<0>{}, s0);
      slot(SlotId<1>{}, s1);
      slot(SlotId<2>{}, s2);
      slot(SlotId<3>{}, s3);
      if constexpr (USAGE) {
        if (lane == 0 && used) us->u[k] = used;
      }
      if (live == 0) break;
      // drop the entries left only in slots that stopped at this one
      todo &= qm[0] | qm[1] | qm[2] | qm[3];
    }
    if constexpr (USAGE) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kFwdBatch / 64; ++r) {
        const int k = r * 64 + lane;
        if (b0 + (uint32_t)k < rg.y && us->u[k]) atomicAdd(usage + us->g[k], us->u[k]);
      }
    }
  }
  const size_t pix = (size_t)W * H;
  double l1sum = 0.0;
  auto write = [&](int w, const FwdSlot& st) {
    // the pixel from its float coordinates (exact): the integer ones need
    // not stay live over the entry loop, which reads only the floats
    const int x = (int)fx0 + 8 * (w & 1), y = (int)fy0 + 8 * (w >> 1);
    if (!(x < W && y < H)) return;
    const size_t p = (size_t)y * W + x;
    const float Tf = fabsf(st.T);
    const float o0 = st.c0 + Tf * bg0, o1 = st.c1 + Tf * bg1, o2 = st.c2 + Tf * bg2;
    if (!L1 || image) {
      image[p] = o0;
      image[pix + p] = o1;
      image[2 * pix + p] = o2;
    }
    if constexpr (L1) {
      const float d[3] = {o0 - l1->target[p], o1 - l1->target[pix + p],
                          o2 - l1->target[2 * pix + p]};
      const float iv = l1->inv_count;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        l1->grad[ch * pix + p] = d[ch] > 0.f ? iv : (d[ch] < 0.f ? -iv : 0.f);
        l1sum += (double)fabsf(d[ch]);
      }
    }
    if (final_T) final_T[p] = Tf;
    if (n_contrib) n_contrib[p] = st.last;
  };
  write(0, s0);
  write(1, s1);
  write(2, s2);
  write(3, s3);
  if constexpr (L1) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) l1sum += __shfl_xor(l1sum, off, 64);
    if (lane == 0) *l1->partial = l1sum;
  }
  if constexpr (COUNT) {
    if (lane == 0) {
      atomicAdd(cnt + kWkFwdStaged, (unsigned long long)wk_staged);
      atomicAdd(cnt + kWkFwdVisits, (unsigned long long)wk_visits);
      atomicAdd(cnt + kWkFwdSlots, (unsigned long long)wk_slots);
      atomicAdd(cnt + kWkFwdUsed, wk_used);
    }
  }
}

template <bool COUNT>
__global__ __launch_bounds__(64) void k_render_fwd(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib, unsigned long long* __restrict__ cnt) {
  __shared__ FwdShared sh;
  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const size_t pix = (size_t)W * H;
  render_tile_fwd<false, false, COUNT>(sh, nullptr, splat + kSplatF4 * (size_t)v * ld, vals,
                                       ranges[seg], tx, ty, W, H, bg0, bg1, bg2,
                                       image + 3 * pix * v, final_T + pix * v,
                                       n_contrib + pix * v, nullptr, nullptr, cnt);
}

// Forward with the L1 term fused: per tile, the pixels' dL/dimage and the sum
// of |image - target| (added up by k_l1_chunk_sum and k_l1_chunks_total).
template <bool COUNT>
__global__ __launch_bounds__(64) void k_render_fwd_l1(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib, const float* __restrict__ target, float* __restrict__ grad,
    float inv_count, double* __restrict__ partial, unsigned long long* __restrict__ cnt) {
  __shared__ FwdShared sh;
  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const size_t pix = (size_t)W * H;
  const L1Out o{target + 3 * pix * v, grad + 3 * pix * v, inv_count, partial + seg};
  render_tile_fwd<false, true, COUNT>(sh, nullptr, splat + kSplatF4 * (size_t)v * ld, vals,
                                      ranges[seg], tx, ty, W, H, bg0, bg1, bg2,
                                      image ? image + 3 * pix * v : nullptr, final_T + pix * v,
                                      n_contrib + pix * v, nullptr, &o, cnt);
}

// loss += (sum of the per-tile partials) / count in two fixed-order steps:
// workgroup b adds partials [b chunk, (b + 1) chunk) (each thread a fixed
// stride pattern, then a tree) and stores the sum over the first of them,
// which no other workgroup reads; one wave then adds those chunk sums.
// One workgroup reading all partials was bound by a single CU's bandwidth.
constexpr int kL1Chunks = 64;

__global__ __launch_bounds__(256) void k_l1_chunk_sum(double* __restrict__ partial, uint32_t n,
                                                      uint32_t chunk) {
  __shared__ double s[4];
  const uint32_t b0 = blockIdx.x * chunk;
  const uint32_t e = min(b0 + chunk, n);
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  uint32_t i = b0 + threadIdx.x;
  for (; i + 3 * 256 < e; i += 4 * 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] += partial[i + u * 256];
  }
  for (int u = 0; i < e; i += 256, ++u) a[u] += partial[i];
  double acc = (a[0] + a[1]) + (a[2] + a[3]);
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && b0 < n) partial[b0] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ __launch_bounds__(64) void k_l1_chunks_total(const double* __restrict__ partial,
                                                        uint32_t n, uint32_t chunk,
                                                        uint32_t n_chunks, double inv_count,
                                                        double* __restrict__ loss) {
  double acc = 0.0;
  for (uint32_t c = threadIdx.x; c < n_chunks; c += 64)
    if (c * chunk < n) acc += partial[(size_t)c * chunk];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (threadIdx.x == 0) atomicAdd(loss, acc * inv_count);
}

__global__ __launch_bounds__(64) void k_render_fwd_usage(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, float* __restrict__ image, float* __restrict__ final_T,
    int32_t* __restrict__ n_contrib, uint32_t* __restrict__ usage) {
  __shared__ FwdShared sh;
  __shared__ UsageShared us;
  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const size_t pix = (size_t)W * H;
  render_tile_fwd<true>(sh, &us, splat + kSplatF4 * (size_t)v * ld, vals, ranges[seg], tx, ty,
                        W, H, bg0, bg1, bg2, image + 3 * pix * v, final_T + pix * v,
                        n_contrib + pix * v, usage);
}

// Per-request geometry for the batched renderer: segment base (V+1), pixel
// base (V+1, in pixels of the packed output), width/height (V).
__global__ void k_batch_info(const gs_camera* __restrict__ cams, int V, uint32_t* seg_base,
                             int64_t* pix_base, int2* wh, uint32_t* queue) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t s = 0;
  int64_t p = 0;
  for (int v = 0; v < V; ++v) {
    const int W = cams[v].width, H = cams[v].height;
    seg_base[v] = s;
    pix_base[v] = p;
    wh[v] = make_int2(W, H);
    s += (uint32_t)(tiles_across(W) * tiles_across(H));
    p += (int64_t)W * H;
  }
  seg_base[V] = s;
  pix_base[V] = p;
  *queue = 0u;
}

// Persistent multi-request renderer: each workgroup repeatedly takes the
// next (request, tile) item from a device-wide counter until the queue is
// drained, so requests of uneven sizes share one launch.
__global__ __launch_bounds__(64) void k_render_persistent(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ seg_base,
    const int64_t* __restrict__ pix_base, const int2* __restrict__ wh, int V, uint32_t total,
    float bg0, float bg1, float bg2, float* __restrict__ images, uint32_t* __restrict__ queue) {
  __shared__ FwdShared sh;
  __shared__ uint32_t s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    if (item >= total) break;
    int lo = 0, hi = V - 1;  // request: last v with seg_base[v] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (seg_base[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int2 d = wh[lo];
    const int TX = tiles_across(d.x);
    const int tile = (int)(item - seg_base[lo]);
    const int ty = tile / TX, tx = tile - ty * TX;
    render_tile_fwd<false>(sh, nullptr, splat + kSplatF4 * (size_t)lo * ld, vals, ranges[item],
                           tx, ty, d.x, d.y, bg0, bg1, bg2, images + 3 * pix_base[lo], nullptr,
                           nullptr, nullptr);
  }
}

// ---------------------------------------------------------------- backward
constexpr int kRowFloats = 9;  // per-instance gradient row

// Index of the instance of a (view, Gaussian) in tile (tx, ty): the binning
// emits its tiles row by row, starting at the base it stores in the record's
// fourth float4 = (tx0 | ty0 << 16, width | kSpanFlag, base, spans): over the
// whole rectangle, or, with the flag, over columns [tx0 + a_r, tx0 + b_r) of
// row r (byte r of spans = a_r | b_r << 4, at most four rows).
__device__ __forceinline__ uint32_t instance_row(float4 q3, int tx, int ty) {
  const uint32_t o = __float_as_uint(q3.x), w = __float_as_uint(q3.y),
                 base = __float_as_uint(q3.z), m = __float_as_uint(q3.w);
  const uint32_t r = (uint32_t)ty - (o >> 16), c = (uint32_t)tx - (o & 0xFFFFu);
  if (w & kSpanFlag) {
    // instances in the rows above: the byte sum of the spans b - a below row r
    const uint32_t sp = ((m >> 4) & 0x0F0F0F0Fu) - (m & 0x0F0F0F0Fu);
    const uint32_t sh = 8u * r;
    const uint32_t pre = ((sp & ((1u << sh) - 1u)) * 0x01010101u) >> 24;
    return base + pre + c - ((m >> sh) & 15u);
  }
  return base + r * w + c;
}

// Row sums of an entry: value cc of row r at acc[entry * kAccStride + 4 cc + r]
// (odd stride: the 36 writers of an entry and the 32 readers of one value at
// flush fall in distinct banks).
constexpr int kAccStride = 37;

struct BwdShared {
  float4 a[kBwdBatch];
  float4 b[kBwdBatch];
  float4 c[kBwdBatch];
  uint32_t g[kBwdBatch];
  float A[kBwdBatch];  // conic A, for the mean gradient at flush
  float4 acc4[(kBwdBatch * kAccStride + 3) / 4];
};

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// With COUNT, the tile's work tallies (entries staged and visited, slot
// evaluations, pairs inside the pixel's prefix with alpha >= 1/255) are
// added to cnt[4..7].
template <bool COUNT>
__global__ __launch_bounds__(64) void k_render_bwd(
    const float4* __restrict__ splat, int ld, const uint32_t* __restrict__ vals,
    const uint2* __restrict__ ranges, int W, int H, int TX, int tiles_per_view, float bg0,
    float bg1, float bg2, const float* __restrict__ final_T, const int32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimage, float* __restrict__ rows,
    unsigned long long* __restrict__ cnt) {
  __shared__ BwdShared sh;
  const int seg = blockIdx.x;
  const int v = seg / tiles_per_view, tile = seg - v * tiles_per_view;
  const int ty = tile / TX, tx = tile - ty * TX;
  const int lane = threadIdx.x;
  const uint2 rg = ranges[seg];
  const float4* sv = splat + kSplatF4 * (size_t)v * ld;
  const size_t pix = (size_t)W * H;
  const float* gi = dL_dimage + 3 * pix * v;

  const int x0 = tx * kTile + (lane & 7), y0 = ty * kTile + (lane >> 3);
  const float fx0 = (float)x0, fy0 = (float)y0;
  // S[w] = dL/dcolour . B, B the colour composited behind the current entry
  // (background included): only this dot product enters dL/dalpha
  float T[4], g0[4], g1[4], g2[4], S[4];
  int nc[4], wmax[4];
  int jmax = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int x = x0 + 8 * (w & 1), y = y0 + 8 * (w >> 1);
    T[w] = 1.f;
    g0[w] = g1[w] = g2[w] = 0.f;
    nc[w] = 0;
    if (x < W && y < H) {
      const size_t p = (size_t)y * W + x;
      T[w] = final_T[pix * v + p];
      nc[w] = n_contrib[pix * v + p];
      g0[w] = gi[p];
      g1[w] = gi[pix + p];
      g2[w] = gi[2 * pix + p];
    }
    S[w] = g0[w] * bg0 + g1[w] * bg1 + g2[w] * bg2;
    wmax[w] = __builtin_amdgcn_readfirstlane(wave_max(nc[w]));
    jmax = max(jmax, wmax[w]);
  }
  const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
  // the row sum this lane ends up holding, and whether it stores it
  const bool u3 = lane & 8, u2 = lane & 4, u1 = lane & 2, u0 = lane & 1;
  const int acc_lane = 4 * (u0 ? 8 : 4 * (int)u1 + 2 * (int)u2 + (int)u3) + (lane >> 4);
  const bool acc_writer = !u0 || (lane & 15) == 1;
  float* acc = reinterpret_cast<float*>(sh.acc4);
  uint32_t wk_staged = 0, wk_visits = 0, wk_slots = 0;
  unsigned long long wk_used = 0;

  for (int hi = jmax; hi > 0; hi -= kBwdBatch) {
    const int lo = hi > kBwdBatch ? hi - kBwdBatch : 0;
    if constexpr (COUNT) wk_staged += (uint32_t)(hi - lo);
    __syncthreads();
    // lanes k and k + 32 both load entry k; the lower lane stages it and
    // tests the upper row of quadrants, the other lane the lower row
    uint32_t qrow = 0;
    {
      const int k = lane & 31, h = lane >> 5;
      if (k < kBwdBatch && lo + k < hi) {
        const uint32_t g = vals[rg.x + (uint32_t)(lo + k)];
        const float4 q0 = sv[kSplatF4 * (size_t)g], q1 = sv[kSplatF4 * (size_t)g + 1],
                     q2 = sv[kSplatF4 * (size_t)g + 2], q3 = sv[kSplatF4 * (size_t)g + 3];
        if (h == 0) {
          const Rec rr = make_rec(q0, q1, q2);
          sh.a[k] = rr.a;
          sh.b[k] = rr.b;
          sh.c[k] = rr.c;
          sh.A[k] = q0.z;
          sh.g[k] = instance_row(q3, tx, ty);
        }
        qrow = quadrant_row_mask(q0, q1, q2, ox, oy + (float)(8 * h));
        // past every pixel's last contributor in a quadrant: nothing to do
        if (lo + k >= (h ? wmax[2] : wmax[0])) qrow &= ~1u;
        if (lo + k >= (h ? wmax[3] : wmax[1])) qrow &= ~2u;
      }
    }
    // bit k of qm[w]: entry lo + k is evaluated in quadrant w
    uint32_t qm[4];
    {
      const unsigned long long b0 = __builtin_amdgcn_ballot_w64((qrow & 1u) != 0);
      const unsigned long long b1 = __builtin_amdgcn_ballot_w64((qrow & 2u) != 0);
      qm[0] = (uint32_t)b0;
      qm[1] = (uint32_t)b1;
      qm[2] = (uint32_t)(b0 >> 32);
      qm[3] = (uint32_t)(b1 >> 32);
    }
    for (int t = lane; t < (kBwdBatch * kAccStride + 3) / 4; t += 64)
      sh.acc4[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // entries back to front, only those evaluated somewhere
    const int lo_u = __builtin_amdgcn_readfirstlane(lo);
    for (uint32_t todo = qm[0] | qm[1] | qm[2] | qm[3]; todo != 0;) {
      const int k = 31 - __builtin_clz(todo);
      todo ^= 1u << k;
      const int j = lo_u + k;  // position in the tile list
      if constexpr (COUNT) ++wk_visits;
      const float4 a = sh.a[k];
      const float4 b = sh.b[k];
      const float4 c = sh.c[k];
      const float dxl = a.x - fx0, dyt = a.y - fy0;
      float gr[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      unsigned long long contrib = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        if ((qm[w] >> k) & 1u) {
          // per-lane decisions as selects; an unused pair gets alpha 0, which
          // leaves T and B unchanged and contributes nothing
          const float dx = (w & 1) ? dxl - 8.f : dxl;
          const float dy = (w >> 1) ? dyt - 8.f : dyt;
          const float dy2 = dy * dy;
          // t = dx + r1 dy, the coordinate the exponent squares (eval_ea)
          const float t = fmaf(a.w, dy, dx);
          const float ea = __builtin_amdgcn_exp2f(fmaf(a.z * t, t, fmaf(b.x, dy2, b.y)));
          const float alpha = fminf(kAlphaMax, ea);
          const bool live = j < nc[w], vis = alpha >= kAlphaMin;
          const bool use = live && vis;
          const float au = use ? alpha : 0.f;
          const float Tk = T[w] * __builtin_amdgcn_rcpf(1.f - au);
          const float wt = au * Tk;
          gr[6] = fmaf(g0[w], wt, gr[6]);
          gr[7] = fmaf(g1[w], wt, gr[7]);
          gr[8] = fmaf(g2[w], wt, gr[8]);
          // g . (c - B) with B updated as B + au (c - B)
          const float gcb = fmaf(g2[w], c.x, fmaf(g1[w], b.w, fmaf(g0[w], b.z, -S[w])));
          // gp = dL/dalpha * alpha = dL/dpower: dL/dalpha = Tk gcb where the
          // pair is used and alpha is not clamped (then alpha = ea), else 0;
          // wt = 0 where unused, so only the clamp needs a select
          const float gp = ea < kAlphaMax ? wt * gcb : 0.f;
          // moments of dL/dpower in (t, dy), which the exponent already
          // formed: the conic and mean gradients are linear in them with
          // per-entry coefficients, applied once per entry at flush
          const float pt = gp * t;
          gr[0] += pt;
          gr[1] = fmaf(gp, dy, gr[1]);
          gr[2] = fmaf(pt, t, gr[2]);
          gr[3] = fmaf(pt, dy, gr[3]);
          gr[4] = fmaf(gp, dy2, gr[4]);
          gr[5] += gp;  // dL/dalpha * ea, times 1/opacity at flush
          S[w] = fmaf(au, gcb, S[w]);
          T[w] = Tk;
          // the ballots of the two compares, so the masks are used as they are
          contrib |= __builtin_amdgcn_ballot_w64(live) & __builtin_amdgcn_ballot_w64(vis);
          if constexpr (COUNT) {
            ++wk_slots;
            wk_used += (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(use));
          }
        }
      }
      if (contrib == 0) continue;
      // nine row sums per row, one per lane; the four rows are added at flush
      const float rs = row_sums9(gr, u1, u0);
      if (acc_writer) acc[k * kAccStride + acc_lane] = rs;
    }
    __syncthreads();
    for (int k = lane; k < kBwdBatch; k += 64) {
      if (lo + k < hi) {
        float* dst = rows + (size_t)sh.g[k] * kRowFloats;
        float mom[9];
#pragma unroll
        for (int cc = 0; cc < 9; ++cc) {
          const float* r4 = acc + k * kAccStride + 4 * cc;
          mom[cc] = (r4[0] + r4[1]) + (r4[2] + r4[3]);
        }
        // back from (t, dy) to (dx, dy) with dx = t - r1 dy: the sums of gp
        // dx, dx^2 and dx dy
        const float r1 = sh.a[k].w;
        const float m_t = mom[0], m_tt = mom[2], m_ty = mom[3], m_yy = mom[4];
        mom[0] = fmaf(-r1, mom[1], m_t);
        mom[2] = fmaf(-r1, fmaf(-r1, m_yy, 2.f * m_ty), m_tt);
        mom[3] = fmaf(-r1, m_yy, m_ty);
        // power = -(A dx^2 + C dy^2)/2 - B dx dy with dx = px - x, dy = py - y
        const float A = sh.A[k], B = sh.c[k].z, C = sh.c[k].w;
        float out[9];
        out[0] = -(A * mom[0] + B * mom[1]);
        out[1] = -(B * mom[0] + C * mom[1]);
        out[2] = -0.5f * mom[2];
        out[3] = -mom[3];
        out[4] = -0.5f * mom[4];
        out[5] = mom[5] * sh.c[k].y;
        out[6] = mom[6];
        out[7] = mom[7];
        out[8] = mom[8];
#pragma unroll
        for (int cc = 0; cc < 9; ++cc) dst[cc] = out[cc];
      }
    }
  }
  // entries behind every pixel's last contributor carry zero gradient
  const int n_entries = (int)(rg.y - rg.x);
  for (int j = jmax + lane; j < n_entries; j += 64) {
    const uint32_t g = vals[rg.x + (uint32_t)j];
    float* dst = rows + (size_t)instance_row(sv[kSplatF4 * (size_t)g + 3], tx, ty) * kRowFloats;
#pragma unroll
    for (int cc = 0; cc < 9; ++cc) dst[cc] = 0.f;
  }
  if constexpr (COUNT) {
    if (lane == 0) {
      atomicAdd(cnt + kWkBwdStaged, (unsigned long long)wk_staged);
      atomicAdd(cnt + kWkBwdVisits, (unsigned long long)wk_visits);
      atomicAdd(cnt + kWkBwdSlots, (unsigned long long)wk_slots);
      atomicAdd(cnt + kWkBwdUsed, wk_used);
    }
  }
}

// One step of a segmented inclusive scan of nine values over the wave: add
// the value of the lane CTRL names when it carries the same pair index q.
// q does not decrease over the lanes, so equal ends mean that every lane in
// between belongs to the same pair.  A lane with no source (outside its row
// for the shifts, or in a row the mask leaves out) adds 0.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ void seg_scan_step(int q, float (&x)[9]) {
  const int qs = __builtin_amdgcn_update_dpp(-1, q, CTRL, ROW_MASK, 0xF, BOUND);
  const bool take = qs == q;
#pragma unroll
  for (int cc = 0; cc < 9; ++cc) {
    const float sum = x[cc] + dpp_take<CTRL, ROW_MASK, BOUND>(x[cc]);
    x[cc] = take ? sum : x[cc];
  }
}

// Screen-space gradient of each (view, Gaussian): the sum of its instance
// rows, which the binning emitted contiguously (one per covered tile).  Each
// wave takes 64 (view, Gaussian) pairs and walks the union of their rows 64
// at a time (row f of the union on lane f mod 64, so long and short runs
// balance and the loads coalesce within a run); a segmented scan over the
// lanes sums each pair's rows of the step, and the lane at the end of a
// pair's segment adds them to that pair's LDS accumulator.
__global__ __launch_bounds__(256) void k_grad_gather(int n, int ld, int V,
                                                     const int32_t* __restrict__ tiles,
                                                     const uint32_t* __restrict__ splat_words,
                                                     const float* __restrict__ rows,
                                                     float* __restrict__ grad2d) {
  __shared__ uint32_t s_pre[4][64];
  __shared__ uint32_t s_base[4][64];
  __shared__ float s_acc[4][9][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t total = (size_t)n * V;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t gv = 0;
  uint32_t c = 0, base = 0;
  if (t < total) {
    const size_t v = t / (size_t)n, i = t - v * (size_t)n;
    gv = v * (size_t)ld + i;
    const int ct = tiles[gv];
    if (ct > 0) {
      c = (uint32_t)ct;
      base = splat_words[gv * (4 * kSplatF4) + 14];  // first instance of the pair
    }
  }
  uint32_t incl = c;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const uint32_t R = __shfl(incl, 63, 64);
  s_pre[wave][lane] = incl - c;
  s_base[wave][lane] = base;
#pragma unroll
  for (int cc = 0; cc < 9; ++cc) s_acc[wave][cc][lane] = 0.f;
  __syncthreads();
  for (uint32_t f0 = 0; f0 < R; f0 += 64) {
    const uint32_t f = f0 + lane;
    const bool valid = f < R;
    int q = 64;  // sentinel for lanes past the end
    float x[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid) {
      q = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if (s_pre[wave][q + step] <= f) q += step;
      const float* r = rows + (size_t)(s_base[wave][q] + (f - s_pre[wave][q])) * kRowFloats;
#pragma unroll
      for (int cc = 0; cc < 9; ++cc) x[cc] = r[cc];
    }
    // segmented inclusive scan over lanes with equal q: shifts by 1, 2, 4, 8
    // within each 16-lane row, then each row's last lane into the rows after
    seg_scan_step<0x111, 0xF, true>(q, x);   // row_shr:1
    seg_scan_step<0x112, 0xF, true>(q, x);   // row_shr:2
    seg_scan_step<0x114, 0xF, true>(q, x);   // row_shr:4
    seg_scan_step<0x118, 0xF, true>(q, x);   // row_shr:8
    seg_scan_step<0x142, 0xA, false>(q, x);  // row_bcast:15 into rows 1, 3
    seg_scan_step<0x143, 0xC, false>(q, x);  // row_bcast:31 into rows 2, 3
    const int qn = __shfl_down(q, 1, 64);
    if (valid && (lane == 63 || qn != q)) {
#pragma unroll
      for (int cc = 0; cc < 9; ++cc) s_acc[wave][cc][q] += x[cc];
    }
  }
  __syncthreads();
  if (t < total) {
    float4* o = reinterpret_cast<float4*>(grad2d + gv * kGrad2dFloats);
    o[0] = make_float4(s_acc[wave][0][lane], s_acc[wave][1][lane], s_acc[wave][2][lane],
                       s_acc[wave][3][lane]);
    o[1] = make_float4(s_acc[wave][4][lane], s_acc[wave][5][lane], s_acc[wave][6][lane],
                       s_acc[wave][7][lane]);
    o[2] = make_float4(s_acc[wave][8][lane], 0.f, 0.f, 0.f);
  }
}

}  // namespace

void launch_render_fwd(const gs_projected& proj, const gs_tile_lists& lists, int V, int W, int H,
                       const float bg[3], float* image, float* final_T, int32_t* n_contrib,
                       uint32_t* usage, hipStream_t s) {
  const int TX = tiles_across(W), TY = tiles_across(H);
  const int tpv = TX * TY;
  const int blocks = tpv * V;
  if (blocks == 0) return;
  StageScope scope(kStRenderFwd, s);
  if (usage)
    hipLaunchKernelGGL(k_render_fwd_usage, dim3(blocks), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                       reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                       bg[2], image, final_T, n_contrib, usage);
  else if (g_work)
    hipLaunchKernelGGL(k_render_fwd<true>, dim3(blocks), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                       reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                       bg[2], image, final_T, n_contrib, g_work);
  else
    hipLaunchKernelGGL(k_render_fwd<false>, dim3(blocks), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                       reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                       bg[2], image, final_T, n_contrib, nullptr);
}

size_t render_fwd_l1_workspace_bytes(int V, int W, int H) {
  return (size_t)V * (size_t)tiles_across(W) * (size_t)tiles_across(H) * sizeof(double);
}

void launch_render_fwd_l1(const gs_projected& proj, const gs_tile_lists& lists, int V, int W,
                          int H, const float bg[3], const float* target, float* image,
                          float* final_T, int32_t* n_contrib, float* grad, double* loss,
                          void* ws, hipStream_t s) {
  const int TX = tiles_across(W), TY = tiles_across(H);
  const int tpv = TX * TY;
  const int blocks = tpv * V;
  if (blocks == 0) return;
  const double count = 3.0 * (double)V * (double)W * (double)H;
  double* partial = static_cast<double*>(ws);
  StageScope scope(kStRenderFwd, s);
  if (g_work)
    hipLaunchKernelGGL(k_render_fwd_l1<true>, dim3(blocks), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                       reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                       bg[2], image, final_T, n_contrib, target, grad, (float)(1.0 / count),
                       partial, g_work);
  else
    hipLaunchKernelGGL(k_render_fwd_l1<false>, dim3(blocks), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                       reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0], bg[1],
                       bg[2], image, final_T, n_contrib, target, grad, (float)(1.0 / count),
                       partial, nullptr);
  const uint32_t chunk = ((uint32_t)blocks + kL1Chunks - 1) / kL1Chunks;
  const uint32_t n_chunks = ((uint32_t)blocks + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_l1_chunk_sum, dim3(n_chunks), dim3(256), 0, s, partial, (uint32_t)blocks,
                     chunk);
  hipLaunchKernelGGL(k_l1_chunks_total, dim3(1), dim3(64), 0, s, (const double*)partial,
                     (uint32_t)blocks, chunk, n_chunks, 1.0 / count, loss);
}

size_t render_batched_workspace_bytes(int V) {
  return 256 + 256 * ((((size_t)V + 1) * 4 + 255) / 256) +
         256 * ((((size_t)V + 1) * 8 + 255) / 256) +
         256 * (((size_t)V * 8 + 255) / 256);
}

void launch_render_batched(const gs_projected& proj, const gs_tile_lists& lists,
                           const gs_camera* cams_dev, int V, int64_t total_segments,
                           const float bg[3], float* images, void* ws, hipStream_t s) {
  char* w = static_cast<char*>(ws);
  uint32_t* queue = reinterpret_cast<uint32_t*>(w);
  w += 256;
  uint32_t* seg_base = reinterpret_cast<uint32_t*>(w);
  w += 256 * ((((size_t)V + 1) * 4 + 255) / 256);
  int64_t* pix_base = reinterpret_cast<int64_t*>(w);
  w += 256 * ((((size_t)V + 1) * 8 + 255) / 256);
  int2* wh = reinterpret_cast<int2*>(w);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;  // the grid size only tunes occupancy; the queue drains either way
  const int64_t want = (int64_t)cus * 16;
  const int blocks = (int)(total_segments < want ? total_segments : want);
  StageScope scope(kStRenderFwd, s);
  hipLaunchKernelGGL(k_batch_info, dim3(1), dim3(64), 0, s, cams_dev, V, seg_base, pix_base, wh,
                     queue);
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_render_persistent, dim3(blocks), dim3(64), 0, s,
                     reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                     reinterpret_cast<const uint2*>(lists.ranges), seg_base, pix_base, wh, V,
                     (uint32_t)total_segments, bg[0], bg[1], bg[2], images, queue);
}

void launch_render_bwd(const gs_projected& proj, const gs_tile_lists& lists, int V, int W, int H,
                       const float bg[3], const float* final_T, const int32_t* n_contrib,
                       const float* dL_dimage, float* rows, float* grad2d, hipStream_t s) {
  const int TX = tiles_across(W), TY = tiles_across(H);
  const int tpv = TX * TY;
  const int blocks = tpv * V;
  if (blocks == 0) return;
  {
    StageScope scope(kStRenderBwd, s);
    if (g_work)
      hipLaunchKernelGGL(k_render_bwd<true>, dim3(blocks), dim3(64), 0, s,
                         reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                         reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0],
                         bg[1], bg[2], final_T, n_contrib, dL_dimage, rows, g_work);
    else
      hipLaunchKernelGGL(k_render_bwd<false>, dim3(blocks), dim3(64), 0, s,
                         reinterpret_cast<const float4*>(proj.splat), proj.ld, lists.vals,
                         reinterpret_cast<const uint2*>(lists.ranges), W, H, TX, tpv, bg[0],
                         bg[1], bg[2], final_T, n_contrib, dL_dimage, rows, nullptr);
  }
  const size_t nv = (size_t)proj.n * (size_t)V;
  if (nv == 0) return;
  StageScope scope(kStGradGather, s);
  hipLaunchKernelGGL(k_grad_gather, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, proj.n,
                     proj.ld, V, proj.tiles_touched,
                     reinterpret_cast<const uint32_t*>(proj.splat), rows, grad2d);
}

}  // namespace gs
