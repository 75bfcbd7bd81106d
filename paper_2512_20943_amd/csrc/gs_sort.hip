// Tile binning and depth ordering.
//
// The order the renderer needs is, per tile segment, the instances sorted by
// (FP32 depth, Gaussian id).  It is reached in two sorts that both use the
// same LDS-resident LSD radix sort (stable, 8- or 9-bit digits; per digit,
// per-partition counts, their scan, then LDS ranking and an LDS-staged
// scatter with those bases; partitions are laid out XCD by XCD, so each of
// the 8 L2s sees a contiguous range).  Both sorts run inside views: the
// elements of view v stay in a range of their own whose start is known
// before the sort, so the digits cover only what varies inside a view:
//   1. the depth keys of the V*n projected Gaussians (only the visible
//      pairs, gathered view by view), on the bits of the visible depth-bit
//      range (a first pass reduces that range together with the instance
//      count, which the host reads back); the key also carries the view
//      above those bits, in 32 bits when it fits, else in the high word of
//      a 64-bit key;
//   2. after emitting every Gaussian's tiles in that depth order (views in
//      order), the instances by their tile index inside the view, on the
//      bits of the largest view's tile count; the last pass turns tile
//      indices into segment ids.
// Stability of (2) keeps the depth order of (1) inside each segment, and
// stability of (1) keeps ascending ids for equal depths, so the result is
// the (segment, depth, id) order -- while the per-instance sort moves only
// ceil(log2(tiles per view)/9) digits of 32-bit keys instead of 5-7 digits
// of 64-bit keys.
#include <algorithm>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 32;
constexpr int kPart = kBlock * kItems;  // keys per radix-sort partition
constexpr int kCountItems = 8;          // entries per thread in the instance count and scan
constexpr int kCountChunk = kBlock * kCountItems;

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <int BITS, typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift) {
  return (uint32_t)(key >> shift) & ((1u << BITS) - 1u);
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_wave,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t v = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  if (lane == 63) s_wave[wave] = v;
  __syncthreads();
  uint32_t pre = 0;
  for (int k = 0; k < wave; ++k) pre += s_wave[k];
  if (total) *total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  __syncthreads();
  return pre + v - x;
}

// Exclusive scan of row[0, n) in place by one block, kIpt consecutive
// values per thread per round; returns the total (to every thread).
template <int kIpt = 16>
__device__ uint32_t block_scan_inplace(uint32_t* __restrict__ row, uint32_t n) {
  __shared__ uint32_t s_wave[4];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < n; b0 += kBlock * kIpt) {
    const uint32_t e0 = b0 + threadIdx.x * kIpt;
    uint32_t x[kIpt], sum = 0;
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      x[i] = e0 + i < n ? row[e0 + i] : 0u;
      sum += x[i];
    }
    uint32_t t;
    uint32_t run = carry + block_exclusive_scan(sum, s_wave, &t);
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      if (e0 + i < n) row[e0 + i] = run;
      run += x[i];
    }
    carry += t;
  }
  return carry;
}

// ------------------------------------------------------------ radix sort
// Every sort here orders keys inside views: view v's elements occupy
// [start(v), start(v + 1)) of the array before and after the sort, with
// start(v) = vstart[v * vstride] for v < V and start(V) = n.  Each view's
// range is cut into partitions of at most kPart keys (none straddles two
// views), so the digits only cover the bits that vary inside a view.

__device__ __forceinline__ uint32_t view_start(const uint32_t* __restrict__ vstart,
                                               uint32_t vstride, int V, uint32_t n, int v) {
  return v < V ? vstart[(size_t)v * vstride] : n;
}

// First partition of each view, pfirst[v] (v < V), and the number of
// partitions, pfirst[V].  One block.
__global__ __launch_bounds__(kBlock) void k_part_first(const uint32_t* __restrict__ vstart,
                                                       uint32_t vstride, int V, uint32_t n,
                                                       uint32_t* __restrict__ pfirst) {
  __shared__ uint32_t s_wave[4];
  uint32_t carry = 0;
  for (int v0 = 0; v0 < V; v0 += kBlock) {
    const int v = v0 + (int)threadIdx.x;
    uint32_t np = 0;
    if (v < V) {
      const uint32_t len = view_start(vstart, vstride, V, n, v + 1) -
                           view_start(vstart, vstride, V, n, v);
      np = (len + kPart - 1) / kPart;
    }
    uint32_t tot;
    const uint32_t e = block_exclusive_scan(np, s_wave, &tot);
    if (v < V) pfirst[v] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) pfirst[V] = carry;
}

// Partition p's {view, first element, end, first partition of its view},
// one thread per partition.
__global__ __launch_bounds__(kBlock) void k_part_desc(const uint32_t* __restrict__ vstart,
                                                      uint32_t vstride, int V, uint32_t n,
                                                      const uint32_t* __restrict__ pfirst,
                                                      uint4* __restrict__ desc) {
  const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= pfirst[V]) return;
  int lo = 0, hi = V - 1;  // last view whose first partition is <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pfirst[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const uint32_t pf = pfirst[lo];
  const uint32_t b = view_start(vstart, vstride, V, n, lo) + (p - pf) * (uint32_t)kPart;
  const uint32_t e = view_start(vstart, vstride, V, n, lo + 1);
  desc[p] = make_uint4((uint32_t)lo, b, min(b + (uint32_t)kPart, e), pf);
}

// Partition table access.  With one view the table is not built: partition
// p is [p kPart, min((p + 1) kPart, n1)) of view 0 and there are
// ceil(n1 / kPart) of them (desc and pfirst are then NULL).
struct PartTable {
  const uint4* desc;
  const uint32_t* pfirst;  // V + 1 entries
  uint32_t n1;             // element count when desc is NULL
  int V;
  __device__ __forceinline__ uint32_t count() const {
    return desc ? pfirst[V] : (n1 + kPart - 1) / kPart;
  }
  __device__ __forceinline__ uint4 at(uint32_t p) const {
    if (desc) return desc[p];
    const uint32_t b = p * (uint32_t)kPart;
    return make_uint4(0u, b, min(b + (uint32_t)kPart, n1), 0u);
  }
  __device__ __forceinline__ uint32_t first_of_view(int v) const { return desc ? pfirst[v] : 0u; }
};

// XCD-aware partition of workgroup b: workgroup b runs on XCD b % 8, and
// each XCD takes a contiguous range of partitions, so one L2 merges the
// neighbouring words of the count rows and the adjacent output runs of a
// digit.
__device__ __forceinline__ uint32_t xcd_part(uint32_t pmax) {
  const uint32_t per = (pmax + 7) / 8;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Per-partition digit counts, digit-major: cnt[d * pmax + p].
template <typename K, int BITS>
__global__ __launch_bounds__(kBlock) void k_part_count(const K* __restrict__ keys, int shift,
                                                       uint32_t pmax, PartTable pt,
                                                       uint32_t* __restrict__ cnt) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t h[R];
  const uint32_t part = xcd_part(pmax);
  if (part >= pt.count()) return;
  for (int t = threadIdx.x; t < R; t += kBlock) h[t] = 0;
  __syncthreads();
  const uint4 ds = pt.at(part);
  K kk[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = ds.y + (uint32_t)j * kBlock + threadIdx.x;
    kk[j] = i < ds.z ? keys[i] : K(0);
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = ds.y + (uint32_t)j * kBlock + threadIdx.x;
    if (i < ds.z) atomicAdd(&h[digit_of<BITS>(kk[j], shift)], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < R; t += kBlock) cnt[(size_t)t * pmax + part] = h[t];
}

// Exclusive scan of each digit's row of partition counts over all
// partitions (one block per digit); the row total goes to tot[d].
__global__ __launch_bounds__(kBlock) void k_part_scan_rows(uint32_t* __restrict__ cnt,
                                                           uint32_t pmax, PartTable pt,
                                                           uint32_t* __restrict__ tot) {
  const uint32_t t = block_scan_inplace<16>(cnt + (size_t)blockIdx.x * pmax, pt.count());
  if (threadIdx.x == 0) tot[blockIdx.x] = t;
}

// One digit pass with bases from the scans: each wave ranks its keys stably
// by digit with ballots (lanes holding the same digit) and per-wave
// counters in LDS, the block scatters them through LDS into digit order,
// and the global writes come out as runs at (the view's digit start + this
// partition's prefix inside the view); the view's digit starts come from
// the scanned count rows at its first partition and the next view's.  No
// partition waits for another.
// With VALS the values move with the keys; without, the keys carry their
// value in the bits below `shift` of the first pass, and a pass given vout
// splits each key on the way out: value = key & umask to vout, key >> ushift
// to kout.  add (optional, last pass): add[view] is added to every key
// written.
template <typename K, int BITS, bool VALS>
__global__ __launch_bounds__(kBlock) void k_scatter_pass(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, int shift, uint32_t pmax, PartTable pt,
    const uint32_t* __restrict__ pbase, const uint32_t* __restrict__ tot,
    const uint32_t* __restrict__ add, int ushift,
    uint32_t umask) {
  constexpr int R = 1 << BITS, DPT = R / kBlock;
  __shared__ uint32_t s_wh[4][R];
  __shared__ uint32_t s_dstart[R];
  __shared__ uint32_t s_gbase[R];
  __shared__ uint32_t s_wave[4];
  __shared__ K s_k[kPart];
  __shared__ uint32_t s_v[VALS ? kPart : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t part = xcd_part(pmax);
  if (part >= pt.count()) return;
  const uint4 ds = pt.at(part);
  const uint32_t view = ds.x, end = ds.z, pf = ds.w;
  for (int t = tid; t < 4 * R; t += kBlock) (&s_wh[0][0])[t] = 0;
  __syncthreads();
  const uint32_t base = ds.y + (uint32_t)wave * 64u * kItems;
  K k[kItems];
  uint32_t val[kItems], rank[kItems], dig[kItems];
  const bool full = end - ds.y == (uint32_t)kPart;
  if (full) {
    const K* kb = kin + base + lane;
#pragma unroll
    for (int j = 0; j < kItems; ++j) k[j] = kb[j * 64];
    if constexpr (VALS) {
      const uint32_t* vb = vin + base + lane;
#pragma unroll
      for (int j = 0; j < kItems; ++j) val[j] = vb[j * 64];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t idx = base + j * 64 + lane;
      k[j] = idx < end ? kin[idx] : K(0);
      if constexpr (VALS) val[j] = idx < end ? vin[idx] : 0u;
    }
  }
  const uint32_t lower_lo = lane >= 32 ? ~0u : ((1u << lane) - 1u);
  const uint32_t lower_hi = lane <= 32 ? 0u : (~0u >> (64 - lane));
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const bool valid = full || base + j * 64 + lane < end;
    const uint32_t d = valid ? digit_of<BITS>(k[j], shift) : 0u;
    const uint64_t vmask = wave_ballot(valid);
    uint32_t pl = (uint32_t)vmask, ph = (uint32_t)(vmask >> 32);
    const uint32_t nd = ~d;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const uint32_t flip = (uint32_t)((int32_t)(nd << (31 - b)) >> 31);
      const uint64_t bb = wave_ballot(flip == 0u);
      pl &= (uint32_t)bb ^ flip;
      ph &= (uint32_t)(bb >> 32) ^ flip;
    }
    const uint32_t below = (uint32_t)(__popc(pl & lower_lo) + __popc(ph & lower_hi));
    const uint32_t cnt = (uint32_t)(__popc(pl) + __popc(ph));
    uint32_t prev = 0;
    if (valid) prev = s_wh[wave][d];
    if (valid && below == cnt - 1) s_wh[wave][d] = prev + cnt;
    rank[j] = prev + below;
    dig[j] = d;
  }
  __syncthreads();
  {
    uint32_t run[DPT], tsum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      uint32_t r = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = s_wh[w][d];
        s_wh[w][d] = r;
        r += c;
      }
      run[i] = r;
      tsum += r;
    }
    uint32_t dstart = block_exclusive_scan(tsum, s_wave, nullptr);
    // the view's digit starts: its start plus the exclusive scan over the
    // digits of its counts, each the difference of the scanned row at the
    // view's first partition and at the next view's (the row total past
    // the last partition); formed here instead of by a launch of their own
    const uint32_t P = pt.count();
    const uint32_t pnext = pt.desc ? pt.first_of_view((int)view + 1) : P;
    const uint32_t vstart0 = ds.y - (part - pf) * (uint32_t)kPart;
    uint32_t tt[DPT], ts = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      const uint32_t* row = pbase + (size_t)d * pmax;
      tt[i] = (pnext < P ? row[pnext] : tot[d]) - row[pf];
      ts += tt[i];
    }
    uint32_t g = vstart0 + block_exclusive_scan(ts, s_wave, nullptr);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      const uint32_t* row = pbase + (size_t)d * pmax;
      s_dstart[d] = dstart;
      s_gbase[d] = g + (row[part] - row[pf]) - dstart;
      dstart += run[i];
      g += tt[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (base + j * 64 + lane < end) {
      const uint32_t lp = s_dstart[dig[j]] + s_wh[wave][dig[j]] + rank[j];
      s_k[lp] = k[j];
      if constexpr (VALS) s_v[lp] = val[j];
    }
  }
  __syncthreads();
  const uint32_t nvalid = end - ds.y;
  const K kadd = add ? (K)add[view] : K(0);
  if constexpr (VALS) {
    for (uint32_t t = tid; t < nvalid; t += kBlock) {
      const K kk = s_k[t];
      const uint32_t g = s_gbase[digit_of<BITS>(kk, shift)] + t;
      kout[g] = kk + kadd;
      vout[g] = s_v[t];
    }
  } else if (vout) {
    for (uint32_t t = tid; t < nvalid; t += kBlock) {
      const K kk = s_k[t];
      const uint32_t g = s_gbase[digit_of<BITS>(kk, shift)] + t;
      kout[g] = (kk >> ushift) + kadd;
      vout[g] = (uint32_t)kk & umask;
    }
  } else {
    for (uint32_t t = tid; t < nvalid; t += kBlock) {
      const K kk = s_k[t];
      kout[s_gbase[digit_of<BITS>(kk, shift)] + t] = kk + kadd;
    }
  }
}

// ------------------------------------------------------------ binning
// Per-view tile geometry from the device cameras, seg_base (V+1) and tx
// (V), one view per thread with a block scan; also initialises the
// stage-1 statistics, stats = {min bits, max bits, count lo, hi, visible}
// (all overwritten when some pair is visible).  One block.
__global__ __launch_bounds__(kBlock) void k_view_info(const gs_camera* __restrict__ cams, int V,
                                                      uint32_t* __restrict__ seg_base,
                                                      int32_t* __restrict__ txv,
                                                      uint32_t* __restrict__ stats) {
  __shared__ uint32_t s_wave[4];
  if (threadIdx.x == 0) {
    stats[0] = 0xFFFFFFFFu;
    stats[1] = 0u;
    stats[2] = 0u;
    stats[3] = 0u;
    stats[4] = 0u;
  }
  uint32_t carry = 0;
  for (int v0 = 0; v0 < V; v0 += kBlock) {
    const int v = v0 + (int)threadIdx.x;
    uint32_t nt = 0;
    if (v < V) {
      const int tx = tiles_across(cams[v].width), ty = tiles_across(cams[v].height);
      txv[v] = tx;
      nt = (uint32_t)(tx * ty);
    }
    uint32_t tot;
    const uint32_t e = block_exclusive_scan(nt, s_wave, &tot);
    if (v < V) seg_base[v] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) seg_base[V] = carry;
}

// The tile counts and depth bits of Gaussians i0 .. i0 + kCountItems - 1
// of one view (0 past n): two 16-B loads per array when the rows are 16-B
// aligned and the run is whole, else one word at a time.
__device__ __forceinline__ void load_run(const int32_t* __restrict__ tv,
                                         const uint32_t* __restrict__ dv, uint32_t i0, int n,
                                         bool vec, uint32_t (&t)[kCountItems],
                                         uint32_t (&d)[kCountItems]) {
  static_assert(kCountItems == 8, "two 16-B loads per array");
  if (vec && i0 + kCountItems <= (uint32_t)n) {
    const int4 ta = *reinterpret_cast<const int4*>(tv + i0);
    const int4 tb = *reinterpret_cast<const int4*>(tv + i0 + 4);
    const uint4 da = *reinterpret_cast<const uint4*>(dv + i0);
    const uint4 db = *reinterpret_cast<const uint4*>(dv + i0 + 4);
    const int tt[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
    const uint32_t dd[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
#pragma unroll
    for (int j = 0; j < kCountItems; ++j) {
      t[j] = (uint32_t)max(tt[j], 0);
      d[j] = dd[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kCountItems; ++j) {
      const uint32_t i = i0 + j;
      t[j] = i < (uint32_t)n ? (uint32_t)max(tv[i], 0) : 0u;
      d[j] = t[j] > 0 ? dv[i] : 0u;
    }
  }
}

__device__ __forceinline__ bool rows_aligned(int ld, const void* a, const void* b) {
  return (ld & 3) == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

// Per chunk of kCountChunk Gaussians of one view (grid x; views on grid y,
// looping past 65535 of them), chunk c = v * gridDim.x + blockIdx.x: the
// range of the depth bits of its visible pairs and their instance count,
// part[c] = {min bits, max bits, count lo, count hi}, the number of its
// visible pairs, vis[c], and the count's low word again, icnt[c] (scanned,
// it places each view's instances).  Thread t owns Gaussians 8t .. 8t + 7.
__global__ __launch_bounds__(kBlock) void k_depth_range(int n, int ld, int V,
                                                        const uint32_t* __restrict__ depth_bits,
                                                        const int32_t* __restrict__ tiles,
                                                        uint4* __restrict__ part,
                                                        uint32_t* __restrict__ vis,
                                                        uint32_t* __restrict__ icnt) {
  __shared__ uint32_t s_min[4], s_max[4], s_cnt[4];
  __shared__ unsigned long long s_sum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool vec = rows_aligned(ld, tiles, depth_bits);
  for (int v = blockIdx.y; v < V; v += gridDim.y) {
    const int32_t* tv = tiles + (size_t)v * ld;
    const uint32_t* dv = depth_bits + (size_t)v * ld;
    const uint32_t i0 = blockIdx.x * (uint32_t)kCountChunk + threadIdx.x * kCountItems;
    uint32_t mn = 0xFFFFFFFFu, mx = 0u, cnt = 0u;
    unsigned long long sum = 0;
    uint32_t t[kCountItems], d[kCountItems];
    load_run(tv, dv, i0, n, vec, t, d);
#pragma unroll
    for (int j = 0; j < kCountItems; ++j) {
      if (t[j] > 0) {
        mn = min(mn, d[j]);
        mx = max(mx, d[j]);
        sum += (unsigned long long)t[j];
        ++cnt;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, 64));
      mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
      sum += __shfl_xor(sum, off, 64);
      cnt += (uint32_t)__shfl_xor((int)cnt, off, 64);
    }
    if (lane == 0) {
      s_min[wave] = mn;
      s_max[wave] = mx;
      s_sum[wave] = sum;
      s_cnt[wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      mn = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
      mx = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
      sum = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
      const size_t c = (size_t)v * gridDim.x + blockIdx.x;
      part[c] = make_uint4(mn, mx, (uint32_t)sum, (uint32_t)(sum >> 32));
      vis[c] = (s_cnt[0] + s_cnt[1]) + (s_cnt[2] + s_cnt[3]);
      icnt[c] = (uint32_t)sum;
    }
    __syncthreads();
  }
}

// stats = {min bits, max bits, count lo, count hi} over the per-block
// partials of k_depth_range, by one block (device-wide atomics on three
// addresses from every block serialise at the memory side).
__device__ __forceinline__ void stats_reduce(const uint4* __restrict__ part, int nb,
                                             uint32_t* __restrict__ stats) {
  __shared__ uint32_t s_min[4], s_max[4];
  __shared__ unsigned long long s_sum[4];
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  unsigned long long sum = 0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    const uint4 q = part[b];
    mn = min(mn, q.x);
    mx = max(mx, q.y);
    sum += (unsigned long long)q.z | ((unsigned long long)q.w << 32);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, 64));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
    sum += __shfl_xor(sum, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_min[wave] = mn;
    s_max[wave] = mx;
    s_sum[wave] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sum = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
    stats[0] = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
    stats[1] = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
    stats[2] = (uint32_t)sum;
    stats[3] = (uint32_t)(sum >> 32);
  }
}

// Keys of the visible (view, Gaussian) pairs only, in (view, Gaussian)
// order: chunk c (as in k_depth_range) writes its visible pairs from
// chunk_off[c] on.  KeyOf(v, bits) gives the key; the value is the
// Gaussian id, with the pair's tile count above bit cpack when cpack >= 0.
template <typename K, typename KeyOf>
__device__ __forceinline__ void visible_keys(int n, int ld, int V,
                                             const uint32_t* __restrict__ depth_bits,
                                             const int32_t* __restrict__ tiles,
                                             const uint32_t* __restrict__ chunk_off, KeyOf key,
                                             int cpack, K* __restrict__ keys,
                                             uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_wave[4];
  const bool vec = rows_aligned(ld, tiles, depth_bits);
  for (int v = blockIdx.y; v < V; v += gridDim.y) {
    const int32_t* tv = tiles + (size_t)v * ld;
    const uint32_t* dv = depth_bits + (size_t)v * ld;
    const uint32_t i0 = blockIdx.x * (uint32_t)kCountChunk + threadIdx.x * kCountItems;
    uint32_t c = 0, t[kCountItems], d[kCountItems];
    load_run(tv, dv, i0, n, vec, t, d);
#pragma unroll
    for (int j = 0; j < kCountItems; ++j) c += t[j] > 0 ? 1u : 0u;
    uint32_t r = chunk_off[(size_t)v * gridDim.x + blockIdx.x] +
                 block_exclusive_scan(c, s_wave, nullptr);
#pragma unroll
    for (int j = 0; j < kCountItems; ++j) {
      if (t[j] > 0) {
        keys[r] = key((uint32_t)v, d[j]);
        vals[r] = cpack >= 0 ? (i0 + j) | (t[j] << cpack) : i0 + j;
        ++r;
      }
    }
  }
}

// Zeroes zero[0, zero_n) over the whole grid (the tile ranges, cleared here
// to save a launch of their own).
__device__ __forceinline__ void grid_zero(uint32_t* __restrict__ zero, size_t zero_n) {
  const size_t nthreads = (size_t)gridDim.x * gridDim.y * kBlock;
  for (size_t z = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kBlock + threadIdx.x;
       z < zero_n; z += nthreads)
    zero[z] = 0u;
}

// 32-bit (view, depth) keys when they fit: view << vshift | (bits - min
// bits), vshift the bits of the visible depth-bit range.
__global__ __launch_bounds__(kBlock) void k_depth_keys32(int n, int ld, int V,
                                                         const uint32_t* __restrict__ depth_bits,
                                                         const int32_t* __restrict__ tiles,
                                                         const uint32_t* __restrict__ chunk_off,
                                                         uint32_t dmin, uint32_t vshift,
                                                         int cpack,
                                                         uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ vals,
                                                         uint32_t* __restrict__ zero,
                                                         size_t zero_n) {
  grid_zero(zero, zero_n);
  visible_keys<uint32_t>(
      n, ld, V, depth_bits, tiles, chunk_off,
      [=](uint32_t v, uint32_t d) { return (uint32_t)((uint64_t)v << vshift) | (d - dmin); },
      cpack, keys, vals);
}

// View of a depth-sorted key: the high word of a 64-bit key, the bits from
// vshift up of a 32-bit one.
__device__ __forceinline__ uint32_t view_of(uint64_t key, uint32_t) {
  return (uint32_t)(key >> 32);
}
__device__ __forceinline__ uint32_t view_of(uint32_t key, uint32_t vshift) {
  return (uint32_t)((uint64_t)key >> vshift);
}

// 64-bit (view << 32 | bits - min bits) keys otherwise.
__global__ __launch_bounds__(kBlock) void k_depth_keys(int n, int ld, int V,
                                                       const uint32_t* __restrict__ depth_bits,
                                                       const int32_t* __restrict__ tiles,
                                                       const uint32_t* __restrict__ chunk_off,
                                                       uint32_t dmin, int cpack,
                                                       uint64_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals,
                                                       uint32_t* __restrict__ zero,
                                                       size_t zero_n) {
  grid_zero(zero, zero_n);
  visible_keys<uint64_t>(
      n, ld, V, depth_bits, tiles, chunk_off,
      [=](uint32_t v, uint32_t d) { return ((uint64_t)v << 32) | (d - dmin); }, cpack, keys,
      vals);
}

// Instance count of each depth-sorted entry and the sums per block of
// kBlock entries: from the value's bits above cpack when the count travels
// there (cpack >= 0), else from tiles_touched (kept in cnt for the emit).
template <typename K>
__global__ __launch_bounds__(kBlock) void k_count_reduce(uint32_t N, int ld, uint32_t vshift,
                                                         const K* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals,
                                                         const int32_t* __restrict__ tiles,
                                                         int cpack, uint32_t* __restrict__ cnt,
                                                         uint32_t* __restrict__ chunk_sums) {
  __shared__ uint32_t s_wave[4];
  const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
  uint32_t c = 0;
  if (e < N) {
    if (cpack >= 0) {
      c = vals[e] >> cpack;
    } else {
      const uint32_t v = view_of(keys[e], vshift);
      c = (uint32_t)tiles[(size_t)v * ld + vals[e]];
      cnt[e] = c;
    }
  }
  uint32_t tot;
  block_exclusive_scan(c, s_wave, &tot);
  if (threadIdx.x == 0) chunk_sums[blockIdx.x] = tot;
}

// Exclusive scan of sums[0, nb) in place (one block), 64 values per thread
// per round (one round up to 16,384 values); total to *total.
__global__ __launch_bounds__(kBlock) void k_chunk_scan(uint32_t* __restrict__ sums, uint32_t nb,
                                                       uint32_t* __restrict__ total) {
  const uint32_t t = block_scan_inplace<64>(sums, nb);
  if (threadIdx.x == 0) *total = t;
}

// The end of stage 1 in one launch: block 0 reduces the chunk partials
// into stats[0..3], blocks 1 and 2 scan the visible-pair and instance
// counts per chunk (totals to stats[4] and stats[5]).
__global__ __launch_bounds__(kBlock) void k_stage1_close(const uint4* __restrict__ part,
                                                         uint32_t* __restrict__ vis,
                                                         uint32_t* __restrict__ icnt,
                                                         uint32_t nchunk,
                                                         uint32_t* __restrict__ stats) {
  if (blockIdx.x == 0) {
    stats_reduce(part, (int)nchunk, stats);
    return;
  }
  uint32_t* a = blockIdx.x == 1 ? vis : icnt;
  const uint32_t t = block_scan_inplace<64>(a, nchunk);
  if (threadIdx.x == 0) stats[3 + blockIdx.x] = t;
}

// Emit (tile of the view, Gaussian id) for each tile of each depth-sorted
// entry, row by row over its tile rectangle, or over its per-row spans when
// the record carries them (the rectangle and spans come from the record's
// words 12, 13 and 15); optionally record where each (view, Gaussian)
// starts in this order.  Each wave takes 64 consecutive entries, whose
// instances form one contiguous output range, and spreads that range over
// its lanes (instance f on lane f mod 64), so that large and small
// rectangles balance and the stores coalesce.  With pack >= 0 each
// instance is one word, tile << pack | id, in seg_out (id_out unused).
template <typename K>
__global__ __launch_bounds__(kBlock) void k_emit(uint32_t N, int ld, uint32_t vshift,
                                                 const K* __restrict__ keys,
                                                 const uint32_t* __restrict__ vals,
                                                 const uint32_t* __restrict__ cnt, int cpack,
                                                 const uint32_t* __restrict__ chunk_off,
                                                 const int32_t* __restrict__ txv,
                                                 uint32_t* __restrict__ seg_out,
                                                 uint32_t* __restrict__ id_out,
                                                 uint32_t* __restrict__ gv_base,
                                                 uint32_t* __restrict__ splat_words,
                                                 int pack) {
  __shared__ uint32_t s_pre[4][64];
  __shared__ uint32_t s_seg0[4][64];  // the rectangle's first tile in its view
  __shared__ uint32_t s_id[4][64];
  __shared__ uint32_t s_w[4][64];     // rectangle width in tiles | kSpanFlag
  __shared__ uint32_t s_sp[4][64];    // per-row spans (record word 15)
  __shared__ uint32_t s_row[4][64];   // tiles per view row
  __shared__ uint32_t s_bwave[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
  uint32_t c = 0, g = 0;
  if (e < N) {
    const uint32_t w = vals[e];
    if (cpack >= 0) {
      c = w >> cpack;
      g = w & ((1u << cpack) - 1u);
    } else {
      c = cnt[e];
      g = w;
    }
  }
  // this entry's first instance: the block's offset + the scan inside it
  const uint32_t o0 = chunk_off[blockIdx.x] + block_exclusive_scan(c, s_bwave, nullptr);
  if (e < N) {
    if (c > 0) {
      const uint32_t v = view_of(keys[e], vshift);
      uint32_t* rw = splat_words + ((size_t)v * ld + g) * (4 * kSplatF4) + 12;
      const uint4 q3 = *reinterpret_cast<const uint4*>(rw);  // o, w | flag, e, spans
      const uint32_t tx = (uint32_t)txv[v];
      s_seg0[wave][lane] = (q3.x >> 16) * tx + (q3.x & 0xFFFFu);
      s_id[wave][lane] = g;
      s_w[wave][lane] = q3.y;
      s_sp[wave][lane] = q3.w;
      s_row[wave][lane] = tx;
      if (gv_base) gv_base[(size_t)v * ld + g] = o0;
      // record word 14: this pair's first instance in emission order
      rw[2] = o0;
    }
  }
  // the wave's entries own output [first, first + total)
  uint32_t incl = c;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  const uint32_t first = __shfl(o0, 0, 64);
  s_pre[wave][lane] = incl - c;
  __syncthreads();
  for (uint32_t f = lane; f < total; f += 64) {
    int q = 0;  // last entry whose first instance is <= f (it has one)
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
      if (s_pre[wave][q + step] <= f) q += step;
    const uint32_t l = f - s_pre[wave][q];
    const uint32_t w = s_w[wave][q];
    uint32_t dy, dx;
    if (w & kSpanFlag) {
      // spans s_r = b_r - a_r per byte; instances before row r: p_r
      const uint32_t m = s_sp[wave][q];
      const uint32_t sp = ((m >> 4) & 0x0F0F0F0Fu) - (m & 0x0F0F0F0Fu);
      const uint32_t p1 = sp & 0xFFu, p2 = p1 + ((sp >> 8) & 0xFFu),
                     p3 = p2 + ((sp >> 16) & 0xFFu);
      dy = (uint32_t)(l >= p1) + (uint32_t)(l >= p2) + (uint32_t)(l >= p3);
      const uint32_t pre = dy == 0 ? 0u : (dy == 1 ? p1 : (dy == 2 ? p2 : p3));
      dx = ((m >> (8 * dy)) & 15u) + (l - pre);
    } else {
      dy = l / w;
      dx = l - dy * w;
    }
    const uint32_t tile = s_seg0[wave][q] + dy * s_row[wave][q] + dx;
    if (pack >= 0) {
      seg_out[first + f] = (tile << pack) | s_id[wave][q];
    } else {
      seg_out[first + f] = tile;
      id_out[first + f] = s_id[wave][q];
    }
  }
}

// Segment boundaries of the sorted segment ids, four per thread (one 16-B
// load; the neighbours across the thread's group come from the adjacent
// lanes, or from memory at the wave's edges).
__global__ __launch_bounds__(kBlock) void k_ranges(uint32_t M, const uint32_t* __restrict__ seg,
                                                   uint32_t* __restrict__ ranges) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t j0 = 4 * t;
  const int lane = threadIdx.x & 63;
  uint32_t s[4] = {0u, 0u, 0u, 0u};
  if (j0 + 3 < M) {
    const uint4 q = *reinterpret_cast<const uint4*>(seg + j0);
    s[0] = q.x; s[1] = q.y; s[2] = q.z; s[3] = q.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (j0 + i < M) s[i] = seg[j0 + i];
  }
  uint32_t prev = (uint32_t)__shfl_up((int)s[3], 1, 64);
  uint32_t next = (uint32_t)__shfl_down((int)s[0], 1, 64);
  if (lane == 0 && j0 > 0 && j0 - 1 < M) prev = seg[j0 - 1];
  if (lane == 63 && j0 + 4 < M) next = seg[j0 + 4];
  if (j0 >= M) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t j = j0 + i;
    if (j >= M) break;
    const uint32_t before = i == 0 ? prev : s[i - 1];
    const uint32_t after = i == 3 ? next : s[i + 1];
    if (j == 0 || before != s[i]) ranges[2 * (size_t)s[i]] = j;
    if (j == M - 1 || after != s[i]) ranges[2 * (size_t)s[i] + 1] = j + 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_keys64(uint32_t M, int V, int ld,
                                                   const uint32_t* __restrict__ seg,
                                                   const uint32_t* __restrict__ ids,
                                                   const uint32_t* __restrict__ seg_base,
                                                   const uint32_t* __restrict__ depth_bits,
                                                   uint64_t* __restrict__ keys) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= M) return;
  const uint32_t s = seg[j];
  int lo = 0, hi = V - 1;  // last view whose base <= s
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_base[mid] <= s) lo = mid; else hi = mid - 1;
  }
  keys[j] = ((uint64_t)s << 32) | depth_bits[(size_t)lo * ld + ids[j]];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_f32(float* p, float value, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ------------------------------------------------------------ host side
inline int bits_for(uint64_t count) {  // bits to hold values 0 .. count-1
  int b = 0;
  while (b < 64 && ((uint64_t)1 << b) < count) ++b;
  return b;
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Fewest passes with digits of 8 or 9 bits (wider digits cost more per pass
// than they save).
struct DigitPlan {
  int passes;
  int bits;
};
inline DigitPlan plan_digits(int key_bits) {
  if (key_bits <= 0) return {0, 8};
  const int passes = (key_bits + 8) / 9;
  int b = (key_bits + passes - 1) / passes;
  if (b < 8) b = 8;
  return {passes, b};
}
inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

struct Layout {
  size_t dk0, dk1, dv0, dv1, cnt, chunks, segk0, segk1, segv_alt, pcount, dtotal,
      pfirst, pdesc, dparts, vparts, iparts, seg_base, txv, total, stats, bytes;
};

// Bound on the partitions of n keys cut per view (at most one partial
// partition per view).
inline size_t max_parts(size_t n, int V) { return (size_t)cdiv(n, kPart) + (size_t)V; }

Layout make_layout(int V, int ld, int64_t cap, int64_t nseg) {
  (void)nseg;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t N = (size_t)V * (size_t)ld;
  const size_t pmax = max_parts(std::max(N, (size_t)cap), V);
  constexpr size_t kMaxDigits = 512;
  L.dk0 = take(N * 8);
  L.dk1 = take(N * 8);
  L.dv0 = take(N * 4);
  L.dv1 = take(N * 4);
  L.cnt = take(N * 4);
  L.chunks = take(((size_t)cdiv(N, kBlock) + 1) * 4);
  L.segk0 = take((size_t)cap * 4);
  L.segk1 = take((size_t)cap * 4);
  L.segv_alt = take((size_t)cap * 4);
  // per-partition digit counts of one pass (reused by every pass), the row
  // totals, the partition table
  L.pcount = take(kMaxDigits * pmax * 4);
  L.dtotal = take(kMaxDigits * 4);
  L.pfirst = take(((size_t)V + 1) * 4);
  L.pdesc = take(pmax * 16);
  L.seg_base = take(((size_t)V + 1) * 4);
  L.txv = take((size_t)V * 4);
  L.total = take(16);
  // {min bits, max bits, instances lo, hi, visible pairs, instances (low
  // word, scanned)}
  L.stats = take(32);
  const size_t nchunk = (size_t)V * cdiv((uint64_t)ld, kCountChunk);
  L.dparts = take(nchunk * 16);
  L.vparts = take((nchunk + 1) * 4);
  L.iparts = take((nchunk + 1) * 4);
  L.bytes = o;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Where each view's elements start: vstart[v * vstride] for v < V (the
// chunk scans of stage 1 with stride = chunks per view), n for v = V.
struct ViewStarts {
  const uint32_t* vstart;
  uint32_t vstride;
  int V;
};

// Stable LSD radix sort of (key, value) pairs inside each view on bits
// [shift0, shift0 + BITS * passes), ping-pong between buffer pair 0 and 1.
// First the partition table (none with one view), then per digit pass:
// per-partition digit counts, their exclusive scan per digit over the
// partitions, and the ranking + scatter, which forms its view's digit
// starts from the scanned counts.  Without values
// (v0 == NULL) the keys carry them in their low bits and the last pass
// splits them: key >> shift0 to the key buffer, key & (2^shift0 - 1) to
// vout_last.  add_last (optional): added per view to the keys the last pass
// writes.
struct SortSpec {
  int shift0;
  const uint32_t* add_last;
  uint32_t* vout_last;  // keys-only sorts
};

template <typename K, int BITS>
void radix_passes(K* k0, K* k1, uint32_t* v0, uint32_t* v1, uint32_t n, int passes,
                  const ViewStarts& vs, const SortSpec& sp, void* ws, const Layout& L,
                  hipStream_t s) {
  constexpr int R = 1 << BITS;
  uint32_t* cnt = at<uint32_t>(ws, L.pcount);
  uint32_t* tot = at<uint32_t>(ws, L.dtotal);
  uint32_t* pfirst = at<uint32_t>(ws, L.pfirst);
  uint4* desc = at<uint4>(ws, L.pdesc);
  // one view: partitions follow from their index, no table to build, and
  // the scatter scans the digit totals itself
  const bool one = vs.V == 1;
  const uint32_t pmax = one ? cdiv(n, kPart) : (uint32_t)max_parts(n, vs.V);
  const uint32_t grid = (pmax + 7) / 8 * 8;  // whole XCD rounds
  const PartTable pt{one ? nullptr : desc, one ? nullptr : pfirst, n, vs.V};
  if (!one) {
    hipLaunchKernelGGL(k_part_first, dim3(1), dim3(kBlock), 0, s, vs.vstart, vs.vstride, vs.V, n,
                       pfirst);
    hipLaunchKernelGGL(k_part_desc, dim3(cdiv(pmax, kBlock)), dim3(kBlock), 0, s, vs.vstart,
                       vs.vstride, vs.V, n, pfirst, desc);
  }
  K* kb[2] = {k0, k1};
  uint32_t* vb[2] = {v0, v1};
  const uint32_t umask = sp.shift0 >= 32 ? ~0u : ((1u << sp.shift0) - 1u);
  for (int p = 0; p < passes; ++p) {
    const int src = p & 1;
    const int shift = sp.shift0 + BITS * p;
    const bool last = p == passes - 1;
    hipLaunchKernelGGL((k_part_count<K, BITS>), dim3(grid), dim3(kBlock), 0, s, kb[src], shift,
                       pmax, pt, cnt);
    hipLaunchKernelGGL(k_part_scan_rows, dim3(R), dim3(kBlock), 0, s, cnt, pmax, pt, tot);
    const uint32_t* add = last ? sp.add_last : nullptr;
    if (v0)
      hipLaunchKernelGGL((k_scatter_pass<K, BITS, true>), dim3(grid), dim3(kBlock), 0, s,
                         kb[src], vb[src], kb[src ^ 1], vb[src ^ 1], shift, pmax, pt, cnt, tot,
                         add, 0, 0u);
    else
      hipLaunchKernelGGL((k_scatter_pass<K, BITS, false>), dim3(grid), dim3(kBlock), 0, s,
                         kb[src], nullptr, kb[src ^ 1], last ? sp.vout_last : nullptr, shift,
                         pmax, pt, cnt, tot, add, sp.shift0, umask);
  }
}

// Returns which key buffer holds the result (0 or 1).
template <typename K>
int radix_sort(K* k0, K* k1, uint32_t* v0, uint32_t* v1, uint32_t n, int bits,
               const ViewStarts& vs, const SortSpec& sp, void* ws, const Layout& L,
               hipStream_t s) {
  const DigitPlan dp = plan_digits(bits);
  if (n == 0 || dp.passes == 0) return 0;
  switch (dp.bits) {
    case 8: radix_passes<K, 8>(k0, k1, v0, v1, n, dp.passes, vs, sp, ws, L, s); break;
    default: radix_passes<K, 9>(k0, k1, v0, v1, n, dp.passes, vs, sp, ws, L, s); break;
  }
  return dp.passes & 1;
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t want = (count + 255) / 256;
  const int blocks = (int)std::min<int64_t>(want, 4096);
  StageScope scope(kStFill, s);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, value, (size_t)count);
}

void launch_fill_f32(float* p, float value, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t want = (count + 255) / 256;
  const int blocks = (int)std::min<int64_t>(want, 4096);
  StageScope scope(kStFill, s);
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, s, p, value, (size_t)count);
}

size_t bin_sort_workspace_bytes(int V, int ld, int64_t cap, int64_t nseg) {
  return make_layout(V, ld, cap, nseg).bytes;
}

hipError_t bin_sort_stage1(const BinSortPlan& p, const gs_projected& proj,
                           const gs_camera* cams_dev, void* ws, hipStream_t s,
                           uint32_t** d_stats) {
  const Layout L = make_layout(p.n_views, p.ld, p.capacity, p.n_segments);
  const uint32_t N = (uint32_t)p.n_views * (uint32_t)p.n;
  uint32_t* stats = at<uint32_t>(ws, L.stats);
  *d_stats = stats;
  hipLaunchKernelGGL(k_view_info, dim3(1), dim3(kBlock), 0, s, cams_dev, p.n_views,
                     at<uint32_t>(ws, L.seg_base), at<int32_t>(ws, L.txv), stats);
  if (N == 0) return hipGetLastError();
  StageScope scope(kStDepthSort, s);
  // chunks of kCountChunk Gaussians per view; views on grid rows (beyond
  // 65535 they loop)
  const uint32_t gx = cdiv((uint64_t)p.n, kCountChunk);
  const uint32_t gy = std::min<uint32_t>((uint32_t)p.n_views, 65535u);
  const uint32_t nchunk = gx * (uint32_t)p.n_views;
  uint4* part = at<uint4>(ws, L.dparts);
  uint32_t* vis = at<uint32_t>(ws, L.vparts);
  uint32_t* icnt = at<uint32_t>(ws, L.iparts);
  hipLaunchKernelGGL(k_depth_range, dim3(gx, gy), dim3(kBlock), 0, s, p.n, p.ld, p.n_views,
                     proj.depth_bits, proj.tiles_touched, part, vis, icnt);
  // the depth-bit range and instance count (stats[0..3]); where each
  // chunk's visible pairs go in the depth sort's input (stats[4] = their
  // number), and where each chunk's instances start in emission order,
  // which keeps the views in order (only read once the host has checked
  // that the total fits 32 bits)
  hipLaunchKernelGGL(k_stage1_close, dim3(3), dim3(kBlock), 0, s, part, vis, icnt, nchunk, stats);
  return hipGetLastError();
}

namespace {
// Depth sort of the (view, Gaussian) pairs with keys K inside each view on
// their dbits low bits, instance offsets and emission into (segk0, v0), or
// packed into segk0 alone with pack >= 0; vshift is where a 32-bit key's
// view starts; with cpack >= 0 each pair's tile count rides above bit
// cpack of its value through the sort.  The key gather also clears
// ranges[0, 2 n_segments).
template <typename K>
void depth_count_emit(const BinSortPlan& p, const gs_projected& proj, const Layout& L, void* ws,
                      uint32_t N, uint32_t dmin, uint32_t vshift, int dbits, int cpack,
                      uint32_t* segk0, uint32_t* v0, int pack, uint32_t* gv_base,
                      uint32_t* ranges, hipStream_t s) {
  K* k0 = at<K>(ws, L.dk0);
  K* k1 = at<K>(ws, L.dk1);
  uint32_t* dv0 = at<uint32_t>(ws, L.dv0);
  uint32_t* dv1 = at<uint32_t>(ws, L.dv1);
  int which;
  {
    StageScope scope(kStDepthSort, s);
    // keys of the visible pairs only (the chunk offsets from stage 1)
    const dim3 key_grid(cdiv((uint64_t)p.n, kCountChunk),
                        std::min<uint32_t>((uint32_t)p.n_views, 65535u));
    const uint32_t* vis_off = at<uint32_t>(ws, L.vparts);
    if constexpr (sizeof(K) == 4)
      hipLaunchKernelGGL(k_depth_keys32, key_grid, dim3(kBlock), 0, s, p.n, p.ld, p.n_views,
                         proj.depth_bits, proj.tiles_touched, vis_off, dmin, vshift, cpack, k0,
                         dv0, ranges, (size_t)2 * (size_t)p.n_segments);
    else
      hipLaunchKernelGGL(k_depth_keys, key_grid, dim3(kBlock), 0, s, p.n, p.ld, p.n_views,
                         proj.depth_bits, proj.tiles_touched, vis_off, dmin, cpack, k0, dv0,
                         ranges, (size_t)2 * (size_t)p.n_segments);
    const ViewStarts vs{vis_off, key_grid.x, p.n_views};
    which = radix_sort<K>(k0, k1, dv0, dv1, N, dbits, vs, SortSpec{0, nullptr, nullptr}, ws, L,
                          s);
  }
  const K* sk = which ? k1 : k0;
  const uint32_t* sv = which ? dv1 : dv0;
  uint32_t* cnt = at<uint32_t>(ws, L.cnt);
  uint32_t* chunks = at<uint32_t>(ws, L.chunks);
  const uint32_t nch = cdiv(N, kBlock);
  {
    // instance counts per block of kBlock entries and their scan; the emit
    // finishes the offsets inside its block
    StageScope scope(kStCountScan, s);
    hipLaunchKernelGGL((k_count_reduce<K>), dim3(nch), dim3(kBlock), 0, s, N, p.ld, vshift, sk,
                       sv, proj.tiles_touched, cpack, cnt, chunks);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kBlock), 0, s, chunks, nch,
                       at<uint32_t>(ws, L.total));
  }
  StageScope scope(kStEmit, s);
  hipLaunchKernelGGL((k_emit<K>), dim3(nch), dim3(kBlock), 0, s, N, p.ld, vshift, sk, sv, cnt,
                     cpack, chunks, at<int32_t>(ws, L.txv), segk0, v0, gv_base,
                     reinterpret_cast<uint32_t*>(proj.splat), pack);
}
}  // namespace

hipError_t bin_sort_stage2(const BinSortPlan& p, const gs_projected& proj,
                           const gs_camera* cams_dev, uint32_t M, uint32_t dmin, uint32_t dmax,
                           uint32_t N, gs_tile_lists& lists, void* ws, hipStream_t s) {
  (void)cams_dev;
  const Layout L = make_layout(p.n_views, p.ld, p.capacity, p.n_segments);
  if (M == 0) {
    launch_fill_u32(lists.ranges, 0u, 2 * p.n_segments, s);
    return hipGetLastError();
  }
  // the tile sort runs inside each view on the bits of its tile index (at
  // least one pass: the last one turns tile indices into segment ids)
  const int sbits = std::max(1, bits_for((uint64_t)p.max_tiles));
  const int spasses = plan_digits(sbits).passes;
  uint32_t* segk0 = at<uint32_t>(ws, L.segk0);
  uint32_t* segk1 = at<uint32_t>(ws, L.segk1);
  uint32_t* alt = at<uint32_t>(ws, L.segv_alt);
  // when a tile index and a Gaussian id fit one word together, the emit
  // writes tile << idbits | id and the tile sort moves those words only
  // (the last pass splits them); otherwise keys and ids move side by side,
  // emitted into the buffer that makes the sorted ids land in lists.vals
  const int idbits = bits_for((uint64_t)p.ld);
  const bool packed = idbits + sbits <= 32;
  uint32_t* v0 = packed ? nullptr : ((spasses & 1) ? alt : lists.vals);
  uint32_t* v1 = packed ? nullptr : ((spasses & 1) ? lists.vals : alt);
  const int pack = packed ? idbits : -1;
  // likewise each pair's tile count (at most the largest view's tiles) rides
  // above its Gaussian id through the depth sort when both fit one word
  const int cpack = idbits + bits_for((uint64_t)p.max_tiles + 1u) <= 32 ? idbits : -1;
  // the depth sort runs inside each view on the bits of the visible depth
  // range; (view, depth) keys are 32-bit when the views fit above those bits
  // (M > 0 means some pair is visible, so dmax >= dmin); only the N visible
  // pairs are sorted
  const int dbits = bits_for((uint64_t)dmax - (uint64_t)dmin + 1u);
  if (((uint64_t)p.n_views << dbits) <= ((uint64_t)1 << 32))
    depth_count_emit<uint32_t>(p, proj, L, ws, N, dmin, (uint32_t)dbits, dbits, cpack, segk0,
                               v0, pack, lists.gv_base, lists.ranges, s);
  else
    depth_count_emit<uint64_t>(p, proj, L, ws, N, dmin, 32u, dbits, cpack, segk0, v0, pack,
                               lists.gv_base, lists.ranges, s);
  int which2;
  {
    StageScope scope(kStSegmentSort, s);
    const ViewStarts vs{at<uint32_t>(ws, L.iparts), cdiv((uint64_t)p.n, kCountChunk), p.n_views};
    const SortSpec sp{packed ? idbits : 0, at<uint32_t>(ws, L.seg_base),
                      packed ? lists.vals : nullptr};
    which2 = radix_sort<uint32_t>(segk0, segk1, v0, v1, M, sbits, vs, sp, ws, L, s);
  }
  const uint32_t* seg_sorted = which2 ? segk1 : segk0;
  StageScope scope(kStRanges, s);
  hipLaunchKernelGGL(k_ranges, dim3(cdiv(cdiv(M, 4u), kBlock)), dim3(kBlock), 0, s, M,
                     seg_sorted, lists.ranges);
  if (lists.keys)
    hipLaunchKernelGGL(k_keys64, dim3(cdiv(M, kBlock)), dim3(kBlock), 0, s, M, p.n_views, p.ld,
                       seg_sorted, lists.vals, at<uint32_t>(ws, L.seg_base), proj.depth_bits,
                       lists.keys);
  return hipGetLastError();
}

}  // namespace gs
