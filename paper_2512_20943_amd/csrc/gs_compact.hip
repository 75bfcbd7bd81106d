// Low-opacity culling for keyframe reconstruction (AirGS Sec. III-B: the
// Gaussians whose opacity has fallen below a threshold are discarded during
// training) as an order-preserving stream compaction, and the gather that
// applies the resulting index list to parameter or optimizer-state planes.
//
// Compaction in three launches over chunks of 1024 Gaussians: count the kept
// ones per chunk, scan the chunk counts in one workgroup, then rank inside
// each chunk with wave ballots and write the kept indices in their original
// order.  HBM-bound: 4 B read twice and at most 4 B written per Gaussian.
#include <cmath>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kChunk = 1024;  // Gaussians per workgroup (256 threads x 4)

__device__ __forceinline__ bool kept(const float* logit, int i, int n, double thr) {
  return i < n && (double)logit[i] >= thr;
}

__global__ __launch_bounds__(256) void k_keep_count(const float* __restrict__ logit, int n,
                                                    double thr, uint32_t* __restrict__ counts) {
  const int base = blockIdx.x * kChunk;
  int c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) c += kept(logit, base + k * 256 + threadIdx.x, n, thr) ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  __shared__ int s[4];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (uint32_t)(s[0] + s[1] + s[2] + s[3]);
}

// Exclusive scan of nb chunk counts in one workgroup of 1024 threads; the
// total goes to counts[nb].
__global__ __launch_bounds__(1024) void k_keep_scan(uint32_t* __restrict__ counts, int nb) {
  __shared__ uint32_t s_wave[16];
  __shared__ uint32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? counts[i] : 0u;
    uint32_t x = v;  // inclusive scan inside the wave
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = s_carry;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    if (i < nb) counts[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[nb] = s_carry;
}

__global__ __launch_bounds__(256) void k_keep_write(const float* __restrict__ logit, int n,
                                                    double thr,
                                                    const uint32_t* __restrict__ offsets,
                                                    int32_t* __restrict__ index) {
  __shared__ uint32_t s_cnt[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = blockIdx.x * kChunk;
  // pass k covers Gaussians base + k*256 + [0, 256): 4 waves of 64, so the
  // rank of a lane is (waves of earlier passes) + (earlier waves of this
  // pass) + (earlier lanes of its own wave)
  bool f[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[k] = kept(logit, base + k * 256 + threadIdx.x, n, thr);
    const uint64_t b = __ballot(f[k]);
    if (lane == 0) s_cnt[k * 4 + wave] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t run = offsets[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t b = __ballot(f[k]);
    uint32_t pre = run;
    for (int w = 0; w < wave; ++w) pre += s_cnt[k * 4 + w];
    if (f[k]) index[pre + (uint32_t)__popcll(b & below)] = base + k * 256 + threadIdx.x;
    for (int w = 0; w < 4; ++w) run += s_cnt[k * 4 + w];
  }
}

__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ src, int64_t src_ld,
                                                int planes, const int32_t* __restrict__ index,
                                                int m, float* __restrict__ dst, int64_t dst_ld) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = index[j];
  for (int p = 0; p < planes; ++p) dst[p * dst_ld + j] = src[p * src_ld + i];
}

}  // namespace

size_t keep_workspace_bytes(int n) {
  const size_t nb = ((size_t)n + kChunk - 1) / kChunk;
  return (nb + 1) * sizeof(uint32_t);
}

double opacity_logit_threshold(float min_opacity) {
  const double m = (double)min_opacity;
  return std::log(m / (1.0 - m));
}

const uint32_t* launch_keep_low_opacity(const float* logit, int n, double thr, int32_t* index,
                                        void* ws, hipStream_t s) {
  const int nb = (n + kChunk - 1) / kChunk;
  uint32_t* counts = static_cast<uint32_t*>(ws);
  StageScope scope(kStCompact, s);
  if (nb > 0) hipLaunchKernelGGL(k_keep_count, dim3(nb), dim3(256), 0, s, logit, n, thr, counts);
  hipLaunchKernelGGL(k_keep_scan, dim3(1), dim3(1024), 0, s, counts, nb);
  if (nb > 0)
    hipLaunchKernelGGL(k_keep_write, dim3(nb), dim3(256), 0, s, logit, n, thr,
                       (const uint32_t*)counts, index);
  return counts + nb;  // the total number kept
}

void launch_gather(const float* src, int64_t src_ld, int planes, const int32_t* index, int m,
                   float* dst, int64_t dst_ld, hipStream_t s) {
  if (m <= 0 || planes <= 0) return;
  StageScope scope(kStCompact, s);
  hipLaunchKernelGGL(k_gather, dim3((m + 255) / 256), dim3(256), 0, s, src, src_ld, planes, index,
                     m, dst, dst_ld);
}

}  // namespace gs
