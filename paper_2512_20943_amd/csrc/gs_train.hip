// Training support, all elementwise and HBM-bound: the L1 photometric term
// (AirGS Eq. (1)), the squared error behind the pruning sweep's PSNR
// (Sec. III-C), the keyframe temporal term (Eq. (9)) and the Adam update
// (Kingma & Ba 2015).
#include "gs_internal.h"

namespace gs {
namespace {

// grad = sign(I - I*) / count; per-block FP64 partial sums of |I - I*| are
// reduced across the wave with shuffles and added to *loss once per block.
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ img,
                                            const float* __restrict__ tgt, int64_t count,
                                            float inv_count, float* __restrict__ grad,
                                            double* __restrict__ loss) {
  __shared__ double s_w[4];
  double acc = 0.0;
  // four values per step with 16-byte accesses when the three buffers allow
  // it (the tail and unaligned buffers go one value at a time)
  const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                     reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
  const int64_t n4 = vec ? count / 4 : 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += stride) {
    const float4 a = reinterpret_cast<const float4*>(img)[q];
    const float4 b = reinterpret_cast<const float4*>(tgt)[q];
    const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
    acc += ((double)fabsf(d0) + (double)fabsf(d1)) + ((double)fabsf(d2) + (double)fabsf(d3));
    reinterpret_cast<float4*>(grad)[q] =
        make_float4(d0 > 0.f ? inv_count : (d0 < 0.f ? -inv_count : 0.f),
                    d1 > 0.f ? inv_count : (d1 < 0.f ? -inv_count : 0.f),
                    d2 > 0.f ? inv_count : (d2 < 0.f ? -inv_count : 0.f),
                    d3 > 0.f ? inv_count : (d3 < 0.f ? -inv_count : 0.f));
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
    const float d = img[i] - tgt[i];
    acc += (double)fabsf(d);
    grad[i] = d > 0.f ? inv_count : (d < 0.f ? -inv_count : 0.f);
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_w[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) / (double)count);
}

// Sum of squared differences: per-block FP64 partials, one atomic per block
// (at most 1024 blocks, since those atomics serialise on the one address);
// four values per step with 16-byte loads when both buffers allow it.
__global__ __launch_bounds__(256) void k_sq_error(const float* __restrict__ a,
                                                  const float* __restrict__ b, int64_t count,
                                                  double* __restrict__ sum) {
  __shared__ double s_w[4];
  double acc = 0.0;
  const bool vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
  const int64_t n4 = vec ? count / 4 : 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += stride) {
    const float4 x = reinterpret_cast<const float4*>(a)[q];
    const float4 y = reinterpret_cast<const float4*>(b)[q];
    const double d0 = (double)x.x - (double)y.x, d1 = (double)x.y - (double)y.y,
                 d2 = (double)x.z - (double)y.z, d3 = (double)x.w - (double)y.w;
    acc += (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
    const double d = (double)a[i] - (double)b[i];
    acc += d * d;
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_w[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(sum, (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]));
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t count, float lr, float b1, float b2,
                                              float eps, float ibc1, float ibc2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * ibc1) / (sqrtf(vi * ibc2) + eps);
  }
}

// Keyframe temporal term (Eq. (9), weight of Eq. (10)): over `rows` planes
// of stride ld and the first `bound` columns, grad += w * sign(x - x_prev)
// and w * sum |x - x_prev| added to *loss.
__global__ __launch_bounds__(256) void k_l1_penalty(const float* __restrict__ x,
                                                    const float* __restrict__ ref, int rows,
                                                    int bound, int64_t ld, float w,
                                                    float* __restrict__ grad,
                                                    double* __restrict__ loss) {
  __shared__ double s_w[4];
  double acc = 0.0;
  const int64_t total = (int64_t)rows * bound;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * 256) {
    const int64_t r = k / bound, c = k - r * bound;
    const int64_t i = r * ld + c;
    const float d = x[i] - ref[i];
    acc += (double)fabsf(d);
    grad[i] += d > 0.f ? w : (d < 0.f ? -w : 0.f);
  }
  if (!loss) return;
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_w[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (double)w * ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])));
}

inline int grid_for(int64_t count) {
  const int64_t want = (count + 255) / 256;
  return (int)(want < 8192 ? want : 8192);
}

}  // namespace

void launch_l1(const float* image, const float* target, int64_t count, float* grad, double* loss,
               hipStream_t s) {
  if (count <= 0) return;
  StageScope scope(kStL1, s);
  // at most 1024 blocks: each adds its partial to *loss with one device-wide
  // atomic, and those serialise on the one address
  const int blocks = std::min(grid_for(count), 1024);
  hipLaunchKernelGGL(k_l1, dim3(blocks), dim3(256), 0, s, image, target, count,
                     (float)(1.0 / (double)count), grad, loss);
}

void launch_sq_error(const float* a, const float* b, int64_t count, double* sum, hipStream_t s) {
  if (count <= 0) return;
  StageScope scope(kStL1, s);
  const int blocks = std::min(grid_for(count), 1024);
  hipLaunchKernelGGL(k_sq_error, dim3(blocks), dim3(256), 0, s, a, b, count, sum);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t s) {
  if (count <= 0) return;
  StageScope scope(kStAdam, s);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(count)), dim3(256), 0, s, p, g, m, v, count, lr, b1,
                     b2, eps, 1.f / bc1, 1.f / bc2);
}

void launch_l1_penalty(const float* x, const float* ref, int rows, int bound, int64_t ld, float w,
                       float* grad, double* loss, hipStream_t s) {
  const int64_t total = (int64_t)rows * bound;
  if (total <= 0) return;
  StageScope scope(kStL1, s);
  hipLaunchKernelGGL(k_l1_penalty, dim3(grid_for(total)), dim3(256), 0, s, x, ref, rows, bound, ld,
                     w, grad, loss);
}

}  // namespace gs
