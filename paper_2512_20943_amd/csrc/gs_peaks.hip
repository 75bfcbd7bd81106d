// Peak-rate probes for the roofline: HBM copy and read bandwidth, LDS read
// bandwidth, FP32 FMA and exp2 issue rates, and float atomic throughput.
// Each kernel does a known amount of work with no dependence on the data
// beyond keeping the compiler from removing it; gs_peak_run times one launch
// with HIP events.  Built with the same flags as the rest of the library
// (no packed FP32 instructions), so the FMA probe measures what the render
// kernels can issue.
#include "gs_internal.h"

namespace gs {
namespace {

// out = in, float4 per thread per step, grid-stride.
__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ in,
                                                   float4* __restrict__ out, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    out[i] = in[i];
}

// Sum of the input, four float4 loads in flight per thread; one float per
// thread written so that the loads are kept.
__global__ __launch_bounds__(256) void k_peak_read(const float4* __restrict__ in, size_t n4,
                                                   float* __restrict__ sink) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a, d = a;
  size_t i = t;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 x = in[i], y = in[i + stride], z = in[i + 2 * stride], w = in[i + 3 * stride];
    a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
    b.x += y.x; b.y += y.y; b.z += y.z; b.w += y.w;
    c.x += z.x; c.y += z.y; c.z += z.z; c.w += z.w;
    d.x += w.x; d.y += w.y; d.z += w.z; d.w += w.w;
  }
  for (; i < n4; i += stride) {
    const float4 x = in[i];
    a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
  }
  sink[t] = (a.x + a.y + a.z + a.w) + (b.x + b.y + b.z + b.w) + (c.x + c.y + c.z + c.w) +
            (d.x + d.y + d.z + d.w);
}

// LDS reads: each lane reads consecutive 16-B words (conflict-free), 4096
// float4 (64 KB) per workgroup, `iters` sweeps.
constexpr int kLdsF4 = 4096;
__global__ __launch_bounds__(256) void k_peak_lds(int iters, float* __restrict__ sink) {
  __shared__ float4 buf[kLdsF4];
  for (int i = threadIdx.x; i < kLdsF4; i += 256)
    buf[i] = make_float4((float)i, 1.f, 2.f, 3.f);
  __syncthreads();
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kLdsF4 / 256; k += 2) {
      const float4 x = buf[(k * 256 + threadIdx.x + it) & (kLdsF4 - 1)];
      const float4 y = buf[((k + 1) * 256 + threadIdx.x + it) & (kLdsF4 - 1)];
      a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
      b.x += y.x; b.y += y.y; b.z += y.z; b.w += y.w;
    }
  }
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] =
      (a.x + a.y + a.z + a.w) + (b.x + b.y + b.z + b.w);
}

// FP32 FMAs: 16 independent chains per lane, `iters` rounds of 16 FMAs.
__global__ __launch_bounds__(256) void k_peak_fma(int iters, float s, float* __restrict__ sink) {
  float v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = (float)(threadIdx.x + k) * 1e-3f;
  const float m = 0.999f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = fmaf(v[k], m, s);
  }
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) acc += v[k];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// exp2: 8 independent chains per lane, x <- exp2(-x) stays in (0, 1].
__global__ __launch_bounds__(256) void k_peak_exp(int iters, float* __restrict__ sink) {
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = (float)((threadIdx.x + k) & 7) * 0.1f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_exp2f(-v[k]);
  }
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += v[k];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Float atomic adds without return: thread t adds to dst[t mod n_addr],
// `iters` times.
__global__ __launch_bounds__(256) void k_peak_atomic(float* __restrict__ dst, uint32_t n_addr,
                                                     int iters) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float* p = dst + (t % n_addr);
  for (int it = 0; it < iters; ++it) atomicAdd(p, 1.f);
}

}  // namespace

hipError_t launch_peak(int kind, void* buf, size_t bytes, int iters, double* work,
                       hipStream_t s) {
  const int blocks = 256 * 16;  // 16 workgroups of 256 threads per CU
  switch (kind) {
    case GS_PEAK_COPY: {
      const size_t n4 = bytes / 2 / sizeof(float4);
      const float4* in = static_cast<const float4*>(buf);
      hipLaunchKernelGGL(k_peak_copy, dim3(blocks), dim3(256), 0, s, in,
                         const_cast<float4*>(in) + n4, n4);
      *work = 2.0 * (double)n4 * sizeof(float4);
      break;
    }
    case GS_PEAK_READ: {
      const size_t sink_bytes = (size_t)blocks * 256 * sizeof(float);
      const size_t n4 = (bytes - sink_bytes) / sizeof(float4);
      float* sink = reinterpret_cast<float*>(static_cast<char*>(buf) + n4 * sizeof(float4));
      hipLaunchKernelGGL(k_peak_read, dim3(blocks), dim3(256), 0, s,
                         static_cast<const float4*>(buf), n4, sink);
      *work = (double)n4 * sizeof(float4);
      break;
    }
    case GS_PEAK_LDS:
      hipLaunchKernelGGL(k_peak_lds, dim3(blocks), dim3(256), 0, s, iters,
                         static_cast<float*>(buf));
      *work = (double)blocks * 256 * (double)iters * (kLdsF4 / 256) * sizeof(float4);
      break;
    case GS_PEAK_FMA:
      hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(256), 0, s, iters, 1e-3f,
                         static_cast<float*>(buf));
      *work = (double)blocks * 256 * (double)iters * 16.0 * 2.0;  // FLOP, FMA = 2
      break;
    case GS_PEAK_EXP:
      hipLaunchKernelGGL(k_peak_exp, dim3(blocks), dim3(256), 0, s, iters,
                         static_cast<float*>(buf));
      *work = (double)blocks * 256 * (double)iters * 8.0;
      break;
    case GS_PEAK_ATOMIC_SPREAD:
    case GS_PEAK_ATOMIC_SAME: {
      const uint32_t n_addr =
          kind == GS_PEAK_ATOMIC_SAME ? 64u : (uint32_t)blocks * 256u;
      hipLaunchKernelGGL(k_peak_atomic, dim3(blocks), dim3(256), 0, s,
                         static_cast<float*>(buf), n_addr, iters);
      *work = (double)blocks * 256 * (double)iters;
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t peak_min_bytes(int kind, int iters) {
  const size_t threads = (size_t)256 * 16 * 256;
  switch (kind) {
    case GS_PEAK_COPY: return 2 * sizeof(float4);
    case GS_PEAK_READ: return threads * sizeof(float) + sizeof(float4);
    case GS_PEAK_LDS:
    case GS_PEAK_FMA:
    case GS_PEAK_EXP: return threads * sizeof(float);
    case GS_PEAK_ATOMIC_SPREAD: return threads * sizeof(float);
    case GS_PEAK_ATOMIC_SAME: return 64 * sizeof(float);
    default: (void)iters; return 0;
  }
}

}  // namespace gs
