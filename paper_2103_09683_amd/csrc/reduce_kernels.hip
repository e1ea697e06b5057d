// Scalar reductions of plan optimisation and measurement probes.
//
// The quadratic objective f = sum_v w_v (d_v - p_v)^2 and the gradient norm
// are accumulated in FP64 with a two-pass reduction whose order depends only
// on n: pass 1 gives workgroup b the fixed range [b*C, (b+1)*C) and reduces
// it with a fixed per-thread stride and a fixed LDS tree; pass 2 reduces the
// partials the same way in one workgroup.  No atomics (Sec. II-D).
#include "dose_internal.h"

namespace dose {
namespace {

constexpr int kRedThreads = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_nt4(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kRedThreads) void k_objective_pass1(int64_t n, int64_t chunk,
                                                                 const float* __restrict__ d,
                                                                 const float* __restrict__ p,
                                                                 const float* __restrict__ w,
                                                                 float* __restrict__ seed,
                                                                 double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kRedThreads) {
    const double r = static_cast<double>(d[i]) - static_cast<double>(p[i]);
    const double wi = static_cast<double>(w[i]);
    acc += wi * r * r;
    if (seed) seed[i] = static_cast<float>(2.0 * wi * r);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_sumsq_pass1(int64_t n, int64_t chunk,
                                                             const float* __restrict__ g,
                                                             double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kRedThreads) {
    const double v = static_cast<double>(g[i]);
    acc += v * v;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_pass2(const double* __restrict__ partial, int n_partial,
                                                       int take_sqrt, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_partial; i += kRedThreads) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(s) : s;
}

// Read-only stream with 16-byte non-temporal loads (as the SpMV streams its
// matrix); the store happens only if the data XORs to a fixed improbable
// pattern, which keeps the loads alive.
__global__ __launch_bounds__(256) void k_probe_read(const uint4* __restrict__ buf, uint64_t n16,
                                                    float* __restrict__ sink) {
  uint32_t acc = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  // four independent 16-byte loads in flight per thread
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 v0 = ld_nt4(buf + i), v1 = ld_nt4(buf + i + stride), v2 = ld_nt4(buf + i + 2 * stride),
                v3 = ld_nt4(buf + i + 3 * stride);
    acc ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w;
    acc ^= v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
  }
  for (; i < n16; i += stride) {
    const uint4 v = buf[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[blockIdx.x & 65535] = __uint_as_float(acc);
}

__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    uint64_t n16) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_objective(int64_t n, const float* d, const float* p, const float* w, float* seed,
                            double* partial, int n_partial, double* f_out, hipStream_t s) {
  const int64_t chunk = n_partial > 0 ? (n + n_partial - 1) / n_partial : 0;
  if (n > 0)
    hipLaunchKernelGGL(k_objective_pass1, dim3(n_partial), dim3(kRedThreads), 0, s, n, chunk, d, p, w, seed,
                       partial);
  hipLaunchKernelGGL(k_pass2, dim3(1), dim3(kRedThreads), 0, s, partial, n > 0 ? n_partial : 0, 0, f_out);
  return hipGetLastError();
}

hipError_t launch_norm2(int64_t n, const float* g, double* partial, int n_partial, double* out, hipStream_t s) {
  const int64_t chunk = n_partial > 0 ? (n + n_partial - 1) / n_partial : 0;
  if (n > 0)
    hipLaunchKernelGGL(k_sumsq_pass1, dim3(n_partial), dim3(kRedThreads), 0, s, n, chunk, g, partial);
  hipLaunchKernelGGL(k_pass2, dim3(1), dim3(kRedThreads), 0, s, partial, n > 0 ? n_partial : 0, 1, out);
  return hipGetLastError();
}

hipError_t launch_probe_read(const void* buf, uint64_t bytes, float* sink, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  uint64_t grid = (n16 + 256 * 8 - 1) / (256 * 8);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_probe_read, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s,
                     static_cast<const uint4*>(buf), n16, sink);
  return hipGetLastError();
}

hipError_t launch_probe_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  uint64_t grid = (n16 + 256 * 8 - 1) / (256 * 8);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_probe_copy, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace dose
