// Scalar reductions of plan optimisation and measurement probes.
//
// The quadratic objective f = sum_v w_v (d_v - p_v)^2 (of one dose vector, or
// of every scenario of a robust plan, whose dose is the sum of its beams'
// doses) and the gradient norm are accumulated in FP64 with a two-pass
// reduction whose order depends only on n: pass 1 gives workgroup b the fixed
// range [b*C, (b+1)*C), in which each thread adds its terms in a fixed order
// (the norm: elements t, t + 256, ...; the objective: 4-element vectors t,
// t + 256, ..., C a multiple of 4) before a fixed LDS tree; pass 2 reduces
// the partials the same way in one workgroup.  No atomics (Sec. II-D).
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

// acc + w (d - p)^2 in FP64; the seed 2 w (d - p) rounded to FP32 in sd.
__device__ __forceinline__ double add_term(double acc, float d, float pf, float wf, float& sd) {
  const double r = static_cast<double>(d) - static_cast<double>(pf);
  const double wi = static_cast<double>(wf);
  sd = static_cast<float>(2.0 * wi * r);
  return acc + wi * r * r;
}

__device__ __forceinline__ float4 ld4(const float* q) { return *reinterpret_cast<const float4*>(q); }
__device__ __forceinline__ float4 ld4_nt(const float* q) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(q));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void add4(float4& d, const float4 e) {
  d.x += e.x;
  d.y += e.y;
  d.z += e.z;
  d.w += e.w;
}

// Scenario pass 1.  Workgroup x takes scenario s = x % n_scen and voxel chunk
// c = x / n_scen (the scenarios of one chunk run side by side, so p and w are
// read from HBM about once); chunks are multiples of 4 voxels.  The dose of
// voxel i in scenario s is the sum of the scenario's beam doses part[s][b][i],
// added in ascending b in FP32.  Thread t takes the 4-voxel vectors
// t, t + 256, t + 512, ... of its chunk and adds their FP64 objective terms in
// that order (voxels of a vector in ascending order) before the LDS tree into
// partial[s][c].  VEC (n a multiple of 4, every array 16-byte aligned) moves
// each vector with one 16-byte access, two vectors at a time, with the loads
// of all beams in flight together when the beam count is a template
// argument (NB); otherwise the
// same order with 4-byte accesses.  So the result depends only on n, never on
// the path.  With n_scen = n_beams = 1 this is the objective of one dose vector.
template <bool VEC, int NB>  // NB > 0: n_beams == NB, known at compile time
__global__ __launch_bounds__(kRedThreads) void k_scenario_pass1(int n_scen, int n_beams, int64_t n,
                                                                int64_t chunk, int n_chunks,
                                                                const float* __restrict__ part,
                                                                const float* __restrict__ p,
                                                                const float* __restrict__ w,
                                                                float* __restrict__ d_out,
                                                                float* __restrict__ seed,
                                                                double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int s = static_cast<int>(blockIdx.x % static_cast<unsigned>(n_scen));
  const int c = static_cast<int>(blockIdx.x / static_cast<unsigned>(n_scen));
  const int64_t b0 = static_cast<int64_t>(c) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  const int64_t nv = b1 > b0 ? (b1 - b0 + 3) / 4 : 0;
  const float* ps = part + static_cast<int64_t>(s) * n_beams * n;
  const int64_t so = static_cast<int64_t>(s) * n;
  double acc = 0.0;
  if constexpr (VEC) {
    auto finish = [&](const float4 d, const int64_t i, const float4 pv, const float4 wv) {
      float4 sd;
      acc = add_term(acc, d.x, pv.x, wv.x, sd.x);
      acc = add_term(acc, d.y, pv.y, wv.y, sd.y);
      acc = add_term(acc, d.z, pv.z, wv.z, sd.z);
      acc = add_term(acc, d.w, pv.w, wv.w, sd.w);
      if (d_out) *reinterpret_cast<float4*>(d_out + so + i) = d;
      if (seed) *reinterpret_cast<float4*>(seed + so + i) = sd;
    };
    int64_t v = threadIdx.x;
    for (; v + kRedThreads < nv; v += 2 * kRedThreads) {
      const int64_t i0 = b0 + 4 * v, i1 = i0 + 4 * kRedThreads;
      const float4 p0 = ld4(p + i0), w0 = ld4(w + i0), p1 = ld4(p + i1), w1 = ld4(w + i1);
      float4 d0 = ld4_nt(ps + i0), d1 = ld4_nt(ps + i1);
      if constexpr (NB > 0) {
        // every beam's loads issue before the first add
#pragma unroll
        for (int b = 1; b < NB; ++b) {
          const float* pb = ps + static_cast<int64_t>(b) * n;
          const float4 e0 = ld4_nt(pb + i0), e1 = ld4_nt(pb + i1);
          add4(d0, e0);
          add4(d1, e1);
        }
      } else {
        for (int b = 1; b < n_beams; ++b) {
          const float* pb = ps + static_cast<int64_t>(b) * n;
          const float4 e0 = ld4_nt(pb + i0), e1 = ld4_nt(pb + i1);
          add4(d0, e0);
          add4(d1, e1);
        }
      }
      finish(d0, i0, p0, w0);
      finish(d1, i1, p1, w1);
    }
    if (v < nv) {
      const int64_t i0 = b0 + 4 * v;
      const float4 p0 = ld4(p + i0), w0 = ld4(w + i0);
      float4 d0 = ld4_nt(ps + i0);
      for (int b = 1; b < n_beams; ++b) add4(d0, ld4_nt(ps + static_cast<int64_t>(b) * n + i0));
      finish(d0, i0, p0, w0);
    }
  } else {
    for (int64_t v = threadIdx.x; v < nv; v += kRedThreads) {
      const int64_t i0 = b0 + 4 * v;
      float d[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) d[j] = i0 + j < b1 ? ps[i0 + j] : 0.0f;
      for (int b = 1; b < n_beams; ++b) {
        const float* pb = ps + static_cast<int64_t>(b) * n;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (i0 + j < b1) d[j] += pb[i0 + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t i = i0 + j;
        if (i < b1) {
          float sd;
          acc = add_term(acc, d[j], p[i], w[i], sd);
          if (d_out) d_out[so + i] = d[j];
          if (seed) seed[so + i] = sd;
        }
      }
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[static_cast<int64_t>(s) * n_chunks + c] = t;
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

// Scenario pass 2, one workgroup: f_s from partial[s][*] in the order of
// k_pass2 (thread t adds partials t, t + 256, ... in ascending order, then the
// same LDS tree), eight scenarios at a time so that their loads and trees
// overlap; then the robust forms in ascending s: worst case max_s f_s (ties
// to the first scenario, whose index is stored as a double) and expectation
// sum_s prob_s f_s, or (sum_s f_s) / n_scen without probabilities.
constexpr int kScenBatch = 8;

__global__ __launch_bounds__(kRedThreads) void k_scenario_pass2(const double* __restrict__ partial,
                                                                int n_partial, int n_scen,
                                                                const double* __restrict__ prob,
                                                                double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double sh[kScenBatch][kRedThreads];
  const int t = threadIdx.x;
  for (int s0 = 0; s0 < n_scen; s0 += kScenBatch) {
    const int ns = n_scen - s0 < kScenBatch ? n_scen - s0 : kScenBatch;
    double acc[kScenBatch];
#pragma unroll
    for (int j = 0; j < kScenBatch; ++j) acc[j] = 0.0;
    for (int i = t; i < n_partial; i += kRedThreads) {
#pragma unroll
      for (int j = 0; j < kScenBatch; ++j)
        if (j < ns) acc[j] += partial[static_cast<int64_t>(s0 + j) * n_partial + i];
    }
#pragma unroll
    for (int j = 0; j < kScenBatch; ++j) sh[j][t] = acc[j];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
      if (t < w) {
#pragma unroll
        for (int j = 0; j < kScenBatch; ++j) sh[j][t] = sh[j][t] + sh[j][t + w];
      }
      __syncthreads();
    }
    if (t == 0)
      for (int j = 0; j < ns; ++j) out[s0 + j] = sh[j][0];
    __syncthreads();
  }
  if (t == 0) {
    double worst = out[0], e = 0.0;
    int arg = 0;
    for (int s = 1; s < n_scen; ++s)
      if (out[s] > worst) {
        worst = out[s];
        arg = s;
      }
    if (prob) {
      for (int s = 0; s < n_scen; ++s) e += prob[s] * out[s];
    } else {
      for (int s = 0; s < n_scen; ++s) e += out[s];
      e = e / static_cast<double>(n_scen);
    }
    out[n_scen] = worst;
    out[n_scen + 1] = e;
    out[n_scen + 2] = static_cast<double>(arg);
  }
}

// Seeds of the robust gradient: the derivative of the robust objective with
// respect to scenario s's dose is c_s times that scenario's seed, c_s = prob_s
// (1 / n_scen without probabilities) for the expectation, and for the worst
// case 1 for the scenario whose index k_scenario_pass2 stored in out[n_scen
// + 2] and 0 for the others.  wseed[s][v] = fl32(c_s g seed[s][v]), the
// product formed in FP64 (exact for c_s in {0, 1}) and rounded once; g is the
// caller's outer derivative (1 when absent).  Workgroups stride over
// (scenario, 1024-voxel chunk) pairs, four voxels per thread.
constexpr int kSeedChunk = 4 * kRedThreads;

__global__ __launch_bounds__(kRedThreads) void k_robust_seed(int n_scen, int64_t n, int64_t n_chunks, int worst,
                                                             const double* __restrict__ out,
                                                             const double* __restrict__ prob,
                                                             const double* __restrict__ gscale,
                                                             const float* seed, float* wseed) {
  const int64_t total = n_chunks * n_scen;
  for (int64_t job = blockIdx.x; job < total; job += gridDim.x) {
    const int s = static_cast<int>(job / n_chunks);
    const int64_t chunk = job - static_cast<int64_t>(s) * n_chunks;
    double c;
    if (worst)
      c = s == static_cast<int>(out[n_scen + 2]) ? 1.0 : 0.0;
    else
      c = prob ? prob[s] : 1.0 / static_cast<double>(n_scen);
    const double cg = gscale ? c * gscale[0] : c;
    const int64_t base = static_cast<int64_t>(s) * n;
    const int64_t v0 = chunk * kSeedChunk + threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = v0 + j * kRedThreads;
      if (v < n) wseed[base + v] = static_cast<float>(cg * static_cast<double>(seed[base + v]));
    }
  }
}

// u_i = fl32(s_i * v_i): an E4M3 matrix's row scales applied to the adjoint's
// seed, so that the product over A^T gathers one value per entry.
__global__ __launch_bounds__(256) void k_scale_vec(int64_t n, const float* __restrict__ sc,
                                                   const float* __restrict__ v, float* __restrict__ u) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    u[i] = sc[i] * v[i];
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

namespace {
bool aligned16(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

// Pass 1 over n_scen scenarios (chunks of whole 4-voxel vectors), then the
// given pass 2.
void scenario_pass1(int n_scen, int n_beams, int64_t n, const float* part, const float* p, const float* w,
                    float* d_out, float* seed, double* partial, int n_partial, hipStream_t s) {
  if (n <= 0) return;
  int64_t chunk = (n + n_partial - 1) / n_partial;
  chunk = (chunk + 3) / 4 * 4;
  const bool vec = n % 4 == 0 && aligned16(part) && aligned16(p) && aligned16(w) && aligned16(d_out) &&
                   aligned16(seed);
  const dim3 grid(static_cast<unsigned>(n_partial) * static_cast<unsigned>(n_scen));
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, dim3(kRedThreads), 0, s, n_scen, n_beams, n, chunk, n_partial, part, p, w,
                       d_out, seed, partial);
  };
  if (!vec) return go(k_scenario_pass1<false, 0>);
  switch (n_beams) {
    case 1: return go(k_scenario_pass1<true, 1>);
    case 2: return go(k_scenario_pass1<true, 2>);
    case 3: return go(k_scenario_pass1<true, 3>);
    case 4: return go(k_scenario_pass1<true, 4>);
    case 5: return go(k_scenario_pass1<true, 5>);
    case 6: return go(k_scenario_pass1<true, 6>);
    case 7: return go(k_scenario_pass1<true, 7>);
    case 8: return go(k_scenario_pass1<true, 8>);
    default: return go(k_scenario_pass1<true, 0>);
  }
}
}  // namespace

hipError_t launch_objective(int64_t n, const float* d, const float* p, const float* w, float* seed,
                            double* partial, int n_partial, double* f_out, hipStream_t s) {
  scenario_pass1(1, 1, n, d, p, w, nullptr, seed, partial, n_partial, s);
  hipLaunchKernelGGL(k_pass2, dim3(1), dim3(kRedThreads), 0, s, partial, n > 0 ? n_partial : 0, 0, f_out);
  return hipGetLastError();
}

hipError_t launch_scenario(int n_scen, int n_beams, int64_t n, const float* part, const float* p, const float* w,
                           const double* prob, float* d_out, float* seed, double* partial, int n_partial,
                           double* out, hipStream_t s) {
  scenario_pass1(n_scen, n_beams, n, part, p, w, d_out, seed, partial, n_partial, s);
  hipLaunchKernelGGL(k_scenario_pass2, dim3(1), dim3(kRedThreads), 0, s, partial, n > 0 ? n_partial : 0, n_scen,
                     prob, out);
  return hipGetLastError();
}

hipError_t launch_robust_seed(int n_scen, int64_t n, int worst, const double* out, const double* prob,
                              const double* gscale, const float* seed, float* wseed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t n_chunks = (n + kSeedChunk - 1) / kSeedChunk;
  const int64_t jobs = n_chunks * n_scen;
  const unsigned grid = static_cast<unsigned>(jobs < 65536 ? jobs : 65536);
  hipLaunchKernelGGL(k_robust_seed, dim3(grid), dim3(kRedThreads), 0, s, n_scen, n, n_chunks, worst, out, prob,
                     gscale, seed, wseed);
  return hipGetLastError();
}

hipError_t launch_norm2(int64_t n, const float* g, double* partial, int n_partial, double* out, hipStream_t s) {
  const int64_t chunk = n_partial > 0 ? (n + n_partial - 1) / n_partial : 0;
  if (n > 0)
    hipLaunchKernelGGL(k_sumsq_pass1, dim3(n_partial), dim3(kRedThreads), 0, s, n, chunk, g, partial);
  hipLaunchKernelGGL(k_pass2, dim3(1), dim3(kRedThreads), 0, s, partial, n > 0 ? n_partial : 0, 1, out);
  return hipGetLastError();
}

hipError_t launch_scale_vec(int64_t n, const float* sc, const float* v, float* u, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 256 * 4 - 1) / (256 * 4);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_scale_vec, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, n, sc, v, u);
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
