// Building A^T in voxel slabs, and the combine of its row partials.
//
// The slab form's rows are (slab, spot) pairs in ascending key
// (slab * n_cols + spot); a stable radix sort of A's entries by that key keeps
// each row's entries in ascending voxel, as A lists them.  Its product is the
// plain row-group product (the same kernels as every other operand); each
// spot's result is then the sum of its rows' partials in ascending slab, one
// thread per spot: a fixed order, so the adjoint stays deterministic and
// independent of the partition.
#include "dose_internal.h"
#include "slab_internal.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>

namespace dose {
namespace {

unsigned slab_blocks(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

__global__ void k_slab_keys(const uint32_t* __restrict__ rows, const uint32_t* __restrict__ cols, uint32_t slab,
                            uint32_t n_cols, int64_t n, uint32_t* __restrict__ keys) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  keys[k] = rows[k] / slab * n_cols + cols[k];
}

template <typename C>
__global__ void k_slab_gather(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ rows,
                              const uint32_t* __restrict__ keys, uint32_t n_cols, uint32_t slab,
                              const uint32_t* __restrict__ slab_off, const C* __restrict__ codes_in,
                              C* __restrict__ codes_out, uint16_t* __restrict__ col_out, int64_t n) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t e = perm[k];
  const uint32_t t = keys[k] / n_cols;
  const int64_t at = k + slab_off[t];
  codes_out[at] = codes_in[e];
  col_out[at] = static_cast<uint16_t>(rows[e] - t * slab);
}

// A spot's partials are added one by one in ascending slab; their loads are
// issued eight at a time (the row indices, then the partials) so that a spot
// of n slabs waits for about n / 4 round trips to memory instead of 2 n.
template <typename V>
__device__ __forceinline__ V combine_spot(const V* __restrict__ part, const uint32_t* __restrict__ ptr,
                                          const uint32_t* __restrict__ rows, int64_t j, V acc) {
  constexpr int kBatch = 8;
  const uint32_t end = ptr[j + 1];
  uint32_t k = ptr[j];
  for (; k + kBatch <= end; k += kBatch) {
    uint32_t r[kBatch];
    V p[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) r[i] = rows[k + i];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) p[i] = part[r[i]];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) acc = acc + p[i];
  }
  for (; k < end; ++k) acc = acc + part[rows[k]];
  return acc;
}

template <typename V>
__global__ void k_slab_combine(const V* __restrict__ part, const uint32_t* __restrict__ ptr,
                               const uint32_t* __restrict__ rows, V* __restrict__ g, int64_t n_cols) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n_cols) g[j] = combine_spot(part, ptr, rows, j, V(0));
}

// Output group blockIdx.y of an adjoint plan; its spots in blocks along x.
__global__ void k_slab_combine_groups(const SlabCombineGroup* __restrict__ groups,
                                      const SlabCombineItem* __restrict__ items) {
  const SlabCombineGroup G = groups[blockIdx.y];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= G.n_cols) return;
  float acc = 0.0f;
  for (int32_t i = G.first; i < G.first + G.count; ++i)
    acc = combine_spot(items[i].part, items[i].ptr, items[i].rows, j, acc);
  G.g[j] = acc;
}

// Item blockIdx.y of an adjoint plan's seed scalings, its elements strided
// over the blocks along x.
__global__ __launch_bounds__(256) void k_scale_items(const ScaleItem* __restrict__ items) {
  const ScaleItem it = items[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < it.n; k += stride)
    it.u[k] = it.scale[k] * it.v[k];
}

}  // namespace

hipError_t launch_scale_items(const ScaleItem* items, int32_t n_items, int64_t max_n, hipStream_t s) {
  if (n_items <= 0 || max_n <= 0) return hipSuccess;
  if (n_items > 65535) return hipErrorInvalidValue;
  const int64_t bx = std::min<int64_t>((max_n + 1023) / 1024, 4096);
  hipLaunchKernelGGL(k_scale_items, dim3(static_cast<unsigned>(bx), static_cast<unsigned>(n_items)), dim3(256), 0, s,
                     items);
  return hipGetLastError();
}

hipError_t launch_slab_keys(const uint32_t* rows, const uint32_t* cols, uint32_t slab, uint32_t n_cols,
                            int64_t n, uint32_t* keys, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (slab == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_slab_keys, dim3(slab_blocks(n, 256)), dim3(256), 0, s, rows, cols, slab, n_cols, n, keys);
  return hipGetLastError();
}

hipError_t run_length_encode(void* tmp, size_t* tmp_bytes, const uint32_t* keys, uint32_t* unique, uint32_t* counts,
                             uint32_t* n_runs, int64_t n, hipStream_t s) {
  if (n > INT32_MAX) return hipErrorInvalidValue;
  return hipcub::DeviceRunLengthEncode::Encode(tmp, *tmp_bytes, keys, unique, counts, n_runs, static_cast<int>(n), s);
}

hipError_t launch_slab_gather(int vf, const uint32_t* perm, const uint32_t* rows, const uint32_t* keys,
                              uint32_t n_cols, uint32_t slab, const uint32_t* slab_off, const void* codes_in,
                              void* codes_out, uint16_t* col_out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n_cols == 0 || slab == 0 || slab > 65536) return hipErrorInvalidValue;
  const dim3 grid(slab_blocks(n, 256)), block(256);
  if (vf == kFp8)
    hipLaunchKernelGGL(k_slab_gather<uint8_t>, grid, block, 0, s, perm, rows, keys, n_cols, slab, slab_off,
                       static_cast<const uint8_t*>(codes_in), static_cast<uint8_t*>(codes_out), col_out, n);
  else if (vf == kFp32)
    hipLaunchKernelGGL(k_slab_gather<uint32_t>, grid, block, 0, s, perm, rows, keys, n_cols, slab, slab_off,
                       static_cast<const uint32_t*>(codes_in), static_cast<uint32_t*>(codes_out), col_out, n);
  else
    hipLaunchKernelGGL(k_slab_gather<uint16_t>, grid, block, 0, s, perm, rows, keys, n_cols, slab, slab_off,
                       static_cast<const uint16_t*>(codes_in), static_cast<uint16_t*>(codes_out), col_out, n);
  return hipGetLastError();
}

hipError_t launch_slab_combine_groups(const SlabCombineGroup* groups, int32_t n_groups, const SlabCombineItem* items,
                                      int64_t max_cols, hipStream_t s) {
  if (n_groups <= 0 || max_cols <= 0) return hipSuccess;
  if (n_groups > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_slab_combine_groups, dim3(slab_blocks(max_cols, 256), static_cast<unsigned>(n_groups)),
                     dim3(256), 0, s, groups, items);
  return hipGetLastError();
}

hipError_t launch_slab_combine(bool f64, const void* part, const uint32_t* ptr, const uint32_t* rows, void* g,
                               int64_t n_cols, hipStream_t s) {
  if (n_cols <= 0) return hipSuccess;
  const dim3 grid(slab_blocks(n_cols, 256)), block(256);
  if (f64)
    hipLaunchKernelGGL(k_slab_combine<double>, grid, block, 0, s, static_cast<const double*>(part), ptr, rows,
                       static_cast<double*>(g), n_cols);
  else
    hipLaunchKernelGGL(k_slab_combine<float>, grid, block, 0, s, static_cast<const float*>(part), ptr, rows,
                       static_cast<float*>(g), n_cols);
  return hipGetLastError();
}

}  // namespace dose
