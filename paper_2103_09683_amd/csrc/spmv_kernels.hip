// SpMV kernels of libdose for gfx950 (CDNA4, wave64).
//
// The product is Listing 1 of the paper: y_i = sum over row i's stored
// entries of data[k] * x[col[k]].  The paper gives every row one 32-lane warp
// that strides the row; here a 256-thread workgroup takes a *row block*, a run
// of whole rows holding at most block_nnz entries (rows longer than that are
// cut into chunks), and works in two phases:
//
//   1. stream: each lane takes 8 consecutive entries of the block, loads their
//      8 codes with one 16-byte load (8-byte for E4M3) and their 8 column
//      indices with two 16-byte loads, decodes the codes to FP32, gathers x
//      and writes the 8 products to LDS.  Loads are contiguous across lanes
//      whatever the row lengths are, so the block is read once, coalesced.
//   2. reduce: G lanes (a power of two picked per block from its mean row
//      length) sum each row's products from LDS, lane j taking every G-th
//      product from the row's start plus j, then combine in a fixed xor tree.
//
// The summation order depends only on the partition (block boundaries and G),
// never on timing: no atomics anywhere, so equal inputs give equal bits
// (Sec. II-D).  Split rows leave one partial per chunk; combine() adds them in
// chunk order.
#include "dose_internal.h"

#include <hip/hip_fp16.h>

namespace dose {
namespace {

// ----------------------------------------------------------------- decoding
__device__ __forceinline__ float dec_fp16(uint32_t h) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(h)));
}

__device__ __forceinline__ float dec_bf16(uint32_t b) { return __uint_as_float(b << 16); }

// OCP E4M3: E = 0 gives m * 2^-9; otherwise 2^(E-7) * (1 + m/8).  The encoder
// never emits the NaN code, so no case is needed for it.
__device__ __forceinline__ float dec_e4m3(uint32_t c) {
  const uint32_t sign = (c & 0x80u) << 24;
  const uint32_t E = (c >> 3) & 15u, m = c & 7u;
  const float mag = E == 0 ? static_cast<float>(m) * 0x1p-9f : __uint_as_float(((E + 120u) << 23) | (m << 20));
  return __uint_as_float(__float_as_uint(mag) | sign);
}

template <int VF>
struct Codes;
template <>
struct Codes<kFp16> {
  uint4 w;
  __device__ __forceinline__ void load(const void* base, uint64_t k0) {
    w = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + k0);
  }
  __device__ __forceinline__ float get(int e) const {
    const uint32_t word = e < 2 ? w.x : e < 4 ? w.y : e < 6 ? w.z : w.w;
    return dec_fp16((word >> ((e & 1) * 16)) & 0xFFFFu);
  }
};
template <>
struct Codes<kBf16> {
  uint4 w;
  __device__ __forceinline__ void load(const void* base, uint64_t k0) {
    w = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + k0);
  }
  __device__ __forceinline__ float get(int e) const {
    const uint32_t word = e < 2 ? w.x : e < 4 ? w.y : e < 6 ? w.z : w.w;
    return dec_bf16((word >> ((e & 1) * 16)) & 0xFFFFu);
  }
};
template <>
struct Codes<kFp8> {
  uint2 w;
  __device__ __forceinline__ void load(const void* base, uint64_t k0) {
    w = *reinterpret_cast<const uint2*>(static_cast<const uint8_t*>(base) + k0);
  }
  __device__ __forceinline__ float get(int e) const {
    const uint32_t word = e < 4 ? w.x : w.y;
    return dec_e4m3((word >> ((e & 3) * 8)) & 0xFFu);
  }
};

template <int NRHS>
struct XVec {
  float v[NRHS];
};

template <int NRHS>
__device__ __forceinline__ XVec<NRHS> load_x(const float* x, int c) {
  XVec<NRHS> r;
  if constexpr (NRHS == 1) {
    r.v[0] = x[c];
  } else if constexpr (NRHS == 2) {
    const float2 t = *reinterpret_cast<const float2*>(x + 2 * static_cast<int64_t>(c));
    r.v[0] = t.x;
    r.v[1] = t.y;
  } else {
    const float4 t = *reinterpret_cast<const float4*>(x + 4 * static_cast<int64_t>(c));
    r.v[0] = t.x;
    r.v[1] = t.y;
    r.v[2] = t.z;
    r.v[3] = t.w;
  }
  return r;
}

// LDS footprint of one block's products, in floats.
template <int NRHS, int CAP>
struct Lds {
  static constexpr int kProd = (CAP + 2 * kChunk) * NRHS;
};

// One row block: stream its entries into LDS products, then reduce rows.
template <int VF, int SM, int NRHS, int CAP>
__device__ __forceinline__ void process_block(const SpmvArgs& a, const BlockDesc& b,
                                              float* __restrict__ prod,
                                              uint32_t* __restrict__ rp) {
  const int tid = threadIdx.x;
  const uint64_t nb0 = b.nnz_begin;
  const uint64_t nb1 = nb0 + b.nnz_count;
  const uint64_t a0 = nb0 & ~static_cast<uint64_t>(kChunk - 1);
  const int lo = static_cast<int>(nb0 - a0);
  const int hi = static_cast<int>(nb1 - a0);
  const int nchunks = (hi + kChunk - 1) / kChunk;

  // ---- phase 1: coalesced stream of codes and indices, products to LDS
  for (int c = tid; c < nchunks; c += kThreads) {
    const uint64_t k0 = a0 + static_cast<uint64_t>(c) * kChunk;
    Codes<VF> codes;
    codes.load(a.val, k0);
    const int4 c0 = *reinterpret_cast<const int4*>(a.col + k0);
    const int4 c1 = *reinterpret_cast<const int4*>(a.col + k0 + 4);
    const int cols[kChunk] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    float p[kChunk][NRHS];
#pragma unroll
    for (int e = 0; e < kChunk; ++e) {
      const int kl = c * kChunk + e;
      const bool in = kl >= lo && kl < hi;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) p[e][r] = 0.0f;
      if (in) {
        float d = codes.get(e);
        if constexpr (SM == kScaleCol) d = d * a.scale[cols[e]];
        const XVec<NRHS> xv = load_x<NRHS>(a.x, cols[e]);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) p[e][r] = d * xv.v[r];
      }
    }
    float* dst = prod + static_cast<int64_t>(c) * kChunk * NRHS;
#pragma unroll
    for (int q = 0; q < kChunk * NRHS; q += 4)
      *reinterpret_cast<float4*>(dst + q) =
          make_float4(p[q / NRHS][q % NRHS], p[(q + 1) / NRHS][(q + 1) % NRHS],
                      p[(q + 2) / NRHS][(q + 2) % NRHS], p[(q + 3) / NRHS][(q + 3) % NRHS]);
  }

  const bool split = b.row_count == 0;
  if (!split) {
    const uint32_t base = static_cast<uint32_t>(a0);
    for (int i = tid; i <= static_cast<int>(b.row_count); i += kThreads)
      rp[i] = a.row_ptr[b.row_begin + i] - base;
  }
  __syncthreads();

  // ---- phase 2: rows reduced by groups of G lanes in a fixed order
  const int lg = static_cast<int>(b.meta & 7u);
  const int G = 1 << lg;
  const int lane = tid & (G - 1);
  const int group = tid >> lg;
  const int ngroups = kThreads >> lg;
  const int nrows = split ? 1 : static_cast<int>(b.row_count);
  for (int r = group; r < nrows; r += ngroups) {
    const int s = split ? lo : static_cast<int>(rp[r]);
    const int e = split ? hi : static_cast<int>(rp[r + 1]);
    float acc[NRHS];
#pragma unroll
    for (int q = 0; q < NRHS; ++q) acc[q] = 0.0f;
    if (e > s) {
      for (int k = s + lane; k < e; k += G) {
        if constexpr (NRHS == 1) {
          acc[0] += prod[k];
        } else if constexpr (NRHS == 2) {
          const float2 t = *reinterpret_cast<const float2*>(prod + 2 * k);
          acc[0] += t.x;
          acc[1] += t.y;
        } else {
          const float4 t = *reinterpret_cast<const float4*>(prod + 4 * k);
          acc[0] += t.x;
          acc[1] += t.y;
          acc[2] += t.z;
          acc[3] += t.w;
        }
      }
      for (int off = G >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NRHS; ++q) acc[q] += __shfl_xor(acc[q], off, G);
      }
    }
    if (lane == 0) {
      if (split) {
        float* dst = a.partials + static_cast<int64_t>(b.partial) * NRHS;
#pragma unroll
        for (int q = 0; q < NRHS; ++q) dst[q] = acc[q];
      } else {
        const int64_t row = static_cast<int64_t>(b.row_begin) + r;
        const float sc = SM == kScaleRow ? a.scale[row] : 1.0f;
        float* dst = a.y + row * NRHS;
#pragma unroll
        for (int q = 0; q < NRHS; ++q) dst[q] = SM == kScaleRow ? acc[q] * sc : acc[q];
      }
    }
  }
  __syncthreads();
}

template <int VF, int SM, int NRHS, int CAP>
__global__ __launch_bounds__(kThreads) void k_spmv(SpmvArgs a) {
  __shared__ __align__(16) float prod[Lds<NRHS, CAP>::kProd];
  __shared__ uint32_t rp[kMaxBlockRows + 1];
  const BlockDesc b = a.blocks[blockIdx.x];
  process_block<VF, SM, NRHS, CAP>(a, b, prod, rp);
}

// Persistent form: workgroups walk a list of (item, block) pairs that may
// belong to many matrices.
template <int VF, int SM, int NRHS, int CAP>
__global__ __launch_bounds__(kThreads) void k_spmv_batched(const SpmvArgs* __restrict__ args,
                                                           const WorkItem* __restrict__ work,
                                                           int64_t n_work) {
  __shared__ __align__(16) float prod[Lds<NRHS, CAP>::kProd];
  __shared__ uint32_t rp[kMaxBlockRows + 1];
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const WorkItem wi = work[w];
    const SpmvArgs a = args[wi.item];
    const BlockDesc b = a.blocks[wi.block];
    process_block<VF, SM, NRHS, CAP>(a, b, prod, rp);
  }
}

// Split rows: y[row] = (scale) * sum of the row's chunk partials, in chunk order.
template <int SM, int NRHS>
__device__ __forceinline__ void combine_one(const SpmvArgs& a, const SplitRow sr, int q) {
  float acc = 0.0f;
  for (uint32_t c = 0; c < sr.n_slots; ++c)
    acc += a.partials[static_cast<int64_t>(sr.first_slot + c) * NRHS + q];
  if constexpr (SM == kScaleRow) acc = acc * a.scale[sr.row];
  a.y[static_cast<int64_t>(sr.row) * NRHS + q] = acc;
}

template <int SM, int NRHS>
__global__ void k_combine(SpmvArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n_splits * NRHS) return;
  combine_one<SM, NRHS>(a, a.splits[t / NRHS], static_cast<int>(t % NRHS));
}

template <int SM, int NRHS>
__global__ void k_combine_batched(const SpmvArgs* __restrict__ args,
                                  const uint32_t* __restrict__ items,
                                  const uint32_t* __restrict__ idx, int64_t n) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * NRHS) return;
  const int64_t i = t / NRHS;
  const SpmvArgs& a = args[items[i]];
  combine_one<SM, NRHS>(a, a.splits[idx[i]], static_cast<int>(t % NRHS));
}

int cap_for(int block_nnz) {
  if (block_nnz <= 1024) return 1024;
  if (block_nnz <= 2048) return 2048;
  if (block_nnz <= 4096) return 4096;
  return 8192;
}

template <int VF, int SM, int NRHS>
hipError_t launch_cap(int cap, const SpmvArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_blocks)), block(kThreads);
  switch (cap) {
    case 1024: hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, 1024>), grid, block, 0, s, a); break;
    case 2048: hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, 2048>), grid, block, 0, s, a); break;
    case 4096: hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, 4096>), grid, block, 0, s, a); break;
    default:
      if constexpr (NRHS <= 2) {
        hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, 8192>), grid, block, 0, s, a);
      } else {
        return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}

template <int VF, int SM, int NRHS>
hipError_t launch_cap_batched(int cap, const SpmvArgs* args, const WorkItem* work, int64_t n_work,
                              int grid, hipStream_t s) {
  const dim3 g(static_cast<unsigned>(grid)), block(kThreads);
  switch (cap) {
    case 1024: hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, 1024>), g, block, 0, s, args, work, n_work); break;
    case 2048: hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, 2048>), g, block, 0, s, args, work, n_work); break;
    case 4096: hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, 4096>), g, block, 0, s, args, work, n_work); break;
    default:
      if constexpr (NRHS <= 2) {
        hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, 8192>), g, block, 0, s, args, work, n_work);
      } else {
        return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}

template <int VF, int SM>
hipError_t launch_rhs(int n_rhs, int cap, const SpmvArgs& a, hipStream_t s) {
  switch (n_rhs) {
    case 1: return launch_cap<VF, SM, 1>(cap, a, s);
    case 2: return launch_cap<VF, SM, 2>(cap, a, s);
    case 4: return launch_cap<VF, SM, 4>(cap, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int VF, int SM>
hipError_t launch_rhs_batched(int n_rhs, int cap, const SpmvArgs* args, const WorkItem* work,
                              int64_t n_work, int grid, hipStream_t s) {
  switch (n_rhs) {
    case 1: return launch_cap_batched<VF, SM, 1>(cap, args, work, n_work, grid, s);
    case 2: return launch_cap_batched<VF, SM, 2>(cap, args, work, n_work, grid, s);
    case 4: return launch_cap_batched<VF, SM, 4>(cap, args, work, n_work, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_spmv(int vf, int scale_mode, int n_rhs, int block_nnz, const SpmvArgs& a,
                       hipStream_t s) {
  if (a.n_blocks <= 0) return hipSuccess;
  const int cap = cap_for(block_nnz);
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_rhs<kFp16, kScaleNone>(n_rhs, cap, a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_rhs<kBf16, kScaleNone>(n_rhs, cap, a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_rhs<kFp8, kScaleRow>(n_rhs, cap, a, s);
  if (vf == kFp8 && scale_mode == kScaleCol) return launch_rhs<kFp8, kScaleCol>(n_rhs, cap, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spmv_batched(int vf, int scale_mode, int n_rhs, int block_nnz,
                               const SpmvArgs* d_args, const WorkItem* d_work, int64_t n_work,
                               int grid, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  const int cap = cap_for(block_nnz);
  if (vf == kFp16 && scale_mode == kScaleNone)
    return launch_rhs_batched<kFp16, kScaleNone>(n_rhs, cap, d_args, d_work, n_work, grid, s);
  if (vf == kBf16 && scale_mode == kScaleNone)
    return launch_rhs_batched<kBf16, kScaleNone>(n_rhs, cap, d_args, d_work, n_work, grid, s);
  if (vf == kFp8 && scale_mode == kScaleRow)
    return launch_rhs_batched<kFp8, kScaleRow>(n_rhs, cap, d_args, d_work, n_work, grid, s);
  if (vf == kFp8 && scale_mode == kScaleCol)
    return launch_rhs_batched<kFp8, kScaleCol>(n_rhs, cap, d_args, d_work, n_work, grid, s);
  return hipErrorInvalidValue;
}

template <int SM>
static hipError_t combine_rhs(int n_rhs, const SpmvArgs& a, hipStream_t s) {
  const int64_t n = a.n_splits * n_rhs;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  switch (n_rhs) {
    case 1: hipLaunchKernelGGL((k_combine<SM, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_combine<SM, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_combine<SM, 4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(int scale_mode, int n_rhs, const SpmvArgs& a, hipStream_t s) {
  if (a.n_splits <= 0) return hipSuccess;
  return scale_mode == kScaleRow ? combine_rhs<kScaleRow>(n_rhs, a, s)
                                 : combine_rhs<kScaleNone>(n_rhs, a, s);
}

template <int SM>
static hipError_t combine_rhs_batched(int n_rhs, const SpmvArgs* args, const uint32_t* items,
                                      const uint32_t* idx, int64_t n, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((n * n_rhs + 255) / 256)), block(256);
  switch (n_rhs) {
    case 1: hipLaunchKernelGGL((k_combine_batched<SM, 1>), grid, block, 0, s, args, items, idx, n); break;
    case 2: hipLaunchKernelGGL((k_combine_batched<SM, 2>), grid, block, 0, s, args, items, idx, n); break;
    case 4: hipLaunchKernelGGL((k_combine_batched<SM, 4>), grid, block, 0, s, args, items, idx, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine_batched(int scale_mode, int n_rhs, const SpmvArgs* d_args,
                                  const uint32_t* d_split_items, const uint32_t* d_split_idx,
                                  int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return scale_mode == kScaleRow
             ? combine_rhs_batched<kScaleRow>(n_rhs, d_args, d_split_items, d_split_idx, n, s)
             : combine_rhs_batched<kScaleNone>(n_rhs, d_args, d_split_items, d_split_idx, n, s);
}

}  // namespace dose
