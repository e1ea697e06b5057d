// One-time kernels of libdose: encoding FP32 source values into the stored
// formats, decoding them back for inspection, and building A^T on the device.
//
// Encoding follows the bit layouts: IEEE binary16 through the hardware
// round-to-nearest-even conversion, bfloat16 and OCP E4M3 by integer rounding
// of the FP32 bit pattern (nearest, ties to even; E4M3 saturates at 448).
#include "dose_internal.h"
#include "sell_internal.h"

#include <hip/hip_fp16.h>

#include <hipcub/hipcub.hpp>

namespace dose {
namespace {

__device__ __forceinline__ uint16_t enc_fp16(float v) { return __half_as_ushort(__float2half_rn(v)); }

__device__ __forceinline__ uint16_t enc_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ uint8_t enc_e4m3(float t) {
  const uint32_t u = __float_as_uint(t);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7FFFFFFFu;
  const float f = __uint_as_float(a);
  if (f >= 448.0f) return static_cast<uint8_t>(sign | 0x7Eu);
  if (f < 0x1p-6f) {
    // below the normal range one quantum is 2^-9: f * 512 < 8 is exact
    const float q = __builtin_rintf(f * 512.0f);
    return static_cast<uint8_t>(sign | static_cast<uint32_t>(q));
  }
  int e = static_cast<int>(a >> 23) - 127;  // -6 .. 8
  const uint32_t mant = a & 0x7FFFFFu;
  const uint32_t keep = mant >> 20, rest = mant & 0xFFFFFu;
  uint32_t q = 8u + keep + ((rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) ? 1u : 0u);
  if (q == 16u) {
    q = 8u;
    e += 1;
  }
  uint32_t code = (static_cast<uint32_t>(e + 7) << 3) | (q - 8u);
  if (code > 0x7Eu) code = 0x7Eu;
  return static_cast<uint8_t>(sign | code);
}

__device__ __forceinline__ float dec_code(int vf, const void* codes, uint64_t k) {
  if (vf == kFp16)
    return __half2float(__ushort_as_half(static_cast<const uint16_t*>(codes)[k]));
  if (vf == kBf16) return __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t*>(codes)[k]) << 16);
  if (vf == kFp32) return static_cast<const float*>(codes)[k];
  const uint32_t c = static_cast<const uint8_t*>(codes)[k];
  const uint32_t sign = (c & 0x80u) << 24;
  const uint32_t E = (c >> 3) & 15u, m = c & 7u;
  const float mag = E == 0 ? static_cast<float>(m) * 0x1p-9f : __uint_as_float(((E + 120u) << 23) | (m << 20));
  return __uint_as_float(__float_as_uint(mag) | sign);
}

// One wave64 per row; entry k of a row is src[k - base].
template <int VF>
__global__ __launch_bounds__(256) void k_encode_rows(const uint32_t* __restrict__ rp, uint32_t base,
                                                     int64_t n_rows,
                                                     const float* __restrict__ src,
                                                     void* __restrict__ dst,
                                                     float* __restrict__ row_scale) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  const uint32_t b = rp[row] - base, e = rp[row + 1] - base;
  if constexpr (VF == kFp8) {
    float amax = 0.0f;
    for (uint32_t k = b + lane; k < e; k += 64) amax = fmaxf(amax, fabsf(src[k]));
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    float s = amax / 448.0f;
    if (s == 0.0f) s = 1.0f;
    if (lane == 0) row_scale[row] = s;
    uint8_t* d8 = static_cast<uint8_t*>(dst);
    for (uint32_t k = b + lane; k < e; k += 64) d8[k] = enc_e4m3(src[k] / s);
  } else if constexpr (VF == kFp32) {
    float* d32 = static_cast<float*>(dst);
    for (uint32_t k = b + lane; k < e; k += 64) d32[k] = src[k];
  } else {
    uint16_t* d16 = static_cast<uint16_t*>(dst);
    for (uint32_t k = b + lane; k < e; k += 64)
      d16[k] = VF == kFp16 ? enc_fp16(src[k]) : enc_bf16(src[k]);
  }
}

// Decoded FP32 entries of rows [row_begin, row_begin + n_rows), one wave per row.
__global__ __launch_bounds__(256) void k_decode_rows(int vf, int scale_mode, const void* __restrict__ codes,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ scale,
                                                     const uint32_t* __restrict__ row_ptr,
                                                     int64_t row_begin, int64_t n_rows,
                                                     uint64_t nnz_begin, float* __restrict__ out) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n_rows) return;
  const int64_t row = row_begin + r;
  const uint32_t base = static_cast<uint32_t>(nnz_begin);
  const uint32_t b = row_ptr[row] - base, e = row_ptr[row + 1] - base;
  for (uint32_t t = b + lane; t < e; t += 64) {
    const uint64_t k = nnz_begin + t;
    float d = dec_code(vf, codes, k);
    if (scale_mode == kScaleRow) d = d * scale[row];
    if (scale_mode == kScaleCol) d = d * scale[col[k]];
    out[t] = d;
  }
}

__global__ __launch_bounds__(256) void k_row_ids(const uint32_t* __restrict__ row_ptr, int64_t n_rows,
                                                 uint64_t nnz, uint32_t* __restrict__ rows) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  // offsets are stored modulo 2^32; nnz < 2^32 here, so they are exact
  const uint32_t b = row_ptr[row], e = row_ptr[row + 1];
  for (uint32_t k = b + lane; k < e; k += 64) rows[k] = static_cast<uint32_t>(row);
  (void)nnz;
}

__global__ void k_iota(uint32_t* __restrict__ out, int64_t n) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) out[t] = static_cast<uint32_t>(t);
}

__global__ void k_widen_u16(const uint16_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) out[t] = in[t];
}

// Padding entries after the last entry take its column, so that a product
// kernel's loads past a group's end read a column of that group's window.
template <typename I>
__global__ void k_fill_pad(I* __restrict__ col, int64_t nnz, int n_pad) {
  const int t = static_cast<int>(threadIdx.x);
  if (t < n_pad) col[nnz + t] = nnz > 0 ? col[nnz - 1] : I(0);
}

template <typename T>
__global__ void k_gather_transpose(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ rows,
                                   const T* __restrict__ codes_in, T* __restrict__ codes_out,
                                   int32_t* __restrict__ col_out, int64_t n) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint32_t k = perm[t];
  codes_out[t] = codes_in[k];
  col_out[t] = static_cast<int32_t>(rows[k]);
}

// row_ptr[j] = first position t of the sorted keys with key >= j.
__global__ void k_row_ptr_from_sorted(const uint32_t* __restrict__ keys, int64_t nnz, int64_t n_cols,
                                      int64_t* __restrict__ row_ptr) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t > nnz) return;
  const int64_t prev = t == 0 ? -1 : static_cast<int64_t>(keys[t - 1]);
  const int64_t cur = t == nnz ? n_cols : static_cast<int64_t>(keys[t]);
  for (int64_t j = prev + 1; j <= cur; ++j) row_ptr[j] = t;
}

unsigned blocks_for(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

// SELL-C-sigma slice layout (dose_internal.h): one 64-thread block per
// chunk, thread i = the row at chunk position i, writing its 8 entries of
// every slice of the chunk.  Entries past the row's end get code 0 and the
// group's padding column.
template <typename C, typename I>
__global__ __launch_bounds__(64) void k_sell_pack(const SellChunk* __restrict__ chunks,
                                                  const uint64_t* __restrict__ start,
                                                  const uint32_t* __restrict__ len,
                                                  const uint32_t* __restrict__ pad_col,
                                                  const C* __restrict__ codes_in, const I* __restrict__ col_in,
                                                  C* __restrict__ codes_out, I* __restrict__ col_out) {
  const int64_t c = blockIdx.x;
  const int i = static_cast<int>(threadIdx.x);
  const int64_t pos = c * kSellC + i;
  const SellChunk ch = chunks[c];
  const uint32_t L = len[pos];
  const uint64_t b = start[pos];
  const I pad = col_out ? static_cast<I>(pad_col[c / kSellGroupChunks]) : I(0);
  for (uint32_t sl = 0; sl < ch.n_slices; ++sl) {
    const uint64_t o = (static_cast<uint64_t>(ch.slice0) + sl) * kSellSliceEntries;
    for (int e = 0; e < kSellLaneEntries; ++e) {
      const uint32_t j = sl * kSellLaneEntries + static_cast<uint32_t>(e);
      codes_out[o + sell_slot(sizeof(C), i, e)] = j < L ? codes_in[b + j] : C(0);
      if (col_out) col_out[o + sell_slot(sizeof(I), i, e)] = j < L ? col_in[b + j] : pad;
    }
  }
}

// Decoded values of the slice layout, written with a row's 8 entries of a
// slice together (offset 8 i + e, whatever the code width): code times its
// row's scale (E4M3), 0 in padding slots.
template <int VF>
__global__ __launch_bounds__(64) void k_sell_decode(const SellChunk* __restrict__ chunks,
                                                    const uint32_t* __restrict__ perm,
                                                    const uint32_t* __restrict__ len,
                                                    const void* __restrict__ codes,
                                                    const float* __restrict__ row_scale, float* __restrict__ out) {
  const int64_t c = blockIdx.x;
  const int i = static_cast<int>(threadIdx.x);
  const int64_t pos = c * kSellC + i;
  const SellChunk ch = chunks[c];
  const uint32_t L = len[pos];
  const float sc = VF == kFp8 && L > 0 ? row_scale[perm[pos]] : 1.0f;
  for (uint32_t sl = 0; sl < ch.n_slices; ++sl) {
    const uint64_t o = (static_cast<uint64_t>(ch.slice0) + sl) * kSellSliceEntries;
    const int vb = VF == kFp8 ? 1 : VF == kFp32 ? 4 : 2;
    for (int e = 0; e < kSellLaneEntries; ++e) {
      const uint32_t j = sl * kSellLaneEntries + static_cast<uint32_t>(e);
      float d = 0.0f;
      if (j < L) {
        d = dec_code(VF, codes, o + sell_slot(vb, i, e));
        if (VF == kFp8) d = d * sc;
      }
      out[o + static_cast<uint64_t>(i) * kSellLaneEntries + e] = d;
    }
  }
}

template <typename C>
hipError_t sell_pack_ix(int idx_bytes, const SellChunk* chunks, int64_t n_chunks, const uint64_t* start,
                        const uint32_t* len, const uint32_t* pad_col, const void* codes_in, const void* col_in,
                        void* codes_out, void* col_out, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(n_chunks)), block(kSellC);
  if (idx_bytes == 2)
    hipLaunchKernelGGL((k_sell_pack<C, uint16_t>), grid, block, 0, s, chunks, start, len, pad_col,
                       static_cast<const C*>(codes_in), static_cast<const uint16_t*>(col_in),
                       static_cast<C*>(codes_out), static_cast<uint16_t*>(col_out));
  else
    hipLaunchKernelGGL((k_sell_pack<C, int32_t>), grid, block, 0, s, chunks, start, len, pad_col,
                       static_cast<const C*>(codes_in), static_cast<const int32_t*>(col_in),
                       static_cast<C*>(codes_out), static_cast<int32_t*>(col_out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_encode_rows(int vf, const uint32_t* row_ptr, uint32_t base, int64_t n_rows, const float* src,
                              void* dst_codes, float* row_scale, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  const dim3 grid(blocks_for(n_rows, 4)), block(256);
  switch (vf) {
    case kFp16: hipLaunchKernelGGL(k_encode_rows<kFp16>, grid, block, 0, s, row_ptr, base, n_rows, src, dst_codes, row_scale); break;
    case kBf16: hipLaunchKernelGGL(k_encode_rows<kBf16>, grid, block, 0, s, row_ptr, base, n_rows, src, dst_codes, row_scale); break;
    case kFp8: hipLaunchKernelGGL(k_encode_rows<kFp8>, grid, block, 0, s, row_ptr, base, n_rows, src, dst_codes, row_scale); break;
    case kFp32: hipLaunchKernelGGL(k_encode_rows<kFp32>, grid, block, 0, s, row_ptr, base, n_rows, src, dst_codes, row_scale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decode(int vf, int scale_mode, const void* codes, const int32_t* col, const float* scale,
                         const uint32_t* row_ptr, int64_t row_begin, int64_t n_rows, uint64_t nnz_begin,
                         int64_t n, float* out, hipStream_t s) {
  if (n_rows <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode_rows, dim3(blocks_for(n_rows, 4)), dim3(256), 0, s, vf, scale_mode, codes, col,
                     scale, row_ptr, row_begin, n_rows, nnz_begin, out);
  return hipGetLastError();
}

hipError_t launch_row_ids(const uint32_t* row_ptr, int64_t n_rows, uint64_t nnz, uint32_t* rows, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_ids, dim3(blocks_for(n_rows, 4)), dim3(256), 0, s, row_ptr, n_rows, nnz, rows);
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

hipError_t launch_widen_u16(const uint16_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen_u16, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_pad(void* col, int idx_bytes, int64_t nnz, int n_pad, hipStream_t s) {
  if (n_pad <= 0) return hipSuccess;
  if (n_pad > 1024) return hipErrorInvalidValue;
  if (idx_bytes == 2)
    hipLaunchKernelGGL(k_fill_pad<uint16_t>, dim3(1), dim3(1024), 0, s, static_cast<uint16_t*>(col), nnz, n_pad);
  else
    hipLaunchKernelGGL(k_fill_pad<int32_t>, dim3(1), dim3(1024), 0, s, static_cast<int32_t*>(col), nnz, n_pad);
  return hipGetLastError();
}

hipError_t launch_gather_transpose(int vf, const uint32_t* perm, const uint32_t* rows, const void* codes_in,
                                   void* codes_out, int32_t* col_out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(blocks_for(n, 256)), block(256);
  if (vf == kFp8)
    hipLaunchKernelGGL(k_gather_transpose<uint8_t>, grid, block, 0, s, perm, rows,
                       static_cast<const uint8_t*>(codes_in), static_cast<uint8_t*>(codes_out), col_out, n);
  else if (vf == kFp32)
    hipLaunchKernelGGL(k_gather_transpose<uint32_t>, grid, block, 0, s, perm, rows,
                       static_cast<const uint32_t*>(codes_in), static_cast<uint32_t*>(codes_out), col_out, n);
  else
    hipLaunchKernelGGL(k_gather_transpose<uint16_t>, grid, block, 0, s, perm, rows,
                       static_cast<const uint16_t*>(codes_in), static_cast<uint16_t*>(codes_out), col_out, n);
  return hipGetLastError();
}

hipError_t launch_row_ptr_from_sorted(const uint32_t* sorted_cols, int64_t nnz, int64_t n_cols,
                                      int64_t* row_ptr_out, hipStream_t s) {
  hipLaunchKernelGGL(k_row_ptr_from_sorted, dim3(blocks_for(nnz + 1, 256)), dim3(256), 0, s, sorted_cols, nnz,
                     n_cols, row_ptr_out);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(void* tmp, size_t* tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                            const uint32_t* vals_in, uint32_t* vals_out, int64_t n, int end_bit, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, keys_in, keys_out, vals_in, vals_out,
                                            static_cast<int>(n), 0, end_bit, s);
}

hipError_t launch_sell_pack(int vf, int idx_bytes, const SellChunk* chunks, int64_t n_chunks, const uint64_t* start,
                            const uint32_t* len, const uint32_t* pad_col, const void* codes_in, const void* col_in,
                            void* codes_out, void* col_out, hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  if (n_chunks > INT32_MAX) return hipErrorInvalidValue;
  if (vf == kFp8)
    return sell_pack_ix<uint8_t>(idx_bytes, chunks, n_chunks, start, len, pad_col, codes_in, col_in, codes_out,
                                 col_out, s);
  if (vf == kFp32)
    return sell_pack_ix<uint32_t>(idx_bytes, chunks, n_chunks, start, len, pad_col, codes_in, col_in, codes_out,
                                  col_out, s);
  return sell_pack_ix<uint16_t>(idx_bytes, chunks, n_chunks, start, len, pad_col, codes_in, col_in, codes_out,
                                col_out, s);
}

hipError_t launch_sell_decode(int vf, const SellChunk* chunks, int64_t n_chunks, const uint32_t* perm,
                              const uint32_t* len, const void* codes, const float* row_scale, float* out,
                              hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  if (n_chunks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(n_chunks)), block(kSellC);
  switch (vf) {
    case kFp16: hipLaunchKernelGGL(k_sell_decode<kFp16>, grid, block, 0, s, chunks, perm, len, codes, row_scale, out); break;
    case kBf16: hipLaunchKernelGGL(k_sell_decode<kBf16>, grid, block, 0, s, chunks, perm, len, codes, row_scale, out); break;
    case kFp8: hipLaunchKernelGGL(k_sell_decode<kFp8>, grid, block, 0, s, chunks, perm, len, codes, row_scale, out); break;
    case kFp32: hipLaunchKernelGGL(k_sell_decode<kFp32>, grid, block, 0, s, chunks, perm, len, codes, row_scale, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dose
