// Internal definitions shared by the host side of libdose and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dose {

// Threads of one SpMV workgroup (four wave64 wavefronts).
constexpr int kThreads = 256;
// Entries one lane loads per step: 8 values and 8 column indices.
constexpr int kChunk = 8;
// Most rows one row block may cover (bounds the LDS copy of its row offsets).
constexpr int kMaxBlockRows = 1024;
// Block sizes the kernels are instantiated for (entries of A per row block).
constexpr int kMinBlockNnz = 256;
constexpr int kMaxBlockNnz = 8192;
// Padding of the value and index streams: every 8-entry load issued for a
// block stays inside the allocation.
constexpr int64_t kStreamPad = 64;

// One unit of work of the SpMV kernels: a run of whole rows holding at most
// block_nnz entries, or one chunk of a row longer than block_nnz.
struct alignas(32) BlockDesc {
  uint64_t nnz_begin;  // first entry of the block
  uint32_t nnz_count;  // entries in the block
  uint32_t row_begin;  // first row
  uint32_t row_count;  // rows covered; 0 marks a chunk of a split row
  uint32_t meta;       // bits 0..2: log2 of the lanes that reduce one row
  uint32_t partial;    // split chunks: slot of the chunk's partial sum
  uint32_t pad;
};
static_assert(sizeof(BlockDesc) == 32, "BlockDesc layout");

// A row longer than block_nnz: its chunks' partial sums sit in slots
// [first_slot, first_slot + n_slots) and are added in slot order.
struct alignas(16) SplitRow {
  uint32_t row;
  uint32_t first_slot;
  uint32_t n_slots;
  uint32_t pad;
};

// Value formats (numbers as in dose.h).
enum ValueFormat : int { kFp16 = 1, kBf16 = 2, kFp8 = 3 };

// How an E4M3 operand's scale enters the product.
enum ScaleMode : int {
  kScaleNone = 0,  // FP16 / BF16
  kScaleRow = 1,   // y_i = s_i * sum_k q_k x_k           (A, row scale)
  kScaleCol = 2    // y_j = sum_k fl32(q_k s_col(k)) v    (A^T, scale of A's rows)
};

// Everything one SpMV kernel needs for one operand and one product.
struct SpmvArgs {
  const BlockDesc* blocks;
  const void* val;         // codes, padded by kStreamPad
  const int32_t* col;      // padded by kStreamPad
  const uint32_t* row_ptr; // n_rows+1 offsets modulo 2^32
  const float* scale;      // row or column scale (E4M3), else null
  const float* x;          // [n_cols][n_rhs]
  float* y;                // [n_rows][n_rhs]
  float* partials;         // [n_partials][n_rhs]
  const SplitRow* splits;
  int64_t n_blocks;
  int64_t n_splits;
};

// Work item of a batched launch: block `block` of item `item`.
struct alignas(8) WorkItem {
  uint32_t item;
  uint32_t block;
};

// ------------------------------------------------------------ launchers
hipError_t launch_spmv(int vf, int scale_mode, int n_rhs, int block_nnz, const SpmvArgs& a,
                       hipStream_t s);
hipError_t launch_spmv_batched(int vf, int scale_mode, int n_rhs, int block_nnz,
                               const SpmvArgs* d_args, const WorkItem* d_work, int64_t n_work,
                               int grid, hipStream_t s);
hipError_t launch_combine(int scale_mode, int n_rhs, const SpmvArgs& a, hipStream_t s);
hipError_t launch_combine_batched(int scale_mode, int n_rhs, const SpmvArgs* d_args,
                                  const uint32_t* d_split_items, const uint32_t* d_split_idx,
                                  int64_t n, hipStream_t s);

// Rows [0, n_rows) of row_ptr (offsets modulo 2^32); entry k of a row sits at
// src[k - base] and its code goes to dst_codes[k - base].
hipError_t launch_encode_rows(int vf, const uint32_t* row_ptr, uint32_t base, int64_t n_rows,
                              const float* src, void* dst_codes, float* row_scale,
                              hipStream_t s);
hipError_t launch_decode(int vf, int scale_mode, const void* codes, const int32_t* col,
                         const float* scale, const uint32_t* row_ptr, int64_t row_begin,
                         int64_t n_rows, uint64_t nnz_begin, int64_t n, float* out,
                         hipStream_t s);
hipError_t launch_row_ids(const uint32_t* row_ptr, int64_t n_rows, uint64_t nnz, uint32_t* rows,
                          hipStream_t s);
hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_gather_transpose(int vf, const uint32_t* perm, const uint32_t* rows,
                                   const void* codes_in, void* codes_out, int32_t* col_out,
                                   int64_t n, hipStream_t s);
hipError_t launch_row_ptr_from_sorted(const uint32_t* sorted_cols, int64_t nnz, int64_t n_cols,
                                      int64_t* row_ptr_out, hipStream_t s);
hipError_t radix_sort_pairs(void* tmp, size_t* tmp_bytes, const uint32_t* keys_in,
                            uint32_t* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                            int64_t n, int end_bit, hipStream_t s);

hipError_t launch_objective(int64_t n, const float* d, const float* p, const float* w,
                            float* seed, double* partial, int n_partial, double* f_out,
                            hipStream_t s);
hipError_t launch_norm2(int64_t n, const float* g, double* partial, int n_partial, double* out,
                        hipStream_t s);
hipError_t launch_probe_read(const void* buf, uint64_t bytes, float* sink, hipStream_t s);
hipError_t launch_probe_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);

}  // namespace dose
