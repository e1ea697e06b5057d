// Internal definitions shared by the host side of libdose and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dose {

// Entries one lane loads per step: two quarters of 4 codes and 4 column indices.
constexpr int kChunk = 8;
// Waves of one SpMV workgroup, and its threads.
constexpr int kGroupWaves = 4;
constexpr int kGroupThreads = kGroupWaves * 64;
// Row-group sizes (entries); a power of two in this range.
constexpr int kMinGroupNnz = 1024;
constexpr int kMaxGroupNnz = 1 << 20;
// Most rows one group may hold (bounds the time a wave spends on empty rows).
constexpr int64_t kMaxGroupRows = 16384;
// Padding of the value and index streams: every 4-entry load of a group
// stays inside the allocation; padding indices repeat the last column.
constexpr int64_t kStreamPad = 64;
// Longest row (entries): positions inside a group, in bytes of a 32-bit
// index stream, stay below 2^31.
constexpr int64_t kMaxRowNnz = int64_t{1} << 28;

// Steps (one step: 64 lanes x 8 entries, on absolute multiples of 512) and
// how a row longer than kRowSlots steps is summed: the lane sums of step s
// meet in a fixed wave reduction, giving T_s; the row is (W_0 + W_1) +
// (W_2 + W_3) with W_j the in-order sum of the T_s with s = j (mod 4) counted
// from the row's first step.  The order depends only on the row, so a row
// summed by one wave and a row shared by the four waves of a split group
// (wave j takes the steps s = j mod 4) give the same bits.  Rows of at most
// kRowSlots steps (never split) sum per lane first and reduce once.
constexpr int kStepEntries = 64 * kChunk;
constexpr int kRowSlots = 4;
static_assert(kRowSlots == kGroupWaves, "a split row gives each wave one slot");
// A row longer than max(group_nnz / 4, kSplitMinNnz) entries forms a split
// group of its own.
constexpr int64_t kSplitMinNnz = 4 * kStepEntries;

// One workgroup's work, and the window of columns its entries touch.  Either
// a run of whole rows split into one contiguous share per wave, or (split)
// one long row shared by all waves.
struct alignas(64) GroupDesc {
  uint64_t nnz_base;              // first entry of the group
  uint32_t row[kGroupWaves + 1];  // wave w takes rows [row[w], row[w+1]); split: the row is row[0]
  uint32_t cmin;                  // first column of the x window (a multiple of kWinAlign)
  uint32_t clen;                  // window columns: the loaded entries' largest column - cmin + 1 (0: no entries)
  uint32_t split;                 // 1: one row shared by all waves
  uint32_t ent[kGroupWaves];      // wave w's entries end at nnz_base + ent[w] (split: ent[3] is the row's length)
  uint32_t item;                  // batched launches: the item the group belongs to
  uint32_t cbase;                 // column of index 0: 0, or (A^T in voxel slabs, 16-bit slab-local
                                  // indices) the first voxel of the group's slab
};
static_assert(sizeof(GroupDesc) == 64, "GroupDesc layout");

// Value formats (numbers as in dose.h).
enum ValueFormat : int { kFp16 = 1, kBf16 = 2, kFp8 = 3, kFp32 = 4 };

// How an E4M3 operand's scale enters the product.
enum ScaleMode : int {
  kScaleNone = 0,  // FP16 / BF16
  kScaleRow = 1,   // y_i = s_i * sum_k q_k x_k           (A, row scale)
  kScaleCol = 2    // y_j = sum_k fl32(q_k s_col(k)) v    (A^T, scale of A's rows)
};

// Everything one SpMV kernel needs for one operand and one product.
struct SpmvArgs {
  const GroupDesc* groups;
  const void* val;          // codes, padded by kStreamPad
  const void* col;          // column indices (int32, or uint16 when idx_bytes is 2), padded by kStreamPad
  const uint32_t* row_ptr;  // n_rows+1 offsets modulo 2^32
  const float* scale;       // row or column scale (E4M3), else null
  const void* x;            // [n_cols][n_rhs] FP32, or [n_cols] FP64 (launch_spmv_f64)
  void* y;                  // [n_rows][n_rhs] FP32, or [n_rows] FP64
  int64_t n_groups;
  int32_t win_floats;       // LDS 4-byte words for the x window (dynamic shared memory)
  int32_t idx_bytes;        // 4 or 2
  int32_t xcd_blocks;       // 0, or 8: workgroups go to the chip's 8 dies round-robin; give each die
                            // one contiguous eighth of the groups (so its L2 sees one eighth of the
                            // gathered vector); the order of every row's sum is unchanged
  int32_t pad0;
};

// Entries of a quarter: lane l of a step loads the 4 entries at 4 l and at
// 256 + 4 l of it.
constexpr int kQuarterEntries = kChunk / 2;
// A group's x window starts at a multiple of this many columns (so that its
// copy moves 16-byte pieces of x).
constexpr int kWinAlign = 8;

// Largest LDS x window of one workgroup, in floats (48 KB).
constexpr int kWinFloatsMax = 12288;

// LDS floats a window of `clen` columns needs for n_rhs vectors (x's own
// layout: column-major runs of n_rhs floats).
__host__ __device__ constexpr int64_t window_floats(uint32_t clen, int n_rhs) {
  return static_cast<int64_t>(clen) * n_rhs;
}

// ------------------------------------------------------------ launchers
hipError_t launch_spmv(int vf, int scale_mode, int n_rhs, const SpmvArgs& a, hipStream_t s);
// One FP64 vector: x, y FP64, products and sums FP64; a.win_floats sized as
// for two FP32 vectors (a window column is 8 bytes).
hipError_t launch_spmv_f64(int vf, int scale_mode, const SpmvArgs& a, hipStream_t s);
// The items of a batched launch, in device memory.  Either a work list (one
// descriptor copy per workgroup, naming its item: batch plans) or, when work
// is null, the first workgroup of every item (n_items + 1 ascending entries,
// the last one the total), each item's workgroups taking its matrix's own
// row groups (args[i].groups) in order.
struct BatchTable {
  const SpmvArgs* args;
  const GroupDesc* work;
  const uint32_t* first;
  int32_t n_items;
};

// Batched launch: n_work workgroups over the groups of all items.  With
// accumulate (one vector only) every row value is added to what y holds
// (empty rows: + 0) instead of stored.
hipError_t launch_spmv_batched(int vf, int scale_mode, int n_rhs, int accumulate, int idx_bytes, const BatchTable& t,
                               int64_t n_work, int lds_floats, hipStream_t s);
hipError_t launch_group_windows(GroupDesc* groups, int64_t n_groups, const void* col, int idx_bytes,
                                const uint32_t* row_ptr, hipStream_t s);
// Sets the n_pad padding indices after entry nnz - 1 to its column (0 when
// nnz is 0); n_pad <= 1024.
hipError_t launch_fill_pad(void* col, int idx_bytes, int64_t nnz, int n_pad, hipStream_t s);
// Widens n uint16 column indices to uint32 (transpose keys).
hipError_t launch_widen_u16(const uint16_t* in, uint32_t* out, int64_t n, hipStream_t s);

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
// Robust epilogue over n_scen scenarios of n_beams beams each: part is
// [n_scen][n_beams][n] beam doses; partial holds n_scen * n_partial doubles;
// out receives n_scen objectives, then worst case, expectation, worst index.
hipError_t launch_scenario(int n_scen, int n_beams, int64_t n, const float* part, const float* p,
                           const float* w, const double* prob, float* d_out, float* seed,
                           double* partial, int n_partial, double* out, hipStream_t s);
hipError_t launch_norm2(int64_t n, const float* g, double* partial, int n_partial, double* out,
                        hipStream_t s);
// wseed[s][v] = fl32(c_s * g * seed[s][v]) for the expectation (worst = 0)
// or the worst case (worst = 1) of n_scen scenarios of n voxels.
hipError_t launch_robust_seed(int n_scen, int64_t n, int worst, const double* out, const double* prob,
                              const double* gscale, const float* seed, float* wseed, hipStream_t s);
// u_i = fl32(sc_i * v_i), i < n.
hipError_t launch_scale_vec(int64_t n, const float* sc, const float* v, float* u, hipStream_t s);
hipError_t launch_probe_read(const void* buf, uint64_t bytes, float* sink, hipStream_t s);
hipError_t launch_probe_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);

}  // namespace dose
