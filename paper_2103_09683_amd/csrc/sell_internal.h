// Internal definitions of libdose's SELL-C-sigma storage, shared by its host
// code and kernels.
#pragma once

#include "dose_internal.h"

namespace dose {

// ------------------------------------------------------------ SELL-C-sigma
// The rows, in sigma-sorted order (descending length inside windows of sigma
// rows), are cut into chunks of kSellC = 64 row positions, one per lane of a
// wave.  A chunk stores its rows' entries in slices: slice j of the chunk is
// kSellSliceEntries consecutive entries holding entries 8 j .. 8 j + 7 of
// each of its rows (where sell_slot puts them: one 16-byte load of FP16 codes
// per lane).  A chunk has ceil(width / 8) slices, width
// being its longest row; slots past a row's end hold code 0 and the first
// column of the chunk's x window.  A workgroup takes a group of
// kSellGroupChunks (one) chunk and its x window.
constexpr int kSellC = 64;
constexpr int kSellLaneEntries = 8;
constexpr int kSellSliceEntries = kSellC * kSellLaneEntries;
constexpr int kSellGroupChunks = 1;
constexpr int kSellGroupRows = kSellC * kSellGroupChunks;

// Offset, inside a slice, of entry e (0..7) of the row at chunk position
// `lane` in a stream of `bytes`-byte elements.  A 4-byte stream (int32
// indices, FP32 codes) holds the slice's entries 0-3 of every row, then its
// entries 4-7: two contiguous halves of 1 KB, each one 16-byte load of the 64
// lanes; narrower streams keep a row's 8 entries together (one load).
__host__ __device__ constexpr uint32_t sell_slot(int bytes, int lane, int e) {
  return bytes == 4 ? static_cast<uint32_t>((e >> 2) * (kSellC * 4) + lane * 4 + (e & 3))
                    : static_cast<uint32_t>(lane * kSellLaneEntries + e);
}

// Largest LDS x window of a SELL-C-sigma workgroup, in floats (32 KB): with
// the row sums' 1 KB per vector, four workgroups of the four-vector kernel
// (the most its registers allow) fit in a compute unit's 160 KB of LDS.
// Chunks with wider windows gather x from global memory.
constexpr int kSellWinFloatsMax = 8192;

struct alignas(16) SellChunk {
  uint32_t slice0;    // first slice of the chunk (slices of all chunks are consecutive)
  uint32_t n_slices;  // ceil(width / 8)
  uint32_t min_len;   // shortest row of the chunk (slices below min_len / 8 hold no padding)
  uint32_t pad;
};
static_assert(sizeof(SellChunk) == 16, "SellChunk layout");

// Run-length column indices (index width 0): the row at position p has the
// runs run_ptr[p] .. run_ptr[p + 1] - 1; a run is (end, delta): the row's
// entries at positions below `end` (and at or past the previous run's end)
// have column position + delta.
struct alignas(8) SellRun {
  int32_t end;
  int32_t delta;
};

struct SellArgs {
  const SellChunk* chunks;  // n_groups * kSellGroupChunks (the last group padded with empty chunks)
  const uint32_t* win;      // per group: cmin, clen (x window [cmin, cmin + clen); clen 0: no entries)
  const void* val;          // codes in the slice layout, padded by one slice
  const void* col;          // column indices (int32 or uint16), same layout
  const uint32_t* perm;     // per row position: its row (n_rows for positions past the last row)
  const uint32_t* len;      // per row position: its row's length
  const float* scale;       // E4M3: row scale by row; else null
  const uint32_t* run_ptr;  // run-length indices: n_positions + 1 offsets into runs
  const SellRun* runs;
  const uint32_t* work;     // the chunks holding entries, ascending (one workgroup each)
  const uint32_t* zero;     // the chunks without entries (their rows get +0; 4 per workgroup)
  const void* x;            // [n_cols][n_rhs] FP32, or [n_cols] FP64 (launch_sell_spmv_f64)
  void* y;                  // [n_rows][n_rhs] FP32, or [n_rows] FP64
  int64_t n_groups;         // chunks holding entries
  int64_t n_zero;           // chunks without entries
  int32_t win_floats;       // LDS window 4-byte words for the launch's vectors (0: no group uses the LDS
                            // window); an FP64 vector's window is that of two FP32 ones
  int32_t idx_bytes;        // 4, 2, or 0 (run-length indices)
  int32_t xcd_blocks;
  int32_t lds_runs;         // run-length indices: most runs of one group (LDS records)
  int32_t n_cols;
  int32_t pad0;
};

// The chunks of many matrices in one launch: work and zero hold (item,
// chunk) pairs, the chunks holding entries and those without; args, one
// SellArgs per item (all of one value and index format and n_rhs).
struct SellBatchTable {
  const SellArgs* args;
  const uint2* work;
  const uint2* zero;
  int64_t n_work;
  int64_t n_zero;
  int32_t xcd_blocks;
  int32_t pad0;
};

// y = A x for n_rhs (1, 2 or 4) row-major vectors.
hipError_t launch_sell_spmv(int vf, int scale_mode, int n_rhs, const SellArgs& a, hipStream_t s);
hipError_t launch_sell_batched(int vf, int scale_mode, int n_rhs, int idx_bytes, const SellBatchTable& t,
                               size_t lds_bytes, hipStream_t s);
// y = A x for one FP64 vector: FP64 products and sums (a.win_floats as for
// two FP32 vectors).
hipError_t launch_sell_spmv_f64(int vf, int scale_mode, const SellArgs& a, hipStream_t s);
// Dynamic LDS bytes of a launch of a (the largest over a batch's items).
size_t sell_launch_lds_bytes(const SellArgs& a);
// Scatter of CSR codes and columns into the slice layout.  start: per row
// position, the row's first entry in the CSR streams; pad_col: per group,
// the column written into padding slots.
hipError_t launch_sell_pack(int vf, int idx_bytes, const SellChunk* chunks, int64_t n_chunks,
                            const uint64_t* start, const uint32_t* len, const uint32_t* pad_col,
                            const void* codes_in, const void* col_in, void* codes_out, void* col_out,
                            hipStream_t s);
// Decoded FP32 values of the slice layout (E4M3 codes times their row's
// scale); padding slots give 0.
hipError_t launch_sell_decode(int vf, const SellChunk* chunks, int64_t n_chunks, const uint32_t* perm,
                              const uint32_t* len, const void* codes, const float* row_scale, float* out,
                              hipStream_t s);

}  // namespace dose
