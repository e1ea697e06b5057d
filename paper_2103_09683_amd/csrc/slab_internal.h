// A^T stored in voxel slabs: the device steps of building it and the combine
// that finishes its adjoint.
//
// The adjoint g = A^T v sums, for every spot j, the entries of column j of A
// times the seed v over the voxels (Sec. I: a gradient every iteration).  A
// column of A runs through the whole depth of the dose grid, far wider than
// an LDS window of v, so the slab form cuts the voxel range into slabs of W
// consecutive voxels and stores A^T with one row per (slab, spot) pair that
// holds entries, ordered slab by slab and, within a slab, by spot; each row
// lists its entries in ascending voxel, as 16-bit offsets from the slab's
// first voxel (the row groups' column base).  The row products are partial sums
// P[r] whose row groups each read v from one slab (so from LDS); the spot's
// result is the sum of its rows' partials in ascending slab order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dose {

// keys[k] = (rows[k] / slab) * n_cols + cols[k]: the (slab, spot) of entry k.
hipError_t launch_slab_keys(const uint32_t* rows, const uint32_t* cols, uint32_t slab, uint32_t n_cols,
                            int64_t n, uint32_t* keys, hipStream_t s);

// The distinct keys of a sorted key array and their run lengths (n_runs is
// written to device memory).  tmp == nullptr: *tmp_bytes gets the scratch size.
hipError_t run_length_encode(void* tmp, size_t* tmp_bytes, const uint32_t* keys, uint32_t* unique, uint32_t* counts,
                             uint32_t* n_runs, int64_t n, hipStream_t s);

// Entry k of the key-sorted order (A's entry perm[k], of A's row rows[perm[k]]
// and key keys[k], slab t = keys[k] / n_cols) goes to position k + slab_off[t]
// of the slab stream: its code, and as its column the voxel's offset from the
// slab's first voxel, rows[perm[k]] - t * slab (16 bits: slab <= 65536).
hipError_t launch_slab_gather(int vf, const uint32_t* perm, const uint32_t* rows, const uint32_t* keys,
                              uint32_t n_cols, uint32_t slab, const uint32_t* slab_off, const void* codes_in,
                              void* codes_out, uint16_t* col_out, int64_t n, hipStream_t s);

// g[j] = sum of part[rows[k]] for k from ptr[j] to ptr[j+1] - 1, added in
// ascending k (ascending slab), starting from +0; f64 selects FP64 partials
// and results.
hipError_t launch_slab_combine(bool f64, const void* part, const uint32_t* ptr, const uint32_t* rows, void* g,
                               int64_t n_cols, hipStream_t s);

// The FP32 combines of several slab adjoints in one launch (adjoint plans).
// Output group k writes g[j] for j < n_cols: starting from +0, for each of
// its items i = first .. first + count - 1 in turn, the item's partials of
// spot j in ascending slab (a group of one item: what launch_slab_combine
// writes).  Items and groups in device memory.
struct SlabCombineItem {
  const float* part;
  const uint32_t* ptr;
  const uint32_t* rows;
};
struct SlabCombineGroup {
  float* g;
  int64_t n_cols;
  int32_t first, count;
};
hipError_t launch_slab_combine_groups(const SlabCombineGroup* groups, int32_t n_groups, const SlabCombineItem* items,
                                      int64_t max_cols, hipStream_t s);

// The E4M3 seed scalings of an adjoint plan in one launch: item i (items in
// device memory) writes u[k] = fl32(scale[k] * v[k]) for k < n, as
// launch_scale_vec does.
struct ScaleItem {
  const float* scale;
  const float* v;
  float* u;
  int64_t n;
};
hipError_t launch_scale_items(const ScaleItem* items, int32_t n_items, int64_t max_n, hipStream_t s);

}  // namespace dose
