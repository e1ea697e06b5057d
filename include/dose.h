/*
 * dose.h — C ABI of libdose, the MI355X (gfx950) dose-product library.
 *
 * The dose in every voxel is one sparse matrix-vector product d = A x
 * (paper Sec. II-A): A is the dose-deposition matrix, one row per voxel and
 * one column per pencil-beam spot, built once per plan and left unchanged
 * while the optimiser varies the spot weights x (Sec. II-A, Sec. IV).  The
 * paper stores A in compressed sparse row form with IEEE-754 half-precision
 * values and 32-bit column indices (Sec. II-C, II-D, Table I); this library
 * keeps that format and adds bfloat16 and 8-bit E4M3 values with a per-row
 * FP32 scale.  Every product accumulates in FP32 and is bitwise reproducible
 * from run to run: no reduction uses atomics (Sec. II-D).
 *
 * Conventions for every call:
 *   - Return value: DOSE_OK (0) or a negative dose_status; nothing throws or
 *     aborts across this boundary.  dose_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 *   - "device" pointers are HIP device memory of the current device, owned by
 *     the caller and valid until the work queued on `hip_stream` completes.
 *     "host" pointers are ordinary CPU memory, read or written before the call
 *     returns.
 *   - `hip_stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     Product calls only enqueue work on it and return; results are ready when
 *     the stream reaches them.
 *   - A dose_matrix is read-only after creation: products on several streams
 *     may use one matrix at the same time.  A dose_batch_plan is not
 *     thread-safe.
 */
#ifndef DOSE_H
#define DOSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dose_status;
enum {
  DOSE_OK = 0,
  DOSE_ERR_INVALID_ARGUMENT = -1, /* null pointer, size mismatch, aliasing x/y  */
  DOSE_ERR_BAD_CSR = -2,          /* row_ptr not monotone, column out of range,
                                     columns not strictly ascending in a row,
                                     value not finite                             */
  DOSE_ERR_UNSUPPORTED = -3,      /* value outside the format's range, sizes
                                     beyond the library's limits                  */
  DOSE_ERR_NO_TRANSPOSE = -4,     /* adjoint requested on a matrix created
                                     without DOSE_CREATE_TRANSPOSE                 */
  DOSE_ERR_OUT_OF_MEMORY = -5,    /* device or pinned host allocation failed     */
  DOSE_ERR_HIP = -6,              /* a HIP runtime call failed (message has it)  */
  DOSE_ERR_INTERNAL = -7
};

/* Stored value formats.  Decoding is exact in FP32 for all four.  Entry
 * points take formats as int32_t values of these enumerations, so that an
 * unknown value is an error (DOSE_ERR_INVALID_ARGUMENT), not undefined
 * behaviour of an out-of-range enumeration. */
typedef enum {
  DOSE_VAL_FP16 = 1,             /* IEEE binary16, the paper's format (Sec. II-D) */
  DOSE_VAL_BF16 = 2,             /* bfloat16                                     */
  DOSE_VAL_FP8E4M3_ROWSCALE = 3, /* OCP E4M3 (max 448) times an FP32 row scale   */
  DOSE_VAL_FP32 = 4              /* FP32 values as given: the paper's Single
                                    control (Sec. V), 4 bytes per value        */
} dose_value_format;

/* Column index formats.  A^T (DOSE_CREATE_TRANSPOSE) always stores 32-bit
 * indices: its columns are A's rows. */
typedef enum {
  DOSE_IDX_I32 = 1, /* 32-bit column indices, as in the paper (Sec. V)            */
  DOSE_IDX_U16 = 2, /* 16-bit column indices (n_cols <= 65536, else UNSUPPORTED):
                       the paper notes that column indices are a large part of
                       the bytes moved (Sec. V); 4 instead of 6 B per entry in
                       FP16 */
  DOSE_IDX_RUNS = 3 /* run-length column indices, SELL-C-sigma only: each row's
                       columns as its maximal runs of consecutive columns (a
                       dose row holds a few: the spots of a scanline, Sec. II-B),
                       8 B per run instead of 2 or 4 B per entry; at most 1024
                       runs per chunk of 64 rows (else DOSE_ERR_UNSUPPORTED);
                       dose_matrix_create refuses it (DOSE_ERR_UNSUPPORTED) */
} dose_index_format;

/* dose_matrix_create flags */
enum {
  DOSE_CREATE_TRANSPOSE = 1u, /* also store A^T for dose_spmv_adjoint */
  DOSE_CREATE_AUTOTUNE = 2u,  /* time the plain one-vector product (and the adjoint
                                 with DOSE_CREATE_TRANSPOSE) under row groups of 8K,
                                 16K, 32K and 64K entries on hip_stream and keep the
                                 fastest, as the paper sweeps its thread-block size
                                 (Sec. V-A); a choice stored in the DOSE_TUNE_CACHE
                                 file is reused.  Speed only: products are bitwise
                                 the same under any partition. */
  DOSE_CREATE_TRANSPOSE_SLABS = 4u /* store A^T in voxel slabs instead (implies
                                 DOSE_CREATE_TRANSPOSE): the voxels are cut into
                                 slabs of W consecutive rows of A (W = the LDS window
                                 cap, 4096 by default, reported as slab_voxels), and
                                 A^T gets one row per (slab, spot) pair holding
                                 entries, slab by slab, so that each row group of the
                                 adjoint reads v from one slab held in LDS instead
                                 of gathering it from global memory.  The adjoint
                                 sums each such row (a partial), then adds spot j's
                                 partials in ascending slab: deterministic and
                                 bitwise the same under any partition, but in a
                                 different order from the spot-row transpose (so
                                 not bitwise equal to it).  Needs
                                 ceil(n_rows / W) * n_cols < 2^32 (else
                                 DOSE_ERR_UNSUPPORTED); dose_matrix_decode of
                                 DOSE_PART_AT returns DOSE_ERR_UNSUPPORTED. */
};

/* Which stored operand dose_matrix_decode reads. */
enum { DOSE_PART_A = 0, DOSE_PART_AT = 1 };

typedef struct dose_matrix_s* dose_matrix;
typedef struct dose_batch_plan_s* dose_batch_plan;

/* A CSR matrix in host memory with FP32 source values (the form the paper
 * converts the planning system's own storage into, Sec. II-C, Sec. IV). */
typedef struct {
  int64_t n_rows;          /* voxels                                          */
  int64_t n_cols;          /* spots                                           */
  int64_t nnz;             /* stored entries                                  */
  const int64_t* row_ptr;  /* host, n_rows+1; [0]=0, non-decreasing, [n_rows]=nnz */
  const int32_t* col_idx;  /* host, nnz; in [0,n_cols), strictly ascending per row */
  const float* values;     /* host, nnz; finite                               */
} dose_csr_host;

typedef struct {
  int64_t n_rows, n_cols, nnz;
  int32_t value_format, index_format, has_transpose;
  int32_t group_nnz;            /* row-group size of the partition of A      */
  int64_t n_groups;             /* row groups of A                           */
  int64_t n_groups_windowed;    /* groups of A whose x window fits in LDS
                                   (single-vector products)                 */
  int32_t group_nnz_t;          /* the same for A^T (0 without transpose)    */
  int32_t slab_voxels;          /* W of DOSE_CREATE_TRANSPOSE_SLABS, else 0   */
  int64_t n_groups_t, n_groups_windowed_t;
  uint64_t device_bytes;        /* device memory held by the matrix          */
  uint64_t spmv_bytes;          /* algorithmic HBM bytes of one dose_spmv:
                                   nnz*(value+index) + (n_rows+1)*4 row
                                   offsets + n_rows*scale + 4*n_cols (x) +
                                   4*n_rows (y)                             */
  uint64_t adjoint_bytes;       /* the same for dose_spmv_adjoint on A^T
                                   (voxel slabs: plus the padding entries,
                                   8 B per slab row for its partial and 4 B
                                   per row and spot for the combine map)    */
  int64_t n_groups_split;       /* split groups of A: one long row whose
                                   steps the four waves share               */
  int64_t n_groups_split_t;     /* the same for A^T                          */
} dose_matrix_info_t;

/* Host-only check of a CSR matrix for a format: structure (row_ptr, column
 * range and order, finite values) and range (binary16 and bfloat16 values
 * must not round to infinity).  No GPU is touched.  Returns DOSE_OK,
 * DOSE_ERR_BAD_CSR, DOSE_ERR_UNSUPPORTED or DOSE_ERR_INVALID_ARGUMENT. */
dose_status dose_csr_validate(const dose_csr_host* csr, int32_t vf /* dose_value_format */,
                              int32_t xf /* dose_index_format */);

/* Encode a host CSR matrix into device streams (Sec. II-C: the conversion to
 * CSR happens once, before optimisation).  Validates first (as above).  The
 * value stream is the format's code of every FP32 source value, rounded to
 * nearest-even; for DOSE_VAL_FP8E4M3_ROWSCALE each row i gets the scale
 * s_i = fl32(max_j |a_ij| / 448) (1 when that is 0) and codes of
 * fl32(a_ij / s_i), saturated at 448.  With DOSE_CREATE_TRANSPOSE the
 * transpose is built on the device, its rows listing entries in ascending
 * row of A, with the same decoded values.  Uses the device that is current
 * on the calling thread; blocks until its uploads on `hip_stream` finish, so
 * the caller may free the host arrays on return.  *out owns all device memory
 * of the matrix until dose_matrix_destroy.  DOSE_ERR_UNSUPPORTED also when a
 * row of A (or, with DOSE_CREATE_TRANSPOSE, of A^T: a column of A) holds 2^28
 * or more entries, or the transpose would hold 2^31 or more. */
dose_status dose_matrix_create(const dose_csr_host* csr, int32_t vf /* dose_value_format */,
                               int32_t xf /* dose_index_format */, uint32_t flags, void* hip_stream,
                               dose_matrix* out);

/* Re-partition a matrix (A, and A^T if stored) into row groups of about
 * group_nnz entries (a power of two, 1024 .. 2^20; a longer row is a group of
 * its own).  A group is the work of one workgroup.  The partition changes
 * speed only: every row is summed in an order fixed by its own entries, so
 * products are bitwise identical under any partition.  Synchronous: waits
 * for the device first.  The one call that changes a matrix after creation:
 * it must not overlap products on the same matrix issued from other threads.
 * Batch plans keep copies of the partition they were built with. */
dose_status dose_matrix_set_partition(dose_matrix m, int32_t group_nnz, int32_t group_nnz_t);

/* Copy rows [row_begin, row_end) of the stored operand `part` (DOSE_PART_A or
 * DOSE_PART_AT) back to the host, decoded to FP32 on the device.
 * row_ptr_out: host, row_end-row_begin+1 offsets, the first one 0.
 * col_out, val_out: host, as many entries as the rows hold (may be NULL to
 * query the offsets only).  Synchronous. */
dose_status dose_matrix_decode(dose_matrix m, int32_t part, int64_t row_begin, int64_t row_end,
                               int64_t* row_ptr_out, int32_t* col_out, float* val_out);

dose_status dose_matrix_info(dose_matrix m, dose_matrix_info_t* info);

/* Frees the matrix's device memory after synchronising its device. */
dose_status dose_matrix_destroy(dose_matrix m);

/* y = A x (Listing 1 of the paper; the dose in every voxel).
 * x: device, n_cols FP32, 4-byte aligned, else DOSE_ERR_INVALID_ARGUMENT
 * (16-byte alignment is faster: the kernels read x in 16-byte pieces).  y: device, n_rows FP32, every entry
 * written (+0 for empty rows).  x and y must not overlap.  Asynchronous on
 * hip_stream. */
dose_status dose_spmv(dose_matrix m, const float* x, float* y, void* hip_stream);

/* g = A^T v, the gradient of an objective of the dose with respect to the
 * spot weights when v is the objective's derivative with respect to the dose
 * (plan optimisation needs gradients every iteration, Sec. I).  Runs the same
 * kernels on the stored transpose: deterministic, no atomics.
 * v: device, n_rows FP32.  g: device, n_cols FP32, every entry written.
 * Both 4-byte aligned (else DOSE_ERR_INVALID_ARGUMENT, as for x and y).
 * DOSE_ERR_NO_TRANSPOSE without DOSE_CREATE_TRANSPOSE.  E4M3 with row
 * scales: the row scales are applied to v first, u_i = fl32(s_i v_i), and
 * entry (i, j) adds fl32(q_ij u_i) (two roundings per term, as fl32(fl32(q_ij
 * s_i) v_i) would have; one gathered value per entry instead of two); the
 * call takes n_rows * 4 bytes of stream-ordered device memory for u.  With
 * DOSE_CREATE_TRANSPOSE_SLABS it also takes 4 bytes (FP64: 8) per slab row
 * for the partials. */
dose_status dose_spmv_adjoint(dose_matrix m, const float* v, float* g, void* hip_stream);

/* The same products with FP64 vectors and FP64 products and sums: the
 * paper's half/double configuration (Sec. II-D: FP16 matrix values, FP64
 * spot weights and dose).  The stored matrix is the same (any value and
 * index format); each product is decoded exactly to FP64, the row sums
 * follow the order of the FP32 products in FP64, and the E4M3 row scale
 * multiplies the FP64 row sum (forward) or the code in FP32, as in the FP32
 * adjoint (adjoint).  x (v): device, n_cols (n_rows) FP64; y (g): device,
 * n_rows (n_cols) FP64, every entry written; all 8-byte aligned, else
 * DOSE_ERR_INVALID_ARGUMENT; inputs and outputs must not overlap.
 * Asynchronous on hip_stream.  The adjoint needs DOSE_CREATE_TRANSPOSE
 * (else DOSE_ERR_NO_TRANSPOSE). */
dose_status dose_spmv_f64(dose_matrix m, const double* x, double* y, void* hip_stream);
dose_status dose_spmv_adjoint_f64(dose_matrix m, const double* v, double* g, void* hip_stream);

/* One item of a batched product: y = A x for n_rhs spot-weight vectors,
 * x stored [n_cols][ldx] and y [n_rows][ldy] (vector r at offset r).
 * n_rhs is 1, 2 or 4; ldx == ldy == n_rhs. */
typedef struct {
  dose_matrix A;
  int32_t n_rhs;
  int32_t reserved;
  const float* x; /* device */
  int64_t ldx;
  float* y;       /* device */
  int64_t ldy;
} dose_batch_item;

/* All items in one launch (robust optimisation needs the dose of many
 * scenarios and beams every iteration, Sec. I, II-A: one matrix per beam and
 * scenario, Sec. II-B).  Each y is bitwise what dose_spmv gives per vector
 * (rows are summed in the same order).  Items must not share outputs; x and y
 * of an item must not overlap and must be aligned to n_rhs floats; all items
 * share one value format, one index format and one n_rhs, and live on one
 * device (else DOSE_ERR_UNSUPPORTED or DOSE_ERR_INVALID_ARGUMENT).
 * Asynchronous on hip_stream: the items' arguments travel to the device
 * through a library-owned pinned ring of 16 slots (kept until the process
 * ends), so the call returns once the launch is queued; it waits only when
 * the launch that used the same slot 16 calls earlier has not finished.  At
 * most 2,048 items per call (DOSE_ERR_UNSUPPORTED beyond; a batch plan takes
 * any number).  Not for HIP graph capture: capture a batch plan instead. */
dose_status dose_spmv_batched(const dose_batch_item* items, int32_t n_items, void* hip_stream);

/* Plans (the same batched product, repeated every optimisation iteration,
 * Sec. I, II-A): the work list of a batch is built once on the device and the
 * launch is captured into a HIP graph that dose_batch_plan_launch replays on
 * hip_stream (asynchronous).  The plan keeps the items' pointers: their x and
 * y, and the matrices themselves (their device streams), must stay valid while
 * the plan is used; dose_matrix_set_partition on them does not affect it
 * (the plan holds its own copies of the row-group descriptors).  With DOSE_PLAN_AUTOTUNE each
 * distinct matrix is timed under candidate row-group sizes on `hip_stream`
 * (x/y of the items are used as scratch for the timing runs; the choice
 * persists in the text file named by DOSE_TUNE_CACHE, if set) and the plan
 * keeps its own copy of the fastest partition: the matrix is not changed, so
 * products on other streams may use it meanwhile, as for any product.  The
 * paper sweeps its thread-block size for the same reason (Sec. V-A); the
 * partition changes speed only, never the result.  create is synchronous. */
enum { DOSE_PLAN_AUTOTUNE = 1u };
dose_status dose_batch_plan_create(const dose_batch_item* items, int32_t n_items, uint32_t flags,
                                   void* hip_stream, dose_batch_plan* out);
dose_status dose_batch_plan_launch(dose_batch_plan p, void* hip_stream);

/* One item of an adjoint plan: g = A^T v for a matrix created with
 * DOSE_CREATE_TRANSPOSE or DOSE_CREATE_TRANSPOSE_SLABS.  v: device, n_rows
 * FP32; g: device, n_cols FP32, every entry written; both 4-byte aligned. */
typedef struct {
  dose_matrix A;
  int32_t reserved; /* 0 */
  const float* v;
  float* g;
} dose_adjoint_item;

/* An adjoint plan: the gradients of every item (a robust objective needs the
 * adjoint of every beam's matrix under every scenario each iteration, Sec. I,
 * II-A) captured once into a HIP graph that dose_batch_plan_launch replays on
 * hip_stream (asynchronous) and dose_batch_plan_destroy frees: E4M3 seeds
 * scaled by the row scales, one launch over the row groups of every item's
 * stored transpose, and (voxel slabs) each item's combine of its slab
 * partials.  Each g is bitwise what dose_spmv_adjoint writes for its item
 * (unless accumulated, below).  All items: a stored transpose (else
 * DOSE_ERR_NO_TRANSPOSE), the same value format and transpose layout (spot
 * rows or voxel slabs; else DOSE_ERR_UNSUPPORTED) and the same device; an
 * item's v and g apart; no g overlapping another item's v or g (items may
 * share v; else DOSE_ERR_INVALID_ARGUMENT).  The plan keeps the items' pointers
 * (v, g and the matrices must stay valid while it is used; re-partitioning
 * a matrix does not affect it) and owns its scratch (n_rows
 * floats per E4M3 item, one per slab row per slab item): overlapping
 * launches of one plan race.  The row groups are sized for the whole launch
 * (plan-owned partitions); with flags DOSE_PLAN_AUTOTUNE the launch is timed
 * on hip_stream under groups of 8K, 16K, 32K and 64K entries and the fastest
 * kept (speed only; the items' g and the plan's scratch are written by the
 * timing runs).  With DOSE_ADJOINT_ACCUMULATE (voxel slabs only, else
 * DOSE_ERR_UNSUPPORTED) items may share the very same g (with as many
 * spots): it receives the sum over those items of A_i^T v_i, formed as one
 * fixed-order sum from +0 of their slab partials, item by item in item order,
 * each item's in ascending slab (the robust gradient of a beam: its
 * matrices under every scenario with each scenario's seed, summed by the
 * library; at most 65,535 distinct outputs).  Other flags:
 * DOSE_ERR_INVALID_ARGUMENT.  create is synchronous. */
enum { DOSE_ADJOINT_ACCUMULATE = 2u };
dose_status dose_adjoint_plan_create(const dose_adjoint_item* items, int32_t n_items, uint32_t flags,
                                     void* hip_stream, dose_batch_plan* out);

/* Scenario doses of a robust plan in one plan launch, the beam sum done by
 * the products themselves (Sec. I, II-A: the dose of every beam under every
 * scenario, every iteration; one matrix per beam, Sec. II-B).  Scenario s's
 * dose is d[s][v] = A_{s,0} x_{s,0} + A_{s,1} x_{s,1} + ... at voxel v, the
 * FP32 sum of its beam doses in ascending beam order: the same bits as the
 * beam products of dose_spmv_batched followed by the beam sum of
 * dose_scenario_objective (whose d_out it equals), without writing or reading
 * the beam doses.  The plan holds one launch per beam, in beam order, over
 * all scenarios: beam 0's products store the voxel doses, every later beam's
 * products add theirs to them (empty rows add +0); the launches are captured
 * in one HIP graph that dose_batch_plan_launch replays.
 *   mats: host array of n_scen * n_beams matrices, [s * n_beams + b], all
 *         with the same number of rows (voxels) and one value and index format.
 *   x:    host array of n_scen * n_beams device pointers, FP32 spot weights
 *         of each matrix (the same beam may share them across scenarios).
 *   d:    device FP32 [n_scen][n_rows], written; must not overlap any x.
 * flags: DOSE_PLAN_AUTOTUNE as for dose_batch_plan_create (d is the timing
 * runs' scratch).  Synchronous; the plan keeps the pointers.  Errors as for
 * dose_batch_plan_create; DOSE_ERR_INVALID_ARGUMENT also for matrices of
 * different row counts.  Destroy with dose_batch_plan_destroy. */
dose_status dose_scenario_plan_create(const dose_matrix* mats, const float* const* x, int32_t n_scen,
                                      int32_t n_beams, float* d, uint32_t flags, void* hip_stream,
                                      dose_batch_plan* out);
dose_status dose_batch_plan_destroy(dose_batch_plan p);

/* Quadratic plan objective f = sum_v w_v (d_v - p_v)^2, accumulated in FP64
 * with a fixed-order two-pass reduction, and the adjoint seed
 * seed_v = 2 w_v (d_v - p_v) in FP32 (may be NULL).  Plan optimisation
 * evaluates the objective and its gradient from the dose every iteration
 * (Sec. I); the paper fixes no objective, so this is the usual quadratic
 * penalty of the dose against a prescription p with voxel weights w.
 * d, p, w: device, n FP32.  f_out: device, one double.  Asynchronous on
 * hip_stream; a partial-sum buffer of at most 8 KB is taken from the
 * stream-ordered allocator and returned in stream order. */
dose_status dose_objective(int64_t n, const float* d, const float* p, const float* w,
                           float* seed, double* f_out, void* hip_stream);

/* Robust-optimisation epilogue (Sec. I, II-A: the dose of several beams under
 * several realisations of the uncertainties is needed every iteration).
 * n_scen scenarios of n_beams beams each share one dose grid of n voxels.
 *   part:  device FP32 [n_scen][n_beams][n], the beam doses (for instance the
 *          outputs of one dose_spmv_batched call, one item per beam).
 *   d_s,v  = part[s][0][v] + part[s][1][v] + ..., in ascending beam order in
 *          FP32; written to d_out [n_scen][n] unless d_out is NULL.
 *   f_s    = sum_v w_v (d_s,v - p_v)^2, FP64, the fixed-order two-pass
 *          reduction of dose_objective (with one scenario of one beam, the
 *          same f bit for bit).
 *   seed (may be NULL): FP32 [n_scen][n], seed_s,v = 2 w_v (d_s,v - p_v).
 *   out:   device, n_scen + 3 doubles: f_0 .. f_{n_scen-1}, then the worst
 *          case max_s f_s, the expectation sum_s prob_s f_s (ascending s;
 *          (sum_s f_s) / n_scen when prob is NULL), then the index of the
 *          first scenario attaining the worst case.
 *   prob:  device, n_scen doubles, or NULL.
 * p, w: device FP32 [n].  Float arrays 4-byte, double arrays 8-byte aligned;
 * 1 <= n_scen, n_beams <= 65536; outputs must not overlap inputs or each
 * other; else DOSE_ERR_INVALID_ARGUMENT.  Asynchronous on hip_stream. */
dose_status dose_scenario_objective(int32_t n_scen, int32_t n_beams, int64_t n, const float* part,
                                    const float* p, const float* w, const double* prob, float* d_out,
                                    float* seed, double* out, void* hip_stream);

/* The same epilogue for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * partial sums live in a library-owned static device array of 65,536 doubles
 * (512 KB, one per device, held until the process ends) instead of the
 * stream-ordered allocation; nothing is allocated, on the device or the host.
 * Limit: n_scen * p <= 65,536 with p = min(1024, max(1, ceil(n / 4096)))
 * partial sums per scenario (at most 64 scenarios for n above 4,190,208
 * voxels), else DOSE_ERR_INVALID_ARGUMENT.  Results are bit for bit those of
 * dose_scenario_objective.  Every call on one device shares the array, so
 * calls that overlap on one device (on different streams, or from different
 * threads) race and must be ordered by the caller; each call rewrites every
 * partial sum it reads, so nothing carries over from an earlier call.  Other
 * arguments and errors as for dose_scenario_objective.  Asynchronous. */
dose_status dose_scenario_objective_noalloc(int32_t n_scen, int32_t n_beams, int64_t n, const float* part,
                                            const float* p, const float* w, const double* prob,
                                            float* d_out, float* seed, double* out, void* hip_stream);

/* out = sqrt(sum_j g_j^2) in FP64, fixed-order two-pass reduction: the size
 * of the gradient an optimiser needs every iteration (Sec. I).
 * g: device, n FP32.  out: device, one double.  Asynchronous on hip_stream
 * (partial sums as for dose_objective). */
dose_status dose_norm2(int64_t n, const float* g, double* out, void* hip_stream);

/* Seeds of the robust objective's gradient (Sec. I, II-A: the gradient of the
 * robust plan objective every iteration).  The derivative of the expectation
 * with respect to scenario s's dose is prob_s (1/n_scen when prob is NULL)
 * times the scenario's seed; that of the worst case is the seed of the first
 * worst scenario (its index in out[n_scen + 2], as dose_scenario_objective
 * writes it) and 0 for the others.  So
 *   wseed[s][v] = fl32(c_s * g * seed[s][v]),  formed in FP64, rounded once,
 * with g = *grad_scale (an outer derivative; 1 when grad_scale is NULL).
 * Every beam b of scenario s then has gradient seed wseed[s] (its adjoint
 * gives that beam's spot-weight gradient under scenario s).
 * mode: DOSE_ROBUST_EXPECTED or DOSE_ROBUST_WORST.  out: device, n_scen + 3
 * doubles (needed for the worst case, else may be NULL).  prob: device,
 * n_scen doubles or NULL.  seed, wseed: device FP32 [n_scen][n]; wseed may be
 * seed itself, else must not overlap it or the other inputs.  Float arrays
 * 4-byte, double arrays 8-byte aligned; 1 <= n_scen <= 65536.  Errors:
 * DOSE_ERR_INVALID_ARGUMENT.  Asynchronous on hip_stream. */
enum { DOSE_ROBUST_EXPECTED = 0, DOSE_ROBUST_WORST = 1 };
dose_status dose_robust_seed(int32_t n_scen, int64_t n, int32_t mode, const double* out, const double* prob,
                             const double* grad_scale, const float* seed, float* wseed, void* hip_stream);

/* Measurement kernels (not part of the dose path): read `bytes` of device
 * memory with 16-byte loads and write one float per workgroup to `sink`
 * (device, 65536 floats), or copy `bytes` from src to dst.  Used to find the
 * achievable HBM read rate and to calibrate hardware byte counters. */
dose_status dose_probe_stream_read(const void* buf, uint64_t bytes, float* sink, void* hip_stream);
dose_status dose_probe_copy(const void* src, void* dst, uint64_t bytes, void* hip_stream);

/* Host-only view of the row-group partition for a row_ptr and group size.
 * Writes up to `cap` groups, 6 int64 each: r0 <= r1 <= r2 <= r3 <= r4 and a
 * split flag.  A group holds rows [r0, r4).  Without the flag its wave w
 * computes rows [r_w, r_(w+1)); with it the group is the single row r0
 * (r1 = ... = r4 = r0 + 1), longer than max(group_nnz / 4, 2048) entries,
 * and its four waves share that row's steps.  Returns the number of groups
 * in *n_groups. */
dose_status dose_partition_preview(const int64_t* row_ptr, int64_t n_rows, int32_t group_nnz,
                                   int64_t* groups, int64_t cap, int64_t* n_groups);

/* ----------------------------------------------------------- SELL-C-sigma
 * The SIMD-oriented sparse format the paper names as the next one to try for
 * dose matrices (Sec. II-C, Sec. VII): SELL-C-sigma (Kreutzer et al., SIAM
 * J. Sci. Comput. 36(5), 2014) with C = 64, one row per lane of a wave64.
 * The rows are taken in consecutive windows of sigma rows, each window
 * ordered by descending row length (rows of equal length keep their order),
 * and the resulting sequence of rows is cut into chunks of 64 positions; a
 * chunk is as wide as its longest row.  The device stores each chunk's
 * entries in slices of 8 entries per row (a lane's 8 codes are contiguous);
 * dose_sell_decode returns Kreutzer's column-major layout. */
typedef struct dose_sell_s* dose_sell;

typedef struct {
  int64_t n_rows, n_cols, nnz;
  int32_t value_format, index_format;
  int32_t chunk_rows;         /* C = 64                                       */
  int32_t sigma;
  int64_t n_chunks;           /* ceil(n_rows / 64)                            */
  int64_t n_groups;           /* row groups: one chunk each (chunk count
                                 rounded up to whole groups)                  */
  int64_t n_groups_windowed;  /* groups whose x window fits in LDS            */
  int64_t std_slots;          /* 64 * sum of chunk widths: Kreutzer's layout  */
  int64_t n_runs;             /* DOSE_IDX_RUNS: runs stored (else 0)          */
  int64_t stored_slots;       /* slots held on the device (widths rounded up
                                 to whole slices of 8)                        */
  uint64_t device_bytes;
  uint64_t spmv_bytes;        /* algorithmic bytes of one product: every code,
                                 index and row offset read once, x read and y
                                 written once, as in dose_matrix_info (with
                                 DOSE_IDX_RUNS: nnz * value + 8 per run + 4 per
                                 row offset + scale + 4 n_cols + 4 n_rows)     */
  uint64_t stream_bytes;      /* what one SELL product reads and writes:
                                 stored_slots * (value + index) + 8 per row
                                 (its position's row and length), + 8 per run
                                 and 4 per row with DOSE_IDX_RUNS, + scale +
                                 4 n_cols + 4 n_rows                           */
} dose_sell_info_t;

/* Host-only layout for a row_ptr: perm[k] (n_rows entries) is the row at
 * sorted position k, width[c] (ceil(n_rows / 64) entries) the length of the
 * longest row of chunk c.  sigma in [1, 2^31).  No GPU is touched. */
dose_status dose_sell_layout(const int64_t* row_ptr, int64_t n_rows, int32_t sigma, int64_t* perm,
                             int64_t* width);

/* Builds the SELL-C-sigma form of a host CSR matrix on the current device
 * (validated and encoded as by dose_matrix_create, including the E4M3 row
 * scale).  Synchronous, like dose_matrix_create; *out owns the device
 * memory until dose_sell_destroy.  DOSE_ERR_UNSUPPORTED beyond 2^32 - 2 rows
 * or 2^32 slices. */
dose_status dose_sell_create(const dose_csr_host* csr, int32_t vf /* dose_value_format */,
                             int32_t xf /* dose_index_format */,
                             int32_t sigma, void* hip_stream, dose_sell* out);

dose_status dose_sell_info(dose_sell m, dose_sell_info_t* info);

/* Kreutzer's layout on the host, values decoded to FP32: perm (n_rows) and
 * width (n_chunks) as dose_sell_layout gives them; val, col (std_slots
 * entries): entry j of the row at position c * 64 + i at
 * 64 * (width_0 + ... + width_(c-1)) + 64 j + i, slots past the row's end
 * 0 and column -1.  Synchronous. */
dose_status dose_sell_decode(dose_sell m, int64_t* perm, int64_t* width, float* val, int32_t* col);

/* DOSE_IDX_RUNS: the stored runs, read back from the device, by row of A (not
 * by sorted position): run_ptr (host, n_rows + 1, [0] = 0), start and length
 * (host, n_runs each): row i's columns are start[r], ..., start[r] +
 * length[r] - 1 for r in [run_ptr[i], run_ptr[i + 1]), in order, each run
 * maximal.  DOSE_ERR_INVALID_ARGUMENT for other index formats.  Synchronous. */
dose_status dose_sell_runs(dose_sell m, int64_t* run_ptr, int32_t* start, int32_t* length);

/* y = A x over the SELL-C-sigma form (the product of Listing 1 in another
 * storage order).  x: device, n_cols FP32; y: device, n_rows FP32, every
 * entry written (+0 for empty rows); both 4-byte aligned, not overlapping
 * (else DOSE_ERR_INVALID_ARGUMENT).  Rows are summed in an order fixed by
 * the layout (FP32; see the product kernel), so results repeat bit for bit
 * and the three index formats give the same bits.  Asynchronous on
 * hip_stream. */
dose_status dose_sell_spmv(dose_sell m, const float* x, float* y, void* hip_stream);

/* y = A x for one FP64 vector over the SELL-C-sigma form: FP64 x (device,
 * n_cols), FP64 y (device, n_rows, every entry written), FP64 products and
 * sums in dose_sell_spmv's order (the paper's half/double arithmetic,
 * Sec. II-D).  Both 8-byte aligned, not overlapping (else
 * DOSE_ERR_INVALID_ARGUMENT); n_cols below 2^30 (else DOSE_ERR_UNSUPPORTED).
 * Asynchronous on hip_stream. */
dose_status dose_sell_spmv_f64(dose_sell m, const double* x, double* y, void* hip_stream);

/* Y = A X for n_rhs spot-weight vectors at once (n_rhs 1, 2 or 4; the
 * multi-vector product of robust planning, Sec. I, II-A): x device
 * [n_cols][n_rhs], y device [n_rows][n_rhs] FP32, row-major (vector r at
 * offset r), both aligned to n_rhs floats, not overlapping (else
 * DOSE_ERR_INVALID_ARGUMENT); n_cols * n_rhs below 2^31 (else
 * DOSE_ERR_UNSUPPORTED).  Every entry is read once; each vector's rows are
 * summed in dose_sell_spmv's order, so column r of y is bitwise
 * dose_sell_spmv of column r of x.  Asynchronous on hip_stream. */
dose_status dose_sell_spmv_multi(dose_sell m, int32_t n_rhs, const float* x, float* y, void* hip_stream);

/* One item of a batched SELL-C-sigma product: Y = S X as for
 * dose_sell_spmv_multi, with ldx == ldy == n_rhs. */
typedef struct {
  dose_sell S;
  int32_t n_rhs;
  int32_t reserved;
  const float* x; /* device */
  int64_t ldx;
  float* y;       /* device */
  int64_t ldy;
} dose_sell_batch_item;

/* A plan of many SELL-C-sigma products in ONE launch (the batch of matrices
 * robust optimisation multiplies every iteration, Sec. I, II-A, II-B): the
 * chunks of every item form one work list on the device, captured into a HIP
 * graph that dose_batch_plan_launch replays (destroy with
 * dose_batch_plan_destroy).  Each y is bitwise dose_sell_spmv_multi's.  All
 * items share one value format, one index format and one n_rhs and live on
 * one device (else DOSE_ERR_UNSUPPORTED / DOSE_ERR_INVALID_ARGUMENT); no y
 * may overlap another item's y or any item's x.  flags must be 0.  The plan
 * keeps the items' pointers.  Synchronous. */
dose_status dose_sell_batch_plan_create(const dose_sell_batch_item* items, int32_t n_items, uint32_t flags,
                                        void* hip_stream, dose_batch_plan* out);

/* Frees the device memory after synchronising the device. */
dose_status dose_sell_destroy(dose_sell m);

const char* dose_status_string(dose_status s);
const char* dose_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DOSE_H */
