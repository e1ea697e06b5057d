// SpMV kernels of libdose for gfx950 (CDNA4, wave64).
//
// The product is Listing 1 of the paper: y_i = sum over row i's stored
// entries of data[k] * x[col[k]], a wavefront reducing each row (the paper
// uses one 32-lane warp per row, Sec. III).  The gfx950 design:
//
//   * A workgroup (four wave64 waves) takes a *row group*: a run of whole rows
//     holding about group_nnz entries, or one long row (a split group).  Dose
//     rows of neighbouring voxels touch a narrow range of spots, so the
//     group's columns span a short window of x; the workgroup copies that
//     window into LDS once and every gather is an LDS read.  A group whose
//     window does not fit reads x from global memory instead.
//   * Each wave owns a contiguous share of the group's rows and streams its
//     entries in *steps* of 512 entries on absolute multiples of 512: lane l
//     of a step loads the two 4-entry quarters at 4 l and 256 + 4 l of it
//     (codes and column indices, non-temporal), so every load instruction
//     reads one contiguous range and each cache line is requested once.  The
//     next step's loads are in flight while one is computed, and with an LDS
//     window a step's buffer is refilled as soon as its products are formed.
//     In a split group wave j takes the steps j, j+4, ... of the row.
//   * Instruction issue and the compute between a step's arrival and its
//     refill set the pace as much as HBM does, so the per-entry work is kept
//     short: FP16 decode and product are one v_fma_mix, E4M3 is converted by
//     the hardware two codes at a time, the LDS address of x is one
//     shift-add, and a lane tests whether an entry belongs to a row with one
//     unsigned compare of its position.
//   * The same kernels, instantiated for FP64 vectors (k_spmv_f64), give FP64
//     products and sums in the same order.
//   * Summation order, fixed by the row's entries and their absolute
//     positions only (not by the partition, the launch or timing; nothing is
//     atomic), so equal inputs give equal bits (Sec. II-D), a split row equals
//     the same row summed by one wave, and batched products equal plain ones:
//       - a row meeting at most 4 steps: each lane adds, step by step and
//         first quarter before second, the pairwise sums of its entries of the
//         row in each quarter that holds any of them ((a + b) + (c + d),
//         entries outside the row as +0), starting from -0; the 64 lane sums
//         then meet in one fixed DPP reduction;
//       - a longer row: per step, the lane sum of its entries of the row
//         (first-quarter sum + second-quarter sum) goes through the DPP
//         reduction, giving T_s; W_j adds the T_s of the row's steps s with
//         (s - first step) = j (mod 4) in order, and the row is
//         (W_0 + W_1) + (W_2 + W_3).
#include "dose_internal.h"

#include <hip/hip_fp16.h>

#include <cstdlib>

// Products are rounded before they are summed, in every kernel instance: no
// multiply-add contraction (it would make the bits depend on which instance
// summed a row).
#pragma clang fp contract(off)

namespace dose {
namespace {

constexpr int kWave = 64;
constexpr int kQuarter = kQuarterEntries;
constexpr int kHalf = kStepEntries / 2;  // the second quarter of a lane sits kHalf entries after the first

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Streamed data is read once: non-temporal loads, at a uniform base plus a
// 32-bit byte offset per lane.
__device__ __forceinline__ uint4 ld_nt4(const char* base, uint32_t off) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + off));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_nt2(const char* base, uint32_t off) {
  const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base + off));
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint32_t ld_nt1(const char* base, uint32_t off) {
  return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(base + off));
}

// ----------------------------------------------------------------- decoding
__device__ __forceinline__ float dec_fp16(uint32_t h) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(h)));
}

// The 8 codes of a lane's step (entries 0..3: first quarter, 4..7: second).
template <int VF>
struct Codes;
template <>
struct Codes<kFp16> {
  static constexpr uint32_t kBytes = 2;
  uint4 w;
  __device__ __forceinline__ void load(const char* base, uint32_t k1, uint32_t k2) {
    const uint2 h1 = ld_nt2(base, k1 * kBytes), h2 = ld_nt2(base, k2 * kBytes);
    w = make_uint4(h1.x, h1.y, h2.x, h2.y);
  }
  // the code as binary16 widened to float: fed straight into an FMA it
  // becomes an operand of v_fma_mix_f32
  __device__ __forceinline__ float get(int e) const {
    const uint32_t word = e < 2 ? w.x : e < 4 ? w.y : e < 6 ? w.z : w.w;
    return dec_fp16((word >> ((e & 1) * 16)) & 0xFFFFu);
  }
};
template <>
struct Codes<kBf16> {
  static constexpr uint32_t kBytes = 2;
  uint4 w;
  __device__ __forceinline__ void load(const char* base, uint32_t k1, uint32_t k2) {
    const uint2 h1 = ld_nt2(base, k1 * kBytes), h2 = ld_nt2(base, k2 * kBytes);
    w = make_uint4(h1.x, h1.y, h2.x, h2.y);
  }
  __device__ __forceinline__ float get(int e) const {
    const uint32_t word = e < 2 ? w.x : e < 4 ? w.y : e < 6 ? w.z : w.w;
    return __uint_as_float((e & 1) ? (word & 0xFFFF0000u) : (word << 16));
  }
};
template <>
struct Codes<kFp8> {
  static constexpr uint32_t kBytes = 1;
  uint2 w;
  __device__ __forceinline__ void load(const char* base, uint32_t k1, uint32_t k2) {
    w = make_uint2(ld_nt1(base, k1), ld_nt1(base, k2));
  }
  // OCP E4M3 to float by the hardware (exact), two codes per instruction.
  // The encoder never emits the NaN code.
  __device__ __forceinline__ void decode(float (&d)[kChunk]) const {
    const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w.x), false);
    const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w.x), true);
    const f32x2 c = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w.y), false);
    const f32x2 e = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w.y), true);
    d[0] = a.x, d[1] = a.y, d[2] = b.x, d[3] = b.y, d[4] = c.x, d[5] = c.y, d[6] = e.x, d[7] = e.y;
  }
};

template <>
struct Codes<kFp32> {
  static constexpr uint32_t kBytes = 4;
  uint4 wa, wb;
  __device__ __forceinline__ void load(const char* base, uint32_t k1, uint32_t k2) {
    wa = ld_nt4(base, k1 * kBytes);
    wb = ld_nt4(base, k2 * kBytes);
  }
  __device__ __forceinline__ float get(int e) const {
    const uint4& w = e < 4 ? wa : wb;
    const int i = e & 3;
    return __uint_as_float(i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w);
  }
};

// Column indices of 4 consecutive entries: four int32 (IX = 4) or four
// uint16 (IX = 2).
template <int IX>
struct ColQuad;
template <>
struct ColQuad<4> {
  uint4 w;
  __device__ __forceinline__ void load(const char* col, uint32_t k) { w = ld_nt4(col, k * 4u); }
  __device__ __forceinline__ void get(int (&c)[4]) const {
    c[0] = static_cast<int>(w.x), c[1] = static_cast<int>(w.y), c[2] = static_cast<int>(w.z), c[3] = static_cast<int>(w.w);
  }
};
template <>
struct ColQuad<2> {
  uint2 w;
  __device__ __forceinline__ void load(const char* col, uint32_t k) { w = ld_nt2(col, k * 2u); }
  __device__ __forceinline__ void get(int (&c)[4]) const {
    c[0] = static_cast<int>(w.x & 0xFFFFu), c[1] = static_cast<int>(w.x >> 16);
    c[2] = static_cast<int>(w.y & 0xFFFFu), c[3] = static_cast<int>(w.y >> 16);
  }
};

// One lane's share of one step: 8 codes and 8 columns, entries 4 l .. 4 l + 3
// and 256 + 4 l .. 256 + 4 l + 3 of the step for lane l.
template <int VF, int IX>
struct Chunk {
  Codes<VF> codes;
  ColQuad<IX> ca, cb;
};

// The vector type: FP32, or FP64 for the FP64 product (one vector).
template <class T, int NRHS>
struct XVec {
  T v[NRHS];
};

template <class T, int NRHS>
__device__ __forceinline__ XVec<T, NRHS> load_x_global(const T* x, int c) {
  static_assert(NRHS == 1 || sizeof(T) == 4, "several vectors are FP32");
  XVec<T, NRHS> r;
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

// x of window column c: xb is the window moved back by cmin columns (below
// the window when cmin > 0; every c read lies inside it).
template <class T, int NRHS>
__device__ __forceinline__ XVec<T, NRHS> load_x_window(const T* xb, int c) {
  static_assert(NRHS == 1 || sizeof(T) == 4, "several vectors are FP32");
  XVec<T, NRHS> r;
  // the column as an opaque value, so that the address is one shift-add
  asm("" : "+v"(c));
  const T* p = xb + c * NRHS;
  if constexpr (NRHS == 1) {
    r.v[0] = p[0];
  } else if constexpr (NRHS == 2) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    r.v[0] = v.x;
    r.v[1] = v.y;
  } else {
    const float4 v = *reinterpret_cast<const float4*>(p);
    r.v[0] = v.x;
    r.v[1] = v.y;
    r.v[2] = v.z;
    r.v[3] = v.w;
  }
  return r;
}

// Sum of the 64 lanes in a fixed order, left in lane 63, with DPP: within
// each row of 16 lanes, shifts by 1, 2, 4 and 8 leave the row's sum in its
// lane 15 (lanes shifted in from outside a row contribute 0); a row broadcast
// then adds row 0's sum into row 1 and row 2's into row 3, and a second one
// adds lane 31 into row 3.  The broadcasts are written as DPP adds whose
// disabled rows keep their value (the builtin form would cost a move and a
// separate add each); s_nop 1 gives the two wait states a DPP read of a VGPR
// needs after a VALU write to it.  All 64 lanes must be active.
__device__ __forceinline__ float wave_reduce(float v) {
  constexpr int kRowShr = 0x110;
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kRowShr + 1, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kRowShr + 2, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kRowShr + 4, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kRowShr + 8, 0xf, 0xf, false));
  asm volatile(
      "s_nop 1\n\t"
      "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
      "s_nop 1"
      : "+v"(v));
  return v;
}

// The same tree for FP64 values, each DPP move taking the two halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0u, static_cast<unsigned>(u), CTRL, ROW_MASK, 0xf, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0u, static_cast<unsigned>(u >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((static_cast<unsigned long long>(hi) << 32) | lo);
}
__device__ __forceinline__ double wave_reduce(double v) {
  constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  v += dpp_f64<kRowShr + 1, 0xf>(v);
  v += dpp_f64<kRowShr + 2, 0xf>(v);
  v += dpp_f64<kRowShr + 4, 0xf>(v);
  v += dpp_f64<kRowShr + 8, 0xf>(v);
  v += dpp_f64<kRowBcast15, 0xa>(v);
  v += dpp_f64<kRowBcast31, 0xc>(v);
  return v;
}

// Positions.  A group's entries are addressed by their position P relative
// to the group's origin, its first entry rounded down to a multiple of 512:
// step k of the group covers positions [512 k, 512 k + 512), and lane l's
// quarters in it start at 512 k + 4 l and 512 k + 256 + 4 l, so steps and
// quarters sit on absolute multiples of 512 and 4 entries, whatever the
// partition.  A group spans fewer than 2^28 + 2^21 positions (rows are
// shorter than 2^28 entries), so byte offsets of positions fit 32 bits.

// The current 64-row window of the wave's rows (lane l: row wb + l's
// positions [lo, hi)) and its non-empty rows not yet started.
struct RowCursor {
  uint32_t wb;
  uint64_t mask;
  int lo, hi;
};

// Row offsets of the 64-row window at wb.  Issued for every lane (rows at or
// past r_end re-read row r_end - 1), so their number is fixed; r_end >= 1.
__device__ __forceinline__ void fetch_rows(const SpmvArgs& a, RowCursor& rc, uint32_t wb, uint32_t r_end,
                                           uint32_t origin32) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t r = min(wb + lane, r_end - 1);
  rc.wb = wb;
  rc.lo = static_cast<int>(a.row_ptr[r] - origin32);
  rc.hi = static_cast<int>(a.row_ptr[r + 1] - origin32);
}

// Lists the fetched window's non-empty rows and writes +0 to its empty ones
// (ACC: adds +0 to them).  ACC is a template parameter, not a run-time flag:
// as a flag, the compiler loaded y unconditionally and waited for all loads
// in flight at every window, stream prefetch included.
template <class T, int NRHS, bool ACC>
__device__ __forceinline__ void settle_rows(const SpmvArgs& a, RowCursor& rc, uint32_t r_end) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t r = rc.wb + lane;
  const bool in = r < r_end;
  if (in && rc.hi == rc.lo) {
    T* dst = static_cast<T*>(a.y) + static_cast<int64_t>(r) * NRHS;
    // accumulating products add +0 (so that a -0 already there becomes +0,
    // as in a sum of doses)
#pragma unroll
    for (int q = 0; q < NRHS; ++q) dst[q] = ACC ? dst[q] + T(0) : T(0);
  }
  rc.mask = __ballot(in && rc.hi > rc.lo);
}

// The row being summed (wave-uniform): its positions [ks, ke), its steps
// kfirst .. klast, and whether it is long (more than kRowSlots steps).  A
// row that is not valid has ks = kNoRow, so that no step takes it.
constexpr int kNoRow = 0x7fffffff;
struct Row {
  uint32_t row;
  int ks, ke;
  int kfirst, klast;
  int lng;  // 0 or 1 (an int, so that testing it is one scalar compare)
  bool valid;
};

// The wave's next non-empty row, moving on to later 64-row windows (and
// writing +0 to the empty rows passed) when the current one is done.
template <class T, int NRHS, bool ACC>
__device__ __forceinline__ Row next_row(const SpmvArgs& a, RowCursor& rc, uint32_t r_end, uint32_t origin32) {
  Row n;
  while (rc.mask == 0) {
    const uint32_t wb = rc.wb + kWave;
    if (wb >= r_end) {
      n.valid = false;
      n.ks = kNoRow;
      return n;
    }
    fetch_rows(a, rc, wb, r_end, origin32);
    settle_rows<T, NRHS, ACC>(a, rc, r_end);
  }
  const int i = __builtin_ctzll(rc.mask);
  rc.mask &= rc.mask - 1;
  n.row = rc.wb + static_cast<uint32_t>(i);
  n.ks = __builtin_amdgcn_readlane(rc.lo, i);
  n.ke = __builtin_amdgcn_readlane(rc.hi, i);
  n.kfirst = n.ks >> 9;
  n.klast = (n.ke - 1) >> 9;
  n.lng = n.klast - n.kfirst >= kRowSlots ? 1 : 0;
  n.valid = true;
  return n;
}

// One lane's entries of step k: two quarters.  Always issued (a fixed number
// of loads per step keeps the compiler's wait counts exact); quarters outside
// the wave's entries re-read the nearest quarter inside them, so the wave
// requests only its own lines and every column it reads lies in the group's
// window.  vb, cb: the code and index streams at the group's origin.
template <int VF, int IX>
__device__ __forceinline__ void load_step(const char* vb, const char* cb, int k, int pmin, int pmax,
                                          Chunk<VF, IX>& ch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int pos = k * kStepEntries + lane * kQuarter;
  const uint32_t e1 = static_cast<uint32_t>(min(max(pos, pmin), pmax));
  const uint32_t e2 = static_cast<uint32_t>(min(max(pos + kHalf, pmin), pmax));
  ch.codes.load(vb, e1, e2);
  ch.ca.load(cb, e1);
  ch.cb.load(cb, e2);
}

template <class T, int NRHS>
struct Gathered {
  XVec<T, NRHS> x[kChunk];
  float sc[kChunk];  // column scales (kScaleCol)
};

template <int IX>
__device__ __forceinline__ void chunk_cols(const ColQuad<IX>& ca, const ColQuad<IX>& cb, int (&cols)[kChunk]) {
  int c1[4], c2[4];
  ca.get(c1);
  cb.get(c2);
#pragma unroll
  for (int e = 0; e < 4; ++e) cols[e] = c1[e], cols[4 + e] = c2[e];
}

// Global-memory gathers of a step (x without a window, column scales of an
// E4M3 A^T), issued before the next step's loads, so that waiting for them
// leaves those loads in flight.  Column c of the step is column cbase + c of
// x and of the scales.
template <class T, int VF, int SM, int IX, int NRHS, bool WIN>
__device__ __forceinline__ void gather_global(const SpmvArgs& a, uint32_t cbase, const Chunk<VF, IX>& ch,
                                              Gathered<T, NRHS>& g) {
  int cols[kChunk];
  chunk_cols(ch.ca, ch.cb, cols);
  const T* x = static_cast<const T*>(a.x) + static_cast<int64_t>(cbase) * NRHS;
  if constexpr (!WIN) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e0 = h * kQuarter;
      if (NRHS == 1 && sizeof(T) == 4 && cols[e0 + 3] - cols[e0] == kQuarter - 1) {
        // 4 consecutive columns (inside one row): one 16-byte load of x
        const float4 v = *reinterpret_cast<const float4*>(x + cols[e0]);
        g.x[e0].v[0] = v.x, g.x[e0 + 1].v[0] = v.y, g.x[e0 + 2].v[0] = v.z, g.x[e0 + 3].v[0] = v.w;
      } else {
#pragma unroll
        for (int e = e0; e < e0 + kQuarter; ++e) g.x[e] = load_x_global<T, NRHS>(x, cols[e]);
      }
    }
  }
  if constexpr (SM == kScaleCol) {
#pragma unroll
    for (int e = 0; e < kChunk; ++e) g.sc[e] = a.scale[cbase + cols[e]];
  }
}

// The 8 products of the lane's step.  Every entry is decoded and multiplied,
// also those outside the wave's rows (their columns lie in the window; see
// load_step); rows select their own entries afterwards, so no Inf or NaN of x
// leaks into another row.  xb: the window base of load_x_window.
template <class T, int VF, int SM, int IX, int NRHS, bool WIN>
__device__ __forceinline__ void products(const Chunk<VF, IX>& ch, Gathered<T, NRHS>& g, const T* xb,
                                         T (&p)[kChunk][NRHS]) {
  if constexpr (WIN) {
    int cols[kChunk];
    chunk_cols(ch.ca, ch.cb, cols);
#pragma unroll
    for (int e = 0; e < kChunk; ++e) g.x[e] = load_x_window<T, NRHS>(xb, cols[e]);
  }
  if constexpr (VF == kFp16 && sizeof(T) == 4) {
    // an FMA with +0 rounds the product once, as a multiply does
#pragma unroll
    for (int e = 0; e < kChunk; ++e)
#pragma unroll
      for (int q = 0; q < NRHS; ++q) p[e][q] = __builtin_fmaf(ch.codes.get(e), g.x[e].v[q], 0.0f);
  } else {
    float d[kChunk];
    if constexpr (VF == kFp8) {
      ch.codes.decode(d);
    } else {
#pragma unroll
      for (int e = 0; e < kChunk; ++e) d[e] = ch.codes.get(e);
    }
#pragma unroll
    for (int e = 0; e < kChunk; ++e) {
      const float de = SM == kScaleCol ? d[e] * g.sc[e] : d[e];
#pragma unroll
      for (int q = 0; q < NRHS; ++q) p[e][q] = static_cast<T>(de) * g.x[e].v[q];
    }
  }
}

// Pairwise sum of quarter H of the lane's products, (a + b) + (c + d), over
// the entries at positions [ks, ks + len); d0 = the quarter's first position
// minus ks.  An entry is in when its position minus ks, taken unsigned, is
// below len; the others count as +0.
template <class T, int H, int NRHS>
__device__ __forceinline__ void quarter_sum(const T (&p)[kChunk][NRHS], int d0, uint32_t len, T (&s)[NRHS]) {
  T m[kQuarter][NRHS];
#pragma unroll
  for (int e = 0; e < kQuarter; ++e) {
    const bool in = static_cast<uint32_t>(d0 + e) < len;
#pragma unroll
    for (int q = 0; q < NRHS; ++q) m[e][q] = in ? p[H * kQuarter + e][q] : T(0);
  }
#pragma unroll
  for (int q = 0; q < NRHS; ++q) s[q] = (m[0][q] + m[1][q]) + (m[2][q] + m[3][q]);
}

// The same for a quarter wholly inside the row.
template <class T, int H, int NRHS>
__device__ __forceinline__ void quarter_full(const T (&p)[kChunk][NRHS], T (&s)[NRHS]) {
  constexpr int b = H * kQuarter;
#pragma unroll
  for (int q = 0; q < NRHS; ++q) s[q] = (p[b][q] + p[b + 1][q]) + (p[b + 2][q] + p[b + 3][q]);
}

// A short row's entries in half H of a step it meets (positions [256 H,
// 256 H + 256) of the step), added to the lane accumulator L.  a, b: the
// row's positions [ks, ke) relative to the step's start (a < 512, b > 0);
// lane4: the lane's first quarter position in the step.  Each test is one
// scalar compare (two-sided ones folded with max), not a pair of compares
// joined into a lane mask.
template <class T, int H, int NRHS>
__device__ __forceinline__ void add_half(const T (&p)[kChunk][NRHS], int lane4, int a, int b, T (&L)[NRHS]) {
  if (H == 0 ? a >= kHalf : b <= kHalf) return;  // the row misses this half
  T s[NRHS];
  if (max(a - H * kHalf, (H + 1) * kHalf - b) <= 0)  // the half lies inside the row
    quarter_full<T, H, NRHS>(p, s);
  else
    quarter_sum<T, H, NRHS>(p, lane4 + H * kHalf - a, static_cast<uint32_t>(b - a), s);
#pragma unroll
  for (int q = 0; q < NRHS; ++q) L[q] += s[q];
}

// Row value (valid in lane 63) times the row scale of an E4M3 operand, stored
// or (ACC: products of several matrices into one y, one launch after
// another) added to what y holds.
template <class T, int SM, int NRHS, bool ACC>
__device__ __forceinline__ void store_row(const SpmvArgs& a, uint32_t row, float sc, const T (&tot)[NRHS]) {
  T* dst = static_cast<T*>(a.y) + static_cast<int64_t>(row) * NRHS;
#pragma unroll
  for (int q = 0; q < NRHS; ++q) {
    const T v = SM == kScaleRow ? tot[q] * static_cast<T>(sc) : tot[q];
    dst[q] = ACC ? dst[q] + v : v;
  }
}

// One wave's share of a group: rows [r_begin, r_end), or with SPLIT the one
// row r_begin whose steps first, first + 4, ... this wave takes.  The wave
// streams its entries step by step with the next DEPTH steps' loads in
// flight (a ring of DEPTH + 1 chunk buffers, unrolled so that no loaded
// register is copied, left at one place only so that the compiler's view of
// the loads in flight stays exact).  In each step the rows that meet it take
// their entries in the order described at the top of this file.  With WIN
// the workgroup first copies the x window [cmin, cmin + clen) into LDS (x's
// layout, so a column c is at xw + (c - cmin) * NRHS); every wave issues its
// first loads before the copy's barrier, which all waves reach.  `safe` is
// any readable 16-byte aligned address (the group's descriptor).  Without
// SPLIT each finished row is stored; with SPLIT the wave's slot sum is left in
// `tot` and the row scale in `sc`.
// Steps whose loads are in flight ahead of the one computed, besides the
// refill (deeper rings were measured no faster for every value and index
// format on the clinical beam: the loads they issue past a wave's last step
// cost more than the added depth gains).
constexpr int kDepth = 1;
// 16-byte pieces of the x window each thread loads at once (a one-vector
// window of 4096 floats in one batch).
constexpr int kCopy = 4;

template <class T, int VF, int SM, int IX, int NRHS, bool WIN, bool SPLIT, bool ACC>
__device__ __forceinline__ void wave_stream(const SpmvArgs& a, uint64_t base, uint32_t r_begin, uint32_t r_end,
                                            uint32_t e_begin, uint32_t e_end, int first, float* xw, int cmin, int clen,
                                            uint32_t cbase, const void* safe, T (&tot)[NRHS], float& sc) {
  constexpr int stride = SPLIT ? kRowSlots : 1;
  constexpr int DEPTH = kDepth;
  const uint64_t origin = base & ~static_cast<uint64_t>(kStepEntries - 1);
  const uint32_t origin32 = static_cast<uint32_t>(origin);
  const char* vb = static_cast<const char*>(a.val) + origin * Codes<VF>::kBytes;
  const char* cb = static_cast<const char*>(a.col) + origin * IX;
#pragma unroll
  for (int q = 0; q < NRHS; ++q) tot[q] = T(0);
  sc = 1.0f;
  // the wave's positions [p0, p1) (from the group descriptor, so the first
  // loads go out at once) and its steps
  const int shift = static_cast<int>(base - origin);
  const int p0 = shift + static_cast<int>(e_begin), p1 = shift + static_cast<int>(e_end);
  const int pmin = p0 & ~(kQuarter - 1), pmax = max(p1 - 1, p0) & ~(kQuarter - 1);
  const int kbeg = (p0 >> 9) + (SPLIT ? first : 0);
  const int kend = p1 > p0 ? (p1 - 1) >> 9 : -1;  // the wave's last step (inclusive)
  // The group's first loads, in the order they are needed: the x window
  // (16-byte pieces of x, a thread's first kCopy of them at once), the wave's
  // first 64 row offsets, then the stream's first steps; waiting for the first
  // two leaves the stream in flight.  Without this order each wait would also
  // wait for the stream, and a copy loop would wait once per piece.
  // window words of 4 bytes (the window is x's own layout), whole 16-byte
  // pieces (x + cmin * NRHS is 32-byte aligned within x)
  const int nf = clen * NRHS * static_cast<int>(sizeof(T) / 4);
  const int n4 = nf >> 2;
  const float* xs =
      reinterpret_cast<const float*>(static_cast<const T*>(a.x) + (static_cast<int64_t>(cmin) + cbase) * NRHS);
  // every load is issued (a lane without a piece reads the group descriptor
  // instead), so that the compiler's count of loads in flight stays exact
  const int tid = static_cast<int>(threadIdx.x);
  const float4* xs4 = reinterpret_cast<const float4*>(xs);
  const float4* safe4 = static_cast<const float4*>(safe);
  float4 w0, w1, w2, w3;  // pieces tid, tid + 256, tid + 512, tid + 768
  float wt = 0.0f;
  if constexpr (WIN) {
    w0 = *(tid < n4 ? xs4 + tid : safe4);
    w1 = *(tid + kGroupThreads < n4 ? xs4 + tid + kGroupThreads : safe4);
    w2 = *(tid + 2 * kGroupThreads < n4 ? xs4 + tid + 2 * kGroupThreads : safe4);
    w3 = *(tid + 3 * kGroupThreads < n4 ? xs4 + tid + 3 * kGroupThreads : safe4);
    const int t = 4 * n4 + tid;  // the last nf mod 4 floats
    wt = *(t < nf ? xs + t : static_cast<const float*>(safe));
  }
  RowCursor rc;
  rc.mask = 0;
  Row cr;
  cr.valid = false;
  cr.ks = kNoRow;
  const bool has_rows = r_begin < r_end;
  // issued by every wave (one without rows re-reads a row before r_begin, or
  // row 0), so that no branch hides it from the compiler's load count
  fetch_rows(a, rc, r_begin, has_rows ? r_end : max(r_begin, 1u), origin32);
  // With an LDS window and no global gathers, a step's buffer is refilled
  // (DEPTH + 1 steps ahead) as soon as its products are formed, before the
  // step's rows are summed: the row work then delays no load.  Global
  // gathers must be issued before the next step's loads (so that waiting for
  // them leaves those loads in flight), so there the buffer of the previous
  // step is refilled first.
  constexpr bool kEarly = WIN && SM != kScaleCol;
  Chunk<VF, IX> cs[DEPTH + 1];
  Gathered<T, NRHS> g;
#pragma unroll
  for (int d = 0; d < (kEarly ? DEPTH + 1 : DEPTH); ++d) load_step<VF, IX>(vb, cb, kbeg + d * stride, pmin, pmax, cs[d]);
  if (has_rows) {
    // the wave's first non-empty row; next_row moves on from rc.wb + 64 once
    // the first row window is done
    settle_rows<T, NRHS, ACC>(a, rc, r_end);
    cr = next_row<T, NRHS, ACC>(a, rc, r_end, origin32);
  }
  if constexpr (WIN) {
    float4* xw4 = reinterpret_cast<float4*>(xw);
    if (tid < n4) xw4[tid] = w0;
    if (tid + kGroupThreads < n4) xw4[tid + kGroupThreads] = w1;
    if (tid + 2 * kGroupThreads < n4) xw4[tid + 2 * kGroupThreads] = w2;
    if (tid + 3 * kGroupThreads < n4) xw4[tid + 3 * kGroupThreads] = w3;
    if (4 * n4 + tid < nf) xw[4 * n4 + tid] = wt;
    // windows larger than one batch (several vectors)
    for (int j = tid + kCopy * kGroupThreads; j < n4; j += kGroupThreads) xw4[j] = xs4[j];
    __syncthreads();
  }
  if (!cr.valid || kbeg > kend) return;
  const T* xb = reinterpret_cast<const T*>(xw) - cmin * NRHS;
  const int lane = threadIdx.x & (kWave - 1);
  // long rows: slot sums (valid in lane 63); short rows: lane sums
  T W[kRowSlots][NRHS], L[NRHS];
#pragma unroll
  for (int q = 0; q < NRHS; ++q) {
    L[q] = T(-0.0);
#pragma unroll
    for (int s = 0; s < kRowSlots; ++s) W[s][q] = T(0);
  }
  int k = kbeg;
  // the rows that meet step k take their entries of the step's products p
  // (none once the wave is past its last step)
  auto rows_of_step = [&](const T (&p)[kChunk][NRHS]) {
    const int s0 = k * kStepEntries;
    const int lane4 = lane * kQuarter;
    // rows starting below lim meet the step (no row once the wave is past
    // its last step; an invalid row starts at kNoRow)
    const int lim = k <= kend ? s0 + kStepEntries : -kNoRow;
    while (cr.ks < lim) {
      const bool lng = SPLIT || cr.lng != 0;
      const int ra = cr.ks - s0, rb = cr.ke - s0;  // the row relative to the step
      if (lng) {
        T h0[NRHS], h1[NRHS];
        if (max(ra, kStepEntries - rb) <= 0) {
          quarter_full<T, 0, NRHS>(p, h0);
          quarter_full<T, 1, NRHS>(p, h1);
        } else {
          const uint32_t len = static_cast<uint32_t>(rb - ra);
          quarter_sum<T, 0, NRHS>(p, lane4 - ra, len, h0);
          quarter_sum<T, 1, NRHS>(p, lane4 + kHalf - ra, len, h1);
        }
        const int slot = (k - cr.kfirst) & (kRowSlots - 1);
#pragma unroll
        for (int q = 0; q < NRHS; ++q) {
          const T t = wave_reduce(h0[q] + h1[q]);
#pragma unroll
          for (int s = 0; s < kRowSlots; ++s) W[s][q] += s == slot ? t : T(0);
        }
      } else {
        add_half<T, 0, NRHS>(p, lane4, ra, rb, L);
        add_half<T, 1, NRHS>(p, lane4, ra, rb, L);
      }
      if (k + stride <= cr.klast) break;  // the row goes on in a later step of this wave
      // the wave's last step of the row; slots that received nothing hold
      // +0, and no slot sum is ever -0, so adding them changes nothing
      if (lng) {
#pragma unroll
        for (int q = 0; q < NRHS; ++q) tot[q] = (W[0][q] + W[1][q]) + (W[2][q] + W[3][q]);
      } else {
#pragma unroll
        for (int q = 0; q < NRHS; ++q) tot[q] = wave_reduce(L[q]);
      }
      if constexpr (SM == kScaleRow) sc = a.scale[cr.row];
      if constexpr (SPLIT) {
        cr.valid = false;
        cr.ks = kNoRow;
      } else {
        if (lane == kWave - 1) store_row<T, SM, NRHS, ACC>(a, cr.row, sc, tot);
#pragma unroll
        for (int q = 0; q < NRHS; ++q) {
          L[q] = T(-0.0);
#pragma unroll
          for (int s = 0; s < kRowSlots; ++s) W[s][q] = T(0);
        }
        cr = next_row<T, NRHS, ACC>(a, rc, r_end, origin32);
      }
    }
  };
  if constexpr (kEarly) {
    while (true) {
#pragma unroll
      for (int ph = 0; ph <= DEPTH; ++ph) {
        T p[kChunk][NRHS];
        products<T, VF, SM, IX, NRHS, WIN>(cs[ph], g, xb, p);
        // the barriers keep the scheduler from moving the loads across the
        // products or sinking them below the row work
        __builtin_amdgcn_sched_barrier(0);
        load_step<VF, IX>(vb, cb, k + (DEPTH + 1) * stride, pmin, pmax, cs[ph]);
        __builtin_amdgcn_sched_barrier(0);
        rows_of_step(p);
        k += stride;
      }
      // one exit per turn of the ring: steps past the wave's last one do nothing
      if (k > kend) break;
    }
  } else {
    // the gathers of a step must go out before the next step's loads (so
    // that waiting for them leaves those loads in flight): the buffer of the
    // previous step is refilled first
    while (true) {
#pragma unroll
      for (int ph = 0; ph <= DEPTH; ++ph) {
        const int cur = ph, nxt = (ph + DEPTH) % (DEPTH + 1);
        T p[kChunk][NRHS];
        gather_global<T, VF, SM, IX, NRHS, WIN>(a, cbase, cs[cur], g);
        load_step<VF, IX>(vb, cb, k + DEPTH * stride, pmin, pmax, cs[nxt]);
        // keep the scheduler from sinking the loads below the compute
        __builtin_amdgcn_sched_barrier(0);
        products<T, VF, SM, IX, NRHS, WIN>(cs[cur], g, xb, p);
        rows_of_step(p);
        k += stride;
      }
      // one exit per turn of the ring: steps past the wave's last one do nothing
      if (k > kend) break;
    }
  }
}

// One group on one workgroup.  `part` is LDS for the four slot sums of a
// split row.
template <class T, int VF, int SM, int NRHS, int IX, bool ACC>
__device__ __forceinline__ void run_group(const SpmvArgs& a, const GroupDesc* gp, float* xw, T* part) {
  // wave-uniform index, so that the row bounds below are scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const uint64_t base = gp->nnz_base;
  const uint32_t clen = gp->clen;
  const bool win = clen > 0 && window_floats(clen, NRHS * static_cast<int>(sizeof(T) / 4)) <= a.win_floats;
  const int cmin = win ? static_cast<int>(gp->cmin) : 0;
  // the group's column indices count from cbase (x and an E4M3 column
  // scale are read from there)
  const uint32_t cbase = gp->cbase;
  T tot[NRHS];
  float sc;
  if (gp->split == 0) {
    const uint32_t r0 = gp->row[wave], r1 = gp->row[wave + 1];
    const uint32_t e0 = wave == 0 ? 0u : gp->ent[wave - 1], e1 = gp->ent[wave];
    if (win)
      wave_stream<T, VF, SM, IX, NRHS, true, false, ACC>(a, base, r0, r1, e0, e1, 0, xw, cmin, static_cast<int>(clen),
                                                    cbase, gp, tot, sc);
    else
      wave_stream<T, VF, SM, IX, NRHS, false, false, ACC>(a, base, r0, r1, e0, e1, 0, xw, 0, 0, cbase, gp, tot, sc);
    return;
  }
  const uint32_t row = gp->row[0], len = gp->ent[kGroupWaves - 1];
  if (win)
    wave_stream<T, VF, SM, IX, NRHS, true, true, ACC>(a, base, row, row + 1, 0, len, wave, xw, cmin, static_cast<int>(clen),
                                                 cbase, gp, tot, sc);
  else
    wave_stream<T, VF, SM, IX, NRHS, false, true, ACC>(a, base, row, row + 1, 0, len, wave, xw, 0, 0, cbase, gp, tot, sc);
  if ((threadIdx.x & (kWave - 1)) == kWave - 1)
#pragma unroll
    for (int q = 0; q < NRHS; ++q) part[wave * NRHS + q] = tot[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    T r[NRHS];
#pragma unroll
    for (int q = 0; q < NRHS; ++q)
      r[q] = (part[0 * NRHS + q] + part[1 * NRHS + q]) + (part[2 * NRHS + q] + part[3 * NRHS + q]);
    store_row<T, SM, NRHS, ACC>(a, row, SM == kScaleRow ? a.scale[row] : 1.0f, r);
  }
}

// The group workgroup b takes.  With a.xcd_blocks = D (the dies workgroups
// are dealt to in turn, b going to die b mod D), die x takes the groups
// [x q + min(x, r), ...) of a split of the n groups into D contiguous runs
// (q = n / D, r = n mod D, the first r runs one longer), in order: a
// bijection of [0, n), so every group is taken once.
__device__ __forceinline__ int64_t group_of_block(const SpmvArgs& a, uint32_t b) {
  const int D = a.xcd_blocks;
  if (D <= 1) return b;
  const int64_t q = a.n_groups / D, r = a.n_groups % D;
  const int64_t x = b % static_cast<uint32_t>(D), i = b / static_cast<uint32_t>(D);
  return x * q + (x < r ? x : r) + i;
}

template <int VF, int SM, int NRHS, int IX>
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_spmv(SpmvArgs a) {
  extern __shared__ __align__(16) float xw[];  // a.win_floats floats
  __shared__ float part[kGroupWaves * NRHS];
  run_group<float, VF, SM, NRHS, IX, false>(a, a.groups + group_of_block(a, blockIdx.x), xw, part);
}

// FP64 x and y, FP64 products and sums (one vector): the paper's
// half/double configuration (Sec. II-D).
template <int VF, int SM, int IX>
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_spmv_f64(SpmvArgs a) {
  extern __shared__ __align__(16) float xw[];  // a.win_floats 4-byte words
  __shared__ double part[kGroupWaves];
  run_group<double, VF, SM, 1, IX, false>(a, a.groups + group_of_block(a, blockIdx.x), xw, part);
}

// The item a workgroup of a batched launch belongs to without a work list:
// the last item whose first workgroup is at or before b (items without groups
// share their first workgroup with the next item and are never chosen).  The
// lanes compare 64 entries of the ascending table at a time.
__device__ __forceinline__ int find_item(const uint32_t* __restrict__ first, int n_items, uint32_t b) {
  const int lane = threadIdx.x & (kWave - 1);
  int below = 0;  // entries i < n_items with first[i] <= b
  for (int i0 = 0; i0 < n_items; i0 += kWave) {
    const int i = i0 + lane;
    const bool le = i < n_items && first[i] <= b;
    const int c = __popcll(__ballot(le));
    below += c;
    if (c < kWave) break;
  }
  return below - 1;
}

// Batched form, one launch for many matrices: workgroup b takes entry b of
// the work list (a copy of a group's descriptor that names its item), or,
// without a work list, group b - first[i] of item i's matrix.  ACC: every
// row value is added to what y holds (one vector only).
template <int VF, int SM, int NRHS, int IX, bool ACC>
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_spmv_batched(BatchTable t) {
  extern __shared__ __align__(16) float xw[];  // the largest win_floats of the items
  __shared__ float part[kGroupWaves * NRHS];
  if (t.work) {
    const GroupDesc* gp = t.work + blockIdx.x;
    run_group<float, VF, SM, NRHS, IX, ACC>(t.args[gp->item], gp, xw, part);
  } else {
    const int i = __builtin_amdgcn_readfirstlane(find_item(t.first, t.n_items, blockIdx.x));
    const SpmvArgs& a = t.args[i];
    run_group<float, VF, SM, NRHS, IX, ACC>(a, a.groups + (blockIdx.x - t.first[i]), xw, part);
  }
}

template <int VF, int SM, int NRHS>
// (FP32 vectors with column scales, the spot-row A^T's, are built for int32
// indices only; launch_spmv refuses other widths.)
void launch_ix(const SpmvArgs& a, size_t lds, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_groups)), block(kGroupThreads);
  if (SM != kScaleCol && a.idx_bytes == 2)
    hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, SM == kScaleCol ? 4 : 2>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((k_spmv<VF, SM, NRHS, 4>), grid, block, lds, s, a);
}

template <int VF, int SM, int NRHS, bool ACC>
void launch_ix_batched(int idx_bytes, const BatchTable& t, int64_t n_work, size_t lds, hipStream_t s) {
  const dim3 g(static_cast<unsigned>(n_work)), block(kGroupThreads);
  if (SM != kScaleCol && idx_bytes == 2)
    hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, SM == kScaleCol ? 4 : 2, ACC>), g, block, lds, s, t);
  else
    hipLaunchKernelGGL((k_spmv_batched<VF, SM, NRHS, 4, ACC>), g, block, lds, s, t);
}

template <int VF, int SM>
hipError_t launch_rhs(int n_rhs, const SpmvArgs& a, hipStream_t s) {
  const size_t lds = static_cast<size_t>(a.win_floats) * sizeof(float);
  switch (n_rhs) {
    case 1: launch_ix<VF, SM, 1>(a, lds, s); break;
    case 2: launch_ix<VF, SM, 2>(a, lds, s); break;
    case 4: launch_ix<VF, SM, 4>(a, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int VF, int SM>
hipError_t launch_rhs_batched(int n_rhs, int accumulate, int idx_bytes, const BatchTable& t, int64_t n_work,
                              int lds_floats, hipStream_t s) {
  const size_t lds = static_cast<size_t>(lds_floats) * sizeof(float);
  if (accumulate && n_rhs != 1) return hipErrorInvalidValue;
  switch (n_rhs) {
    case 1:
      if (accumulate)
        launch_ix_batched<VF, SM, 1, true>(idx_bytes, t, n_work, lds, s);
      else
        launch_ix_batched<VF, SM, 1, false>(idx_bytes, t, n_work, lds, s);
      break;
    case 2: launch_ix_batched<VF, SM, 2, false>(idx_bytes, t, n_work, lds, s); break;
    case 4: launch_ix_batched<VF, SM, 4, false>(idx_bytes, t, n_work, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Column window of every group: the smallest and largest column over the
// entries its waves load -- its own entries widened to whole 4-entry quarters
// at both ends (the neighbours' entries there, or padding, which repeats the
// last column) -- with the first column rounded down to a multiple of 8.
template <class I>
__global__ __launch_bounds__(256) void k_group_windows(GroupDesc* __restrict__ groups, int64_t n_groups,
                                                       const I* __restrict__ col,
                                                       const uint32_t* __restrict__ row_ptr) {
  __shared__ int smin[256], smax[256];
  const GroupDesc g = groups[blockIdx.x];
  const uint32_t base32 = static_cast<uint32_t>(g.nnz_base);
  const uint64_t n = static_cast<uint64_t>(row_ptr[g.row[kGroupWaves]] - base32);
  const uint64_t first = g.nnz_base & ~uint64_t{kQuarterEntries - 1};
  const uint64_t span = n == 0 ? 0 : ((g.nnz_base + n - 1) | uint64_t{kQuarterEntries - 1}) + 1 - first;
  int mn = 0x7fffffff, mx = -1;
  for (uint64_t k = threadIdx.x; k < span; k += 256) {
    const int c = static_cast<int>(col[first + k]);
    mn = min(mn, c);
    mx = max(mx, c);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int c0 = smin[0] & ~(kWinAlign - 1);
    groups[blockIdx.x].cmin = smax[0] >= 0 ? static_cast<uint32_t>(c0) : 0u;
    groups[blockIdx.x].clen = smax[0] >= 0 ? static_cast<uint32_t>(smax[0] - c0 + 1) : 0u;
  }
  (void)n_groups;
}

}  // namespace

hipError_t launch_spmv(int vf, int scale_mode, int n_rhs, const SpmvArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if (a.idx_bytes != 4 && a.idx_bytes != 2) return hipErrorInvalidValue;
  if (scale_mode == kScaleCol && a.idx_bytes != 4) return hipErrorInvalidValue;
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_rhs<kFp16, kScaleNone>(n_rhs, a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_rhs<kBf16, kScaleNone>(n_rhs, a, s);
  if (vf == kFp32 && scale_mode == kScaleNone) return launch_rhs<kFp32, kScaleNone>(n_rhs, a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_rhs<kFp8, kScaleRow>(n_rhs, a, s);
  if (vf == kFp8 && scale_mode == kScaleCol) return launch_rhs<kFp8, kScaleCol>(n_rhs, a, s);
  if (vf == kFp8 && scale_mode == kScaleNone && n_rhs == 1) {
    // E4M3 codes without their scale (the FP32 adjoint, whose seed carries the row scales)
    launch_ix<kFp8, kScaleNone, 1>(a, static_cast<size_t>(a.win_floats) * sizeof(float), s);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int VF, int SM>
hipError_t launch_f64(const SpmvArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_groups)), block(kGroupThreads);
  const size_t lds = static_cast<size_t>(a.win_floats) * sizeof(float);
  // every scale mode with either index width (column scales with 16-bit
  // indices: the E4M3 FP64 adjoint over A^T in voxel slabs)
  if (a.idx_bytes == 2)
    hipLaunchKernelGGL((k_spmv_f64<VF, SM, 2>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((k_spmv_f64<VF, SM, 4>), grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_spmv_f64(int vf, int scale_mode, const SpmvArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if (a.idx_bytes != 4 && a.idx_bytes != 2) return hipErrorInvalidValue;
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_f64<kFp16, kScaleNone>(a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_f64<kBf16, kScaleNone>(a, s);
  if (vf == kFp32 && scale_mode == kScaleNone) return launch_f64<kFp32, kScaleNone>(a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_f64<kFp8, kScaleRow>(a, s);
  if (vf == kFp8 && scale_mode == kScaleCol) return launch_f64<kFp8, kScaleCol>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spmv_batched(int vf, int scale_mode, int n_rhs, int accumulate, int idx_bytes, const BatchTable& t,
                               int64_t n_work, int lds_floats, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  if (idx_bytes != 4 && idx_bytes != 2) return hipErrorInvalidValue;
  if (scale_mode == kScaleCol && idx_bytes != 4) return hipErrorInvalidValue;
  if (vf == kFp16 && scale_mode == kScaleNone)
    return launch_rhs_batched<kFp16, kScaleNone>(n_rhs, accumulate, idx_bytes, t, n_work, lds_floats, s);
  if (vf == kBf16 && scale_mode == kScaleNone)
    return launch_rhs_batched<kBf16, kScaleNone>(n_rhs, accumulate, idx_bytes, t, n_work, lds_floats, s);
  if (vf == kFp32 && scale_mode == kScaleNone)
    return launch_rhs_batched<kFp32, kScaleNone>(n_rhs, accumulate, idx_bytes, t, n_work, lds_floats, s);
  if (vf == kFp8 && scale_mode == kScaleRow)
    return launch_rhs_batched<kFp8, kScaleRow>(n_rhs, accumulate, idx_bytes, t, n_work, lds_floats, s);
  if (vf == kFp8 && scale_mode == kScaleCol)
    return launch_rhs_batched<kFp8, kScaleCol>(n_rhs, accumulate, idx_bytes, t, n_work, lds_floats, s);
  if (vf == kFp8 && scale_mode == kScaleNone && n_rhs == 1 && !accumulate) {
    // E4M3 codes without their scale (adjoint plans, whose seeds carry the row scales)
    launch_ix_batched<kFp8, kScaleNone, 1, false>(idx_bytes, t, n_work, static_cast<size_t>(lds_floats) * sizeof(float),
                                                   s);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_group_windows(GroupDesc* groups, int64_t n_groups, const void* col, int idx_bytes,
                                const uint32_t* row_ptr, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  if (idx_bytes == 2)
    hipLaunchKernelGGL(k_group_windows<uint16_t>, dim3(static_cast<unsigned>(n_groups)), dim3(256), 0, s, groups,
                       n_groups, static_cast<const uint16_t*>(col), row_ptr);
  else
    hipLaunchKernelGGL(k_group_windows<int32_t>, dim3(static_cast<unsigned>(n_groups)), dim3(256), 0, s, groups,
                       n_groups, static_cast<const int32_t*>(col), row_ptr);
  return hipGetLastError();
}

}  // namespace dose
