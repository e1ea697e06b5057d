// SELL-C-sigma product kernel of libdose for gfx950 (CDNA4, wave64).
//
// SELL-C-sigma (Kreutzer et al., SIAM J. Sci. Comput. 36(5), 2014) is the
// SIMD-oriented sparse format the paper names as the next one to try for dose
// matrices (Sec. II-C, Sec. VII).  Rows are sorted by descending length
// inside windows of sigma rows and cut into chunks of C = 64 rows, one row per
// lane of a wave64, so no row needs a cross-lane reduction and the lanes of a
// wave stream their rows side by side.  Here a chunk stores its entries in
// slices of 8 per lane (sell_internal.h): a lane reads its row's next 8 codes
// with one 16-byte load (FP16), and a wave's load instruction covers 1 KB of
// consecutive codes (or indices).
//
//   * A workgroup (four waves) takes one chunk and copies the chunk's x
//     window into LDS once (the rows of a sigma window are neighbouring
//     voxels, so their spots lie in a narrow range); a chunk whose window
//     exceeds the LDS cap gathers x from global memory.
//   * The chunk's slices are dealt to the waves in turn (wave j takes slices
//     j, j + 4, ...); the next slices' loads are in flight while one is
//     computed.
//   * Run-length column indices: the chunk's runs are staged in LDS; a lane
//     keeps a cursor on its row's runs, and a slice whose 8 entries lie in
//     one run (the common case) reads 8 consecutive x from one LDS address.
//   * Several vectors (n_rhs = 2 or 4, x and y row-major [.][n_rhs]): every
//     entry is loaded once and multiplied by the n_rhs values of its column
//     (one LDS read); each vector's sums follow the order below, so the
//     product equals n_rhs single-vector products bit for bit.  A batched
//     launch takes the chunks of many matrices from one work list.
//   * One FP64 vector (the paper's half/double arithmetic, Sec. II-D): the
//     same kernel with FP64 x, products, sums and y, in the same order.
//   * Summation order, fixed by the stored layout (so equal inputs give equal
//     bits): a lane's 8 products of a slice add pairwise, ((p0 + p1) +
//     (p2 + p3)) + ((p4 + p5) + (p6 + p7)), slots past the row's end counting
//     as +0; each wave adds its slice sums of the row in order, eight at a
//     time into an inner sum that is then added to an outer one (the FP32
//     error of a row of L entries stays below (14 + L / 256) * 2^-24 of
//     sum |a x|); the four waves' sums of a row meet as (S0 + S1) + (S2 + S3).
//     The order depends only on the row's own entries.  Empty rows get +0.
#include "dose_internal.h"
#include "sell_internal.h"

#include <hip/hip_fp16.h>

// Products are rounded before they are summed (no multiply-add contraction).
#pragma clang fp contract(off)

namespace dose {
namespace {

constexpr int kWave = 64;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint4 ld_nt4(const char* base, uint32_t off) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + off));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_nt2(const char* base, uint32_t off) {
  const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(base + off));
  return make_uint2(v.x, v.y);
}

template <int VF>
constexpr int code_bytes() {
  return VF == kFp8 ? 1 : VF == kFp32 ? 4 : 2;
}

// One lane's 8 codes and 8 column indices of a slice.
template <int VF, int IX>
struct Lane8 {
  uint4 c0, c1;  // codes (c1: FP32 only)
  uint4 i0, i1;  // indices (i1: int32 only)
};

// Slices in flight per wave (one being computed, the others loading): about
// 128 bytes per lane, so that the narrower streams keep as many bytes in
// flight as the wide ones (a lane's slice is 8 codes plus 8 indices).  With
// four vectors two slices: each vector's products take registers, and a
// deeper ring was measured slower (the 36-matrix batch at a quarter scale,
// 16-bit indices: 1.74 against 1.67 ms).
template <int VF, int IX, int NRHS>
constexpr int ring_depth() {
  constexpr int bytes = kSellLaneEntries * (code_bytes<VF>() + IX);
  constexpr int d = 128 / bytes < 2 ? 2 : 128 / bytes > 4 ? 4 : 128 / bytes;
  return NRHS == 4 ? 2 : d;
}

// Loads lane `lane`'s part of slice `slice` (wave-uniform).
template <int VF, int IX>
__device__ __forceinline__ void load_slice(const char* val, const char* col, uint32_t slice, int lane,
                                           Lane8<VF, IX>& L) {
  const uint64_t e = static_cast<uint64_t>(slice) * kSellSliceEntries;
  const char* vb = val + e * code_bytes<VF>();
  const char* cb = IX ? col + e * IX : col;
  const uint32_t o = static_cast<uint32_t>(lane) * kSellLaneEntries;
  if constexpr (VF == kFp8) {
    const uint2 v = ld_nt2(vb, o);
    L.c0 = make_uint4(v.x, v.y, 0u, 0u);
  } else if constexpr (VF == kFp32) {
    L.c0 = ld_nt4(vb, sell_slot(4, lane, 0) * 4u);
    L.c1 = ld_nt4(vb, sell_slot(4, lane, 4) * 4u);
  } else {
    L.c0 = ld_nt4(vb, o * 2u);
  }
  if constexpr (IX == 4) {
    L.i0 = ld_nt4(cb, sell_slot(4, lane, 0) * 4u);
    L.i1 = ld_nt4(cb, sell_slot(4, lane, 4) * 4u);
  } else if constexpr (IX == 2) {
    L.i0 = ld_nt4(cb, o * 2u);
  }
}

template <int VF, int IX>
__device__ __forceinline__ void lane_cols(const Lane8<VF, IX>& L, int (&c)[kSellLaneEntries]) {
  if constexpr (IX == 4) {
    c[0] = static_cast<int>(L.i0.x), c[1] = static_cast<int>(L.i0.y);
    c[2] = static_cast<int>(L.i0.z), c[3] = static_cast<int>(L.i0.w);
    c[4] = static_cast<int>(L.i1.x), c[5] = static_cast<int>(L.i1.y);
    c[6] = static_cast<int>(L.i1.z), c[7] = static_cast<int>(L.i1.w);
  } else {
    const uint32_t w[4] = {L.i0.x, L.i0.y, L.i0.z, L.i0.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) c[2 * j] = static_cast<int>(w[j] & 0xFFFFu), c[2 * j + 1] = static_cast<int>(w[j] >> 16);
  }
#pragma unroll
  for (int e = 0; e < kSellLaneEntries; ++e) asm("" : "+v"(c[e]));  // keep each LDS address one shift-add
}

// The n_rhs values of x at p (row-major x aligned to n_rhs values; V is
// float, or double for one FP64 vector).
template <class V, int NRHS>
struct XV {
  V v[NRHS];
};
template <class V, int NRHS>
__device__ __forceinline__ XV<V, NRHS> x_at(const V* p) {
  static_assert(NRHS == 1 || sizeof(V) == 4, "several vectors are FP32");
  XV<V, NRHS> r;
  if constexpr (NRHS == 1) {
    r.v[0] = p[0];
  } else if constexpr (NRHS == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    r.v[0] = t.x, r.v[1] = t.y;
  } else {
    const float4 t = *reinterpret_cast<const float4*>(p);
    r.v[0] = t.x, r.v[1] = t.y, r.v[2] = t.z, r.v[3] = t.w;
  }
  return r;
}

// The lane's 8 decoded codes of a slice (E4M3 without its row scale).
template <int VF, int IX>
__device__ __forceinline__ void slice_codes(const Lane8<VF, IX>& L, float (&d)[kSellLaneEntries]) {
  if constexpr (VF == kFp16) {
    const uint32_t w[4] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e)
      d[e] = __half2float(__ushort_as_half(static_cast<unsigned short>((w[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu)));
  } else if constexpr (VF == kBf16) {
    const uint32_t w[4] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) {
      const uint32_t word = w[e >> 1];
      d[e] = __uint_as_float((e & 1) ? (word & 0xFFFF0000u) : (word << 16));
    }
  } else if constexpr (VF == kFp8) {
    const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.x), false);
    const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.x), true);
    const f32x2 cc = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.y), false);
    const f32x2 dd = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.y), true);
    d[0] = a.x, d[1] = a.y, d[2] = b.x, d[3] = b.y, d[4] = cc.x, d[5] = cc.y, d[6] = dd.x, d[7] = dd.y;
  } else {
    const uint32_t w[8] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w, L.c1.x, L.c1.y, L.c1.z, L.c1.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) d[e] = __uint_as_float(w[e]);
  }
}

// The lane's 8 products of a slice for each vector: decoded code times x of
// its column, rounded once (in FP64 for an FP64 vector: the decoded code is
// exact in both).  x comes from the LDS window (xb: the window moved back by
// cmin columns) or from global memory.
template <class V, int VF, int IX, bool WIN, int NRHS>
__device__ __forceinline__ void slice_products(const Lane8<VF, IX>& L, const int (&c)[kSellLaneEntries],
                                               const V* xb, const V* x, V (&p)[kSellLaneEntries][NRHS]) {
  XV<V, NRHS> xv[kSellLaneEntries];
#pragma unroll
  for (int e = 0; e < kSellLaneEntries; ++e) {
    if constexpr (WIN) {
      xv[e] = x_at<V, NRHS>(xb + c[e] * NRHS);
    } else {
      xv[e] = x_at<V, NRHS>(x + static_cast<int64_t>(c[e]) * NRHS);
    }
  }
  float d[kSellLaneEntries];
  slice_codes<VF, IX>(L, d);
#pragma unroll
  for (int e = 0; e < kSellLaneEntries; ++e)
#pragma unroll
    for (int q = 0; q < NRHS; ++q) {
      if constexpr (VF == kFp16 && sizeof(V) == 4) {
        // an FMA with +0 rounds the product once, as a multiply does (v_fma_mix)
        p[e][q] = __builtin_fmaf(d[e], xv[e].v[q], 0.0f);
      } else {
        p[e][q] = static_cast<V>(d[e]) * xv[e].v[q];
      }
    }
}

template <class V, int NRHS>
__device__ __forceinline__ V slice_sum(const V (&p)[kSellLaneEntries][NRHS], int q) {
  return ((p[0][q] + p[1][q]) + (p[2][q] + p[3][q])) + ((p[4][q] + p[5][q]) + (p[6][q] + p[7][q]));
}

// The work item of workgroup b of n (see group_of_block in the CSR kernels:
// with D dies dealt workgroups in turn, die x takes one contiguous run of
// the items).
__device__ __forceinline__ int64_t sell_group_of_block(int D, int64_t n, uint32_t b) {
  if (D <= 1) return b;
  const int64_t q = n / D, r = n % D;
  const int64_t x = b % static_cast<uint32_t>(D), i = b / static_cast<uint32_t>(D);
  return x * q + (x < r ? x : r) + i;
}

// Columns of a lane's 8 entries at positions P .. P + 7 of its row from the
// row's runs (rare path: some entry lies beyond the run after the current
// one): walk the runs from the current one; entries past the row take the
// padding column.
__device__ __forceinline__ void walk_runs(const SellRun* lruns, int ri, int re, int cur_end, int cur_delta, int P,
                                          int cmin, int (&cols)[kSellLaneEntries]) {
  int j = ri, ce = cur_end, cd = cur_delta;
  for (int e = 0; e < kSellLaneEntries; ++e) {
    const int p = P + e;
    while (p >= ce && j + 1 < re) {
      ++j;
      ce = lruns[j].end, cd = lruns[j].delta;
    }
    const int cv = p < ce ? p + cd : cmin;
    // registers, not memory: select into the array element
#pragma unroll
    for (int k = 0; k < kSellLaneEntries; ++k) cols[k] = k == e ? cv : cols[k];
  }
}

// Stores a row's n_rhs values (y row-major, aligned to n_rhs values).
template <class V, int NRHS>
__device__ __forceinline__ void store_rhs(V* dst, const V (&v)[NRHS]) {
  if constexpr (NRHS == 1) {
    dst[0] = v[0];
  } else if constexpr (NRHS == 2) {
    *reinterpret_cast<float2*>(dst) = make_float2(v[0], v[1]);
  } else {
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Chunk c of a's matrix on one workgroup.  part: LDS for the waves' row
// sums, kGroupWaves * NRHS * 64 values.  V: the vectors' type (float, or
// double for one FP64 vector: FP64 products and sums in the same order).
template <class V, int VF, int SM, int IX, bool WIN, int NRHS>
__device__ __forceinline__ void sell_chunk(const SellArgs& a, int64_t c, float* xw, V* part) {
  const int tid = static_cast<int>(threadIdx.x);
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const SellChunk* ch = a.chunks + c;
  const uint32_t slice0 = ch->slice0;
  const int T = static_cast<int>(ch->n_slices);
  const uint32_t min_len = ch->min_len;
  const int64_t pos = c * kSellC + lane;
  // the lane's row (written by the first wave at the end) and its length
  const uint32_t my_row = a.perm[pos];
  const int len = static_cast<int>(a.len[pos]);
  const char* val = static_cast<const char*>(a.val);
  const char* col = static_cast<const char*>(a.col);
  // run-length indices: the chunk's runs (staged in LDS after the window) and
  // the lane's run range, relative to the chunk's first run
  SellRun* lruns = reinterpret_cast<SellRun*>(xw + a.win_floats + kSellLaneEntries);
  int nruns = 0, rb = 0, re = 0;
  SellRun q0{}, q1{};
  uint32_t g0 = 0;
  if constexpr (IX == 0) {
    g0 = a.run_ptr[c * kSellC];
    nruns = static_cast<int>(a.run_ptr[(c + 1) * kSellC] - g0);
    rb = static_cast<int>(a.run_ptr[pos] - g0);
    re = static_cast<int>(a.run_ptr[pos + 1] - g0);
    const SellRun* gr = a.runs + g0;
    const SellRun* safe = reinterpret_cast<const SellRun*>(ch);
    q0 = *(tid < nruns ? gr + tid : safe);
    q1 = *(tid + kGroupThreads < nruns ? gr + tid + kGroupThreads : safe);
  }
  // Loads in the order they are needed, every one issued whatever the chunk
  // (a thread without a window piece reads the chunk record instead; a chunk
  // without slices re-reads its first slice position, inside the padded
  // streams), so that the compiler's count of loads in flight stays exact and
  // waiting for the window leaves the slices in flight: the x window (16-byte
  // pieces, a thread's first four at once), then the wave's first NB slices.
  const int cmin = static_cast<int>(a.win[2 * c]);  // also the padding column
  // window 4-byte words (its columns times NRHS, two per FP64 value), whole 16-byte pieces
  int nf = 0, n4 = 0;
  const float* xs = static_cast<const float*>(a.x);
  float4 w0, w1, w2, w3;
  float wt = 0.0f;
  if constexpr (WIN) {
    nf = static_cast<int>(a.win[2 * c + 1]) * NRHS * static_cast<int>(sizeof(V) / 4);
    xs = reinterpret_cast<const float*>(static_cast<const V*>(a.x) + static_cast<int64_t>(cmin) * NRHS);
    n4 = nf >> 2;
    const float4* xs4 = reinterpret_cast<const float4*>(xs);
    const float4* safe4 = reinterpret_cast<const float4*>(ch);
    w0 = *(tid < n4 ? xs4 + tid : safe4);
    w1 = *(tid + kGroupThreads < n4 ? xs4 + tid + kGroupThreads : safe4);
    w2 = *(tid + 2 * kGroupThreads < n4 ? xs4 + tid + 2 * kGroupThreads : safe4);
    w3 = *(tid + 3 * kGroupThreads < n4 ? xs4 + tid + 3 * kGroupThreads : safe4);
    const int tt = 4 * n4 + tid;
    wt = *(tt < nf ? xs + tt : reinterpret_cast<const float*>(ch));
  }
  constexpr int NB = ring_depth<VF, IX, NRHS>();
  // slice k of the wave, clamped to the chunk's last (or, without slices, its
  // first slice position)
  auto slice_of = [&](int t) { return slice0 + static_cast<uint32_t>(max(min(t, T - 1), 0)); };
  Lane8<VF, IX> r[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) load_slice<VF, IX>(val, col, slice_of(wave + k * kGroupWaves), lane, r[k]);
  if constexpr (WIN) {
    float4* xw4 = reinterpret_cast<float4*>(xw);
    const float4* xs4 = reinterpret_cast<const float4*>(xs);
    if (tid < n4) xw4[tid] = w0;
    if (tid + kGroupThreads < n4) xw4[tid + kGroupThreads] = w1;
    if (tid + 2 * kGroupThreads < n4) xw4[tid + 2 * kGroupThreads] = w2;
    if (tid + 3 * kGroupThreads < n4) xw4[tid + 3 * kGroupThreads] = w3;
    if (4 * n4 + tid < nf) xw[4 * n4 + tid] = wt;
    // windows larger than one batch
    for (int j = tid + 4 * kGroupThreads; j < n4; j += kGroupThreads) xw4[j] = xs4[j];
  }
  if constexpr (IX == 0) {
    if (tid < nruns) lruns[tid] = q0;
    if (tid + kGroupThreads < nruns) lruns[tid + kGroupThreads] = q1;
    for (int j = tid + 2 * kGroupThreads; j < nruns; j += kGroupThreads) lruns[j] = a.runs[g0 + j];
  }
#pragma unroll
  for (int q = 0; q < NRHS; ++q) part[(wave * NRHS + q) * kWave + lane] = V(0);
  __syncthreads();
  if (wave < T) {
    const V* xb = reinterpret_cast<const V*>(xw) - cmin * NRHS;
    const V* xg = static_cast<const V*>(a.x);
    V inner[NRHS], outer[NRHS];
#pragma unroll
    for (int q = 0; q < NRHS; ++q) inner[q] = V(0), outer[q] = V(0);
    int cnt = 0;
    // run cursor: run ri (of the lane's [rb, re)) ends at cur_end and its
    // entries have column = position + cur_delta; the next run (nx_end,
    // nx_delta) is held too (nx_end = cur_end when there is none)
    int ri = rb, cur_end = 0, cur_delta = 0, nx_end = 0, nx_delta = 0;
    auto next_run = [&]() {
      nx_end = cur_end, nx_delta = 0;
      if (ri + 1 < re) nx_end = lruns[ri + 1].end, nx_delta = lruns[ri + 1].delta;
    };
    if constexpr (IX == 0) {
      if (ri < re) cur_end = lruns[ri].end, cur_delta = lruns[ri].delta;
      next_run();
    }
    int t = wave;
    // one slice (a step past the chunk's slices only refills its buffer):
    // the columns, products, refill with the slice NB turns ahead, then the
    // slice sum
    auto step = [&](Lane8<VF, IX>& buf) {
      const bool live = t < T;
      const int P = t * kSellLaneEntries;
      V pr[kSellLaneEntries][NRHS];
      if (live) {
        int cols[kSellLaneEntries];
        if constexpr (IX == 0) {
          while (cur_end <= P && ri + 1 < re) {
            ++ri;
            cur_end = nx_end, cur_delta = nx_delta;
            next_run();
          }
          // an entry lies in the current run, in the next one, or past the
          // row (padding column)
#pragma unroll
          for (int e = 0; e < kSellLaneEntries; ++e) {
            const int p = P + e;
            cols[e] = p < cur_end ? p + cur_delta : p < nx_end ? p + nx_delta : cmin;
          }
          // an entry beyond the next run and inside the row: walk the runs
          const bool far = P + kSellLaneEntries > nx_end && nx_end < len;
          if (__ballot(far) != 0) {
            if (far) walk_runs(lruns, ri, re, cur_end, cur_delta, P, cmin, cols);
          }
        } else {
          lane_cols(buf, cols);
        }
        slice_products<V, VF, IX, WIN, NRHS>(buf, cols, xb, xg, pr);
      }
      __builtin_amdgcn_sched_barrier(0);
      load_slice<VF, IX>(val, col, slice_of(t + NB * kGroupWaves), lane, buf);
      __builtin_amdgcn_sched_barrier(0);
      if (live) {
        if (static_cast<uint32_t>(P + kSellLaneEntries) > min_len) {
          // some lane's row ends in or before this slice
          const int lim = len - P;
#pragma unroll
          for (int e = 0; e < kSellLaneEntries; ++e)
#pragma unroll
            for (int q = 0; q < NRHS; ++q) pr[e][q] = e < lim ? pr[e][q] : V(0);
        }
#pragma unroll
        for (int q = 0; q < NRHS; ++q) inner[q] += slice_sum<V, NRHS>(pr, q);
        if (++cnt == 8) {
#pragma unroll
          for (int q = 0; q < NRHS; ++q) {
            outer[q] += inner[q];
            inner[q] = V(0);
          }
          cnt = 0;
        }
      }
      t += kGroupWaves;
    };
    // one exit per turn of the ring
    while (true) {
#pragma unroll
      for (int k = 0; k < NB; ++k) step(r[k]);
      if (t >= T) break;
    }
#pragma unroll
    for (int q = 0; q < NRHS; ++q) part[(wave * NRHS + q) * kWave + lane] = outer[q] + inner[q];
  }
  __syncthreads();
  if (wave == 0 && my_row != 0xFFFFFFFFu) {
    V v[NRHS];
#pragma unroll
    for (int q = 0; q < NRHS; ++q) {
      const V* pq = part + q * kWave + lane;
      v[q] = (pq[0 * NRHS * kWave] + pq[1 * NRHS * kWave]) + (pq[2 * NRHS * kWave] + pq[3 * NRHS * kWave]);
      if constexpr (SM == kScaleRow) v[q] = v[q] * static_cast<V>(a.scale[my_row]);
    }
    store_rhs<V, NRHS>(static_cast<V*>(a.y) + static_cast<int64_t>(my_row) * NRHS, v);
  }
}

// Chunk c of a's matrix on one workgroup: through the LDS window when the
// chunk's window, for NRHS vectors of V, fits a's.
template <class V, int VF, int SM, int IX, int NRHS>
__device__ __forceinline__ void sell_run_chunk(const SellArgs& a, int64_t c, float* xw, V* part) {
  const uint32_t clen = a.win[2 * c + 1];
  if (clen > 0 && static_cast<int64_t>(clen) * NRHS * static_cast<int64_t>(sizeof(V) / 4) <= a.win_floats)
    sell_chunk<V, VF, SM, IX, true, NRHS>(a, c, xw, part);
  else
    sell_chunk<V, VF, SM, IX, false, NRHS>(a, c, xw, part);
}

// +0 to the rows of chunk c of a's matrix (one wave).
template <class V, int NRHS>
__device__ __forceinline__ void sell_zero_rows(const SellArgs& a, int64_t c) {
  const uint32_t row = a.perm[c * kSellC + (threadIdx.x & (kWave - 1))];
  if (row != 0xFFFFFFFFu) {
    const V z[NRHS] = {};
    store_rhs<V, NRHS>(static_cast<V*>(a.y) + static_cast<int64_t>(row) * NRHS, z);
  }
}

// Workgroups [0, n_groups) take the chunks holding entries (through the die
// regrouping); the rest write +0 to the rows of four chunks without entries
// each.
template <int VF, int SM, int IX, int NRHS>
__global__ __launch_bounds__(kGroupThreads) void k_sell(SellArgs a) {
  extern __shared__ __align__(16) float xw[];
  __shared__ float part[kGroupWaves * NRHS * kWave];
  if (blockIdx.x >= a.n_groups) {
    const int64_t z = (static_cast<int64_t>(blockIdx.x) - a.n_groups) * kGroupWaves + threadIdx.x / kWave;
    if (z < a.n_zero) sell_zero_rows<float, NRHS>(a, a.zero[z]);
    return;
  }
  sell_run_chunk<float, VF, SM, IX, NRHS>(a, a.work[sell_group_of_block(a.xcd_blocks, a.n_groups, blockIdx.x)], xw,
                                         part);
}

// One FP64 vector: FP64 x and y, products and sums (the paper's half/double
// arithmetic, Sec. II-D) in the same order.
template <int VF, int SM, int IX>
__global__ __launch_bounds__(kGroupThreads) void k_sell_f64(SellArgs a) {
  extern __shared__ __align__(16) float xw[];
  __shared__ double part[kGroupWaves * kWave];
  if (blockIdx.x >= a.n_groups) {
    const int64_t z = (static_cast<int64_t>(blockIdx.x) - a.n_groups) * kGroupWaves + threadIdx.x / kWave;
    if (z < a.n_zero) sell_zero_rows<double, 1>(a, a.zero[z]);
    return;
  }
  sell_run_chunk<double, VF, SM, IX, 1>(a, a.work[sell_group_of_block(a.xcd_blocks, a.n_groups, blockIdx.x)], xw,
                                        part);
}

// Batched form: the same over the work lists of many matrices, each entry
// naming its item.
template <int VF, int SM, int IX, int NRHS>
__global__ __launch_bounds__(kGroupThreads) void k_sell_batched(SellBatchTable t) {
  extern __shared__ __align__(16) float xw[];
  __shared__ float part[kGroupWaves * NRHS * kWave];
  if (blockIdx.x >= t.n_work) {
    const int64_t z = (static_cast<int64_t>(blockIdx.x) - t.n_work) * kGroupWaves + threadIdx.x / kWave;
    if (z < t.n_zero) {
      const uint2 w = t.zero[z];
      sell_zero_rows<float, NRHS>(t.args[w.x], w.y);
    }
    return;
  }
  const uint2 w = t.work[sell_group_of_block(t.xcd_blocks, t.n_work, blockIdx.x)];
  sell_run_chunk<float, VF, SM, IX, NRHS>(t.args[w.x], w.y, xw, part);
}

// LDS of a launch: the window, then (run-length indices) one lane's entries
// of padding and the chunk's runs.
size_t sell_lds_bytes(const SellArgs& a) {
  if (a.idx_bytes != 0) return static_cast<size_t>(a.win_floats) * sizeof(float);
  return (static_cast<size_t>(a.win_floats) + kSellLaneEntries) * sizeof(float) +
         static_cast<size_t>(a.lds_runs) * sizeof(SellRun);
}

template <int VF, int SM, int NRHS>
void launch_ix(const SellArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_groups + (a.n_zero + kGroupWaves - 1) / kGroupWaves)),
      block(kGroupThreads);
  const size_t lds = sell_lds_bytes(a);
  if (a.idx_bytes == 0)
    hipLaunchKernelGGL((k_sell<VF, SM, 0, NRHS>), grid, block, lds, s, a);
  else if (a.idx_bytes == 2)
    hipLaunchKernelGGL((k_sell<VF, SM, 2, NRHS>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((k_sell<VF, SM, 4, NRHS>), grid, block, lds, s, a);
}

template <int VF, int SM, int NRHS>
void launch_ix_batched(int idx_bytes, const SellBatchTable& t, size_t lds, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(t.n_work + (t.n_zero + kGroupWaves - 1) / kGroupWaves)),
      block(kGroupThreads);
  if (idx_bytes == 0)
    hipLaunchKernelGGL((k_sell_batched<VF, SM, 0, NRHS>), grid, block, lds, s, t);
  else if (idx_bytes == 2)
    hipLaunchKernelGGL((k_sell_batched<VF, SM, 2, NRHS>), grid, block, lds, s, t);
  else
    hipLaunchKernelGGL((k_sell_batched<VF, SM, 4, NRHS>), grid, block, lds, s, t);
}

template <int VF, int SM>
hipError_t launch_vf_f64(const SellArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_groups + (a.n_zero + kGroupWaves - 1) / kGroupWaves)),
      block(kGroupThreads);
  const size_t lds = sell_lds_bytes(a);
  if (a.idx_bytes == 0)
    hipLaunchKernelGGL((k_sell_f64<VF, SM, 0>), grid, block, lds, s, a);
  else if (a.idx_bytes == 2)
    hipLaunchKernelGGL((k_sell_f64<VF, SM, 2>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((k_sell_f64<VF, SM, 4>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <int VF, int SM>
hipError_t launch_vf(int n_rhs, const SellArgs& a, hipStream_t s) {
  switch (n_rhs) {
    case 1: launch_ix<VF, SM, 1>(a, s); break;
    case 2: launch_ix<VF, SM, 2>(a, s); break;
    case 4: launch_ix<VF, SM, 4>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int VF, int SM>
hipError_t launch_vf_batched(int n_rhs, int idx_bytes, const SellBatchTable& t, size_t lds, hipStream_t s) {
  switch (n_rhs) {
    case 1: launch_ix_batched<VF, SM, 1>(idx_bytes, t, lds, s); break;
    case 2: launch_ix_batched<VF, SM, 2>(idx_bytes, t, lds, s); break;
    case 4: launch_ix_batched<VF, SM, 4>(idx_bytes, t, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t sell_launch_lds_bytes(const SellArgs& a) { return sell_lds_bytes(a); }

hipError_t launch_sell_spmv(int vf, int scale_mode, int n_rhs, const SellArgs& a, hipStream_t s) {
  if (a.n_groups <= 0 && a.n_zero <= 0) return hipSuccess;
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_vf<kFp16, kScaleNone>(n_rhs, a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_vf<kBf16, kScaleNone>(n_rhs, a, s);
  if (vf == kFp32 && scale_mode == kScaleNone) return launch_vf<kFp32, kScaleNone>(n_rhs, a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_vf<kFp8, kScaleRow>(n_rhs, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_sell_spmv_f64(int vf, int scale_mode, const SellArgs& a, hipStream_t s) {
  if (a.n_groups <= 0 && a.n_zero <= 0) return hipSuccess;
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_vf_f64<kFp16, kScaleNone>(a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_vf_f64<kBf16, kScaleNone>(a, s);
  if (vf == kFp32 && scale_mode == kScaleNone) return launch_vf_f64<kFp32, kScaleNone>(a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_vf_f64<kFp8, kScaleRow>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_sell_batched(int vf, int scale_mode, int n_rhs, int idx_bytes, const SellBatchTable& t,
                               size_t lds_bytes, hipStream_t s) {
  if (t.n_work <= 0 && t.n_zero <= 0) return hipSuccess;
  if (vf == kFp16 && scale_mode == kScaleNone)
    return launch_vf_batched<kFp16, kScaleNone>(n_rhs, idx_bytes, t, lds_bytes, s);
  if (vf == kBf16 && scale_mode == kScaleNone)
    return launch_vf_batched<kBf16, kScaleNone>(n_rhs, idx_bytes, t, lds_bytes, s);
  if (vf == kFp32 && scale_mode == kScaleNone)
    return launch_vf_batched<kFp32, kScaleNone>(n_rhs, idx_bytes, t, lds_bytes, s);
  if (vf == kFp8 && scale_mode == kScaleRow)
    return launch_vf_batched<kFp8, kScaleRow>(n_rhs, idx_bytes, t, lds_bytes, s);
  return hipErrorInvalidValue;
}

}  // namespace dose
