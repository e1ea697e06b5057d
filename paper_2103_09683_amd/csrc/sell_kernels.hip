// SELL-C-sigma product kernel of libdose for gfx950 (CDNA4, wave64).
//
// SELL-C-sigma (Kreutzer et al., SIAM J. Sci. Comput. 36(5), 2014) is the
// SIMD-oriented sparse format the paper names as the next one to try for dose
// matrices (Sec. II-C, Sec. VII).  Rows are sorted by descending length
// inside windows of sigma rows and cut into chunks of C = 64 rows, one row per
// lane of a wave64, so no row needs a cross-lane reduction and the lanes of a
// wave stream their rows side by side.  Here a chunk stores its entries in
// slices of 8 per lane (dose_internal.h): a lane reads its row's next 8 codes
// with one 16-byte load (FP16), and a wave's load instruction covers 1 KB of
// consecutive codes.
//
//   * A workgroup (four waves) takes a group of four consecutive chunks and
//     copies the group's x window into LDS once (the rows of a sigma window
//     are neighbouring voxels, so their spots lie in a narrow range); a group
//     whose window exceeds the LDS cap gathers x from global memory.
//   * The group's slices, chunk after chunk, are dealt to the waves in turn
//     (wave j takes slices j, j + 4, ...), so a wide chunk keeps all four
//     waves busy; the next slice's loads are in flight while one is computed.
//   * Summation order, fixed by the stored layout (so equal inputs give equal
//     bits): a lane's 8 products of a slice add pairwise, ((p0 + p1) +
//     (p2 + p3)) + ((p4 + p5) + (p6 + p7)), slots past the row's end counting
//     as +0; each wave adds its slice sums of a chunk in order, eight at a
//     time into an inner sum that is then added to an outer one (the FP32
//     error of a row of L entries stays below (14 + L / 256) * 2^-24 of
//     sum |a x|); the four waves' sums of a row meet as (S0 + S1) + (S2 + S3).
//     Empty rows get +0.
#include "dose_internal.h"

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
    L.c0 = ld_nt4(vb, o * 4u);
    L.c1 = ld_nt4(vb, o * 4u + 16u);
  } else {
    L.c0 = ld_nt4(vb, o * 2u);
  }
  if constexpr (IX == 4) {
    L.i0 = ld_nt4(cb, o * 4u);
    L.i1 = ld_nt4(cb, o * 4u + 16u);
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

// The lane's 8 products of a slice: decoded code times x of its column.
// x comes from the LDS window (xb: the window moved back by cmin columns) or
// from global memory.
template <int VF, int IX, bool WIN>
__device__ __forceinline__ void slice_products(const Lane8<VF, IX>& L, const int (&c)[kSellLaneEntries],
                                               const float* xb, const float* x, float (&p)[kSellLaneEntries]) {
  float xv[kSellLaneEntries];
#pragma unroll
  for (int e = 0; e < kSellLaneEntries; ++e) {
    if constexpr (WIN) {
      xv[e] = xb[c[e]];
    } else {
      xv[e] = x[c[e]];
    }
  }
  if constexpr (VF == kFp16) {
    const uint32_t w[4] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) {
      const float d = __half2float(__ushort_as_half(static_cast<unsigned short>((w[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu)));
      // an FMA with +0 rounds the product once, as a multiply does (v_fma_mix)
      p[e] = __builtin_fmaf(d, xv[e], 0.0f);
    }
  } else if constexpr (VF == kBf16) {
    const uint32_t w[4] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) {
      const uint32_t word = w[e >> 1];
      p[e] = __uint_as_float((e & 1) ? (word & 0xFFFF0000u) : (word << 16)) * xv[e];
    }
  } else if constexpr (VF == kFp8) {
    const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.x), false);
    const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.x), true);
    const f32x2 cc = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.y), false);
    const f32x2 d = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(L.c0.y), true);
    const float q[8] = {a.x, a.y, b.x, b.y, cc.x, cc.y, d.x, d.y};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) p[e] = q[e] * xv[e];
  } else {
    const uint32_t w[8] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w, L.c1.x, L.c1.y, L.c1.z, L.c1.w};
#pragma unroll
    for (int e = 0; e < kSellLaneEntries; ++e) p[e] = __uint_as_float(w[e]) * xv[e];
  }
}

__device__ __forceinline__ float slice_sum(const float (&p)[kSellLaneEntries]) {
  return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

// The workgroup of group b (see group_of_block in the CSR kernels: with D
// dies dealt workgroups in turn, die x takes one contiguous run of groups).
__device__ __forceinline__ int64_t sell_group_of_block(const SellArgs& a, uint32_t b) {
  const int D = a.xcd_blocks;
  if (D <= 1) return b;
  const int64_t q = a.n_groups / D, r = a.n_groups % D;
  const int64_t x = b % static_cast<uint32_t>(D), i = b / static_cast<uint32_t>(D);
  return x * q + (x < r ? x : r) + i;
}

// Wave-uniform pick of one of four values by a wave-uniform index.
template <class T>
__device__ __forceinline__ T pick4(int c, T v0, T v1, T v2, T v3) {
  return c == 0 ? v0 : c == 1 ? v1 : c == 2 ? v2 : v3;
}

template <int VF, int SM, int IX, bool WIN>
__device__ __forceinline__ void sell_group(const SellArgs& a, int64_t g, float* xw,
                                           float (*part)[kGroupWaves][kWave]) {
  const int tid = static_cast<int>(threadIdx.x);
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const SellChunk* chs = a.chunks + g * kSellGroupChunks;
  const uint32_t slice0 = chs[0].slice0;
  const int b1 = static_cast<int>(chs[0].n_slices);
  const int b2 = b1 + static_cast<int>(chs[1].n_slices);
  const int b3 = b2 + static_cast<int>(chs[2].n_slices);
  const int T = b3 + static_cast<int>(chs[3].n_slices);
  const uint32_t m0 = chs[0].min_len, m1 = chs[1].min_len, m2 = chs[2].min_len, m3 = chs[3].min_len;
  const int64_t pos0 = g * kSellGroupRows;
  // this thread's row position at the end, and the lane's row lengths in the
  // four chunks (a wave's slices may belong to any of them)
  const uint32_t my_row = a.perm[pos0 + tid];
  const uint32_t len0 = a.len[pos0 + lane], len1 = a.len[pos0 + kWave + lane];
  const uint32_t len2 = a.len[pos0 + 2 * kWave + lane], len3 = a.len[pos0 + 3 * kWave + lane];
  const char* val = static_cast<const char*>(a.val);
  const char* col = static_cast<const char*>(a.col);
  // run-length indices: the group's runs (staged in LDS after the window) and
  // each lane's run range in the four chunks, relative to the group's first run
  SellRun* lruns = reinterpret_cast<SellRun*>(xw + a.win_floats + kSellLaneEntries);
  int nruns = 0, rb0 = 0, rb1 = 0, rb2 = 0, rb3 = 0, re0 = 0, re1 = 0, re2 = 0, re3 = 0;
  SellRun q0{}, q1{};
  if constexpr (IX == 0) {
    const uint32_t g0 = a.run_ptr[pos0];
    nruns = static_cast<int>(a.run_ptr[pos0 + kSellGroupRows] - g0);
    const uint32_t* rp = a.run_ptr + pos0 + lane;
    rb0 = static_cast<int>(rp[0] - g0), re0 = static_cast<int>(rp[1] - g0);
    rb1 = static_cast<int>(rp[kWave] - g0), re1 = static_cast<int>(rp[kWave + 1] - g0);
    rb2 = static_cast<int>(rp[2 * kWave] - g0), re2 = static_cast<int>(rp[2 * kWave + 1] - g0);
    rb3 = static_cast<int>(rp[3 * kWave] - g0), re3 = static_cast<int>(rp[3 * kWave + 1] - g0);
    const SellRun* gr = a.runs + g0;
    const SellRun* safe = reinterpret_cast<const SellRun*>(chs);
    q0 = *(tid < nruns ? gr + tid : safe);
    q1 = *(tid + kGroupThreads < nruns ? gr + tid + kGroupThreads : safe);
  }
  // Loads in the order they are needed: the x window (16-byte pieces, a
  // thread's first four at once; a thread without a piece reads the chunk
  // records instead, so that the number of loads is fixed), then the wave's
  // first two slices; waiting for the window leaves the slices in flight.
  int cmin = 0, clen = 0, n4 = 0;
  const float* xs = a.x;
  float4 w0, w1, w2, w3;
  float wt = 0.0f;
  if constexpr (WIN) {
    cmin = static_cast<int>(a.win[2 * g]);
    clen = static_cast<int>(a.win[2 * g + 1]);
    xs = a.x + cmin;
    n4 = clen >> 2;
    const float4* xs4 = reinterpret_cast<const float4*>(xs);
    const float4* safe4 = reinterpret_cast<const float4*>(chs);
    w0 = *(tid < n4 ? xs4 + tid : safe4);
    w1 = *(tid + kGroupThreads < n4 ? xs4 + tid + kGroupThreads : safe4);
    w2 = *(tid + 2 * kGroupThreads < n4 ? xs4 + tid + 2 * kGroupThreads : safe4);
    w3 = *(tid + 3 * kGroupThreads < n4 ? xs4 + tid + 3 * kGroupThreads : safe4);
    const int tt = 4 * n4 + tid;
    wt = *(tt < clen ? xs + tt : reinterpret_cast<const float*>(chs));
  } else {
    cmin = static_cast<int>(a.win[2 * g]);  // the padding column, a valid column of the group
  }
  Lane8<VF, IX> r0, r1;
  const bool has = wave < T;
  if (has) {
    load_slice<VF, IX>(val, col, slice0 + static_cast<uint32_t>(wave), lane, r0);
    load_slice<VF, IX>(val, col, slice0 + static_cast<uint32_t>(min(wave + kGroupWaves, T - 1)), lane, r1);
  }
  if constexpr (WIN) {
    float4* xw4 = reinterpret_cast<float4*>(xw);
    const float4* xs4 = reinterpret_cast<const float4*>(xs);
    if (tid < n4) xw4[tid] = w0;
    if (tid + kGroupThreads < n4) xw4[tid + kGroupThreads] = w1;
    if (tid + 2 * kGroupThreads < n4) xw4[tid + 2 * kGroupThreads] = w2;
    if (tid + 3 * kGroupThreads < n4) xw4[tid + 3 * kGroupThreads] = w3;
    if (4 * n4 + tid < clen) xw[4 * n4 + tid] = wt;
    // windows larger than one batch
    for (int j = tid + 4 * kGroupThreads; j < n4; j += kGroupThreads) xw4[j] = xs4[j];
  }
  if constexpr (IX == 0) {
    if (tid < nruns) lruns[tid] = q0;
    if (tid + kGroupThreads < nruns) lruns[tid + kGroupThreads] = q1;
    for (int j = tid + 2 * kGroupThreads; j < nruns; j += kGroupThreads) lruns[j] = a.runs[a.run_ptr[pos0] + j];
  }
#pragma unroll
  for (int c = 0; c < kSellGroupChunks; ++c) part[c][wave][lane] = 0.0f;
  __syncthreads();
  if (has) {
    const float* xb = xw - cmin;
    float inner = 0.0f, outer = 0.0f;
    int cnt = 0, cc = -1;
    // run cursor of the lane's row in chunk cc: run ri (of [ri, rend)) ends
    // at cur_end, with column = position + cur_delta
    int ri = 0, rend = 0, cur_end = 0, cur_delta = 0;
    int t = wave;
    // one slice: the columns, products, refill of its buffer with the slice
    // two turns ahead, then the slice sum into the current chunk's sums
    auto step = [&](Lane8<VF, IX>& buf) {
      const int c = (t >= b1) + (t >= b2) + (t >= b3);
      if (c != cc) {
        if (cc >= 0) part[cc][wave][lane] = outer + inner;
        inner = 0.0f, outer = 0.0f, cnt = 0;
        cc = c;
        if constexpr (IX == 0) {
          ri = pick4(c, rb0, rb1, rb2, rb3);
          rend = pick4(c, re0, re1, re2, re3);
          cur_end = 0, cur_delta = 0;
          if (ri < rend) cur_end = lruns[ri].end, cur_delta = lruns[ri].delta;
        }
      }
      const int sl = t - pick4(c, 0, b1, b2, b3);
      const int lenc = static_cast<int>(pick4(c, len0, len1, len2, len3));
      int cols[kSellLaneEntries];
      if constexpr (IX == 0) {
        const int P = sl * kSellLaneEntries;
        while (cur_end <= P && ri + 1 < rend) {
          ++ri;
          cur_end = lruns[ri].end, cur_delta = lruns[ri].delta;
        }
        // a lane whose 8 entries lie in one run (or, with the LDS window
        // padded by 8 columns, wholly past its row) reads 8 consecutive x
        const bool past = WIN && P >= lenc;
        const bool run8 = past || P + kSellLaneEntries <= cur_end;
        if (__ballot(!run8) == 0) {
          const int base = past ? cmin : P + cur_delta;
#pragma unroll
          for (int e = 0; e < kSellLaneEntries; ++e) cols[e] = base + e;
        } else {
          // some lane's run ends inside the slice: walk the runs entry by
          // entry; entries past the row take the group's padding column
          int j = ri, ce = cur_end, cd = cur_delta;
#pragma unroll
          for (int e = 0; e < kSellLaneEntries; ++e) {
            const int pos = P + e;
            while (pos >= ce && j + 1 < rend) {
              ++j;
              ce = lruns[j].end, cd = lruns[j].delta;
            }
            cols[e] = pos < ce ? pos + cd : cmin;
          }
        }
      } else {
        lane_cols(buf, cols);
      }
      float p[kSellLaneEntries];
      slice_products<VF, IX, WIN>(buf, cols, xb, a.x, p);
      __builtin_amdgcn_sched_barrier(0);
      load_slice<VF, IX>(val, col, slice0 + static_cast<uint32_t>(min(t + 2 * kGroupWaves, T - 1)), lane, buf);
      __builtin_amdgcn_sched_barrier(0);
      if (static_cast<uint32_t>(sl + 1) * kSellLaneEntries > pick4(c, m0, m1, m2, m3)) {
        // some lane's row ends in or before this slice
        const int lim = lenc - sl * kSellLaneEntries;
#pragma unroll
        for (int e = 0; e < kSellLaneEntries; ++e) p[e] = e < lim ? p[e] : 0.0f;
      }
      inner += slice_sum(p);
      if (++cnt == 8) {
        outer += inner;
        inner = 0.0f;
        cnt = 0;
      }
      t += kGroupWaves;
    };
    while (true) {
      step(r0);
      if (t >= T) break;
      step(r1);
      if (t >= T) break;
    }
    part[cc][wave][lane] = outer + inner;
  }
  __syncthreads();
  if (my_row != 0xFFFFFFFFu) {
    const int c = tid / kWave;
    float v = (part[c][0][lane] + part[c][1][lane]) + (part[c][2][lane] + part[c][3][lane]);
    if constexpr (SM == kScaleRow) v = v * a.scale[my_row];
    a.y[my_row] = v;
  }
}

template <int VF, int SM, int IX>
__global__ __launch_bounds__(kGroupThreads) void k_sell(SellArgs a) {
  extern __shared__ __align__(16) float xw[];
  __shared__ float part[kSellGroupChunks][kGroupWaves][kWave];
  const int64_t g = sell_group_of_block(a, blockIdx.x);
  const uint32_t clen = a.win[2 * g + 1];
  if (clen > 0 && static_cast<int64_t>(clen) <= a.win_floats)
    sell_group<VF, SM, IX, true>(a, g, xw, part);
  else
    sell_group<VF, SM, IX, false>(a, g, xw, part);
}

template <int VF, int SM>
hipError_t launch_vf(const SellArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.n_groups)), block(kGroupThreads);
  if (a.idx_bytes == 0) {
    // the window padded by one lane's entries, then the group's runs
    const size_t lds = (static_cast<size_t>(a.win_floats) + kSellLaneEntries) * sizeof(float) +
                       static_cast<size_t>(a.lds_runs) * sizeof(SellRun);
    hipLaunchKernelGGL((k_sell<VF, SM, 0>), grid, block, lds, s, a);
    return hipGetLastError();
  }
  const size_t lds = static_cast<size_t>(a.win_floats) * sizeof(float);
  if (a.idx_bytes == 2)
    hipLaunchKernelGGL((k_sell<VF, SM, 2>), grid, block, lds, s, a);
  else
    hipLaunchKernelGGL((k_sell<VF, SM, 4>), grid, block, lds, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sell_spmv(int vf, int scale_mode, const SellArgs& a, hipStream_t s) {
  if (a.n_groups <= 0) return hipSuccess;
  if (vf == kFp16 && scale_mode == kScaleNone) return launch_vf<kFp16, kScaleNone>(a, s);
  if (vf == kBf16 && scale_mode == kScaleNone) return launch_vf<kBf16, kScaleNone>(a, s);
  if (vf == kFp32 && scale_mode == kScaleNone) return launch_vf<kFp32, kScaleNone>(a, s);
  if (vf == kFp8 && scale_mode == kScaleRow) return launch_vf<kFp8, kScaleRow>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace dose
