// Host side of libdose: the C ABI declared in include/dose.h.
//
// Responsibilities: argument and CSR validation, the row-block partition that
// fixes every summation order, device memory of matrices and plans, the
// one-time encode/transpose pipeline, batched work lists captured into HIP
// graphs, and a small autotuner whose choices persist in a text cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dose.h"
#include "dose_internal.h"
#include "sell_internal.h"
#include "slab_internal.h"

using namespace dose;

// ------------------------------------------------------------------ errors
namespace {

thread_local std::string g_last_error;

struct DoseError {
  dose_status code;
  std::string msg;
};

[[noreturn]] void fail(dose_status code, const std::string& msg) { throw DoseError{code, msg}; }

#define HIP_CHECK(expr)                                                                       \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) {                                                                   \
      if (_e == hipErrorOutOfMemory) fail(DOSE_ERR_OUT_OF_MEMORY, std::string(#expr) + ": " + \
                                                                      hipGetErrorString(_e)); \
      fail(DOSE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));                  \
    }                                                                                         \
  } while (0)

template <typename F>
dose_status guarded(F&& f) {
  try {
    f();
    return DOSE_OK;
  } catch (const DoseError& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DOSE_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DOSE_ERR_INTERNAL;
  } catch (...) {
    g_last_error = "unknown error";
    return DOSE_ERR_INTERNAL;
  }
}

// --------------------------------------------------- allocation fault injection
// DOSE_FAULT_INJECT=alloc:<n> makes the n-th device allocation, counted from
// the moment the variable took that value, report out-of-memory (to test
// cleanup paths); read at every allocation, so a process can arm it again.
std::mutex g_fault_mu;
std::string g_fault_spec;
int64_t g_fault_count = 0;

bool injected_fault() {
  std::lock_guard<std::mutex> lk(g_fault_mu);
  const char* e = std::getenv("DOSE_FAULT_INJECT");
  const std::string spec = e ? e : "";
  if (spec != g_fault_spec) {
    g_fault_spec = spec;
    g_fault_count = 0;
  }
  if (spec.compare(0, 6, "alloc:") != 0) return false;
  return ++g_fault_count == std::atoll(spec.c_str() + 6);
}

void* dev_alloc(size_t bytes) {
  if (injected_fault()) fail(DOSE_ERR_OUT_OF_MEMORY, "injected allocation failure");
  void* p = nullptr;
  HIP_CHECK(hipMalloc(&p, bytes == 0 ? 256 : bytes));
  return p;
}

// Device memory owned by one object.
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) : p_(dev_alloc(bytes)), n_(bytes) {}
  ~DevBuf() { reset(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr, o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p_ = o.p_, n_ = o.n_;
      o.p_ = nullptr, o.n_ = 0;
    }
    return *this;
  }
  void reset() {
    if (p_) (void)hipFree(p_);
    p_ = nullptr, n_ = 0;
  }
  template <typename T = void>
  T* get() const {
    return static_cast<T*>(p_);
  }
  size_t bytes() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// Restores the calling thread's current device on scope exit.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    HIP_CHECK(hipGetDevice(&prev_));
    if (prev_ != dev) HIP_CHECK(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev_); }

 private:
  int prev_ = 0;
};

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int value_bytes(int vf) { return vf == kFp8 ? 1 : vf == kFp32 ? 4 : 2; }

// ------------------------------------------------------------- validation
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// FP32 value that rounds to infinity in the target 16-bit format?
bool overflows(int vf, float v) {
  const float a = std::fabs(v);
  if (vf == kFp16) return a >= 65520.0f;
  if (vf == kBf16) {
    uint32_t u;
    std::memcpy(&u, &a, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u >> 16) >= 0x7F80u;
  }
  return false;
}

void validate_csr(const dose_csr_host* c, int vf, int xf) {
  if (!c) fail(DOSE_ERR_INVALID_ARGUMENT, "csr is null");
  if (vf != kFp16 && vf != kBf16 && vf != kFp8 && vf != kFp32) fail(DOSE_ERR_INVALID_ARGUMENT, "unknown value format");
  if (xf != DOSE_IDX_I32 && xf != DOSE_IDX_U16 && xf != DOSE_IDX_RUNS)
    fail(DOSE_ERR_INVALID_ARGUMENT, "unknown index format");
  if (c && xf == DOSE_IDX_U16 && c->n_cols > 65536) fail(DOSE_ERR_UNSUPPORTED, "16-bit indices need n_cols <= 65536");
  if (c->n_rows < 0 || c->n_cols < 0 || c->nnz < 0) fail(DOSE_ERR_INVALID_ARGUMENT, "negative size");
  if (c->n_rows >= (int64_t{1} << 32) - 1) fail(DOSE_ERR_UNSUPPORTED, "more than 2^32-2 rows");
  if (c->n_cols > INT32_MAX) fail(DOSE_ERR_UNSUPPORTED, "more than 2^31-1 columns");
  if (!c->row_ptr) fail(DOSE_ERR_INVALID_ARGUMENT, "row_ptr is null");
  if (c->nnz > 0 && (!c->col_idx || !c->values)) fail(DOSE_ERR_INVALID_ARGUMENT, "col_idx or values is null");
  if (c->row_ptr[0] != 0) fail(DOSE_ERR_BAD_CSR, "row_ptr[0] != 0");
  if (c->row_ptr[c->n_rows] != c->nnz) fail(DOSE_ERR_BAD_CSR, "row_ptr[n_rows] != nnz");
  if (c->nnz > 0 && c->n_cols == 0) fail(DOSE_ERR_BAD_CSR, "entries in a matrix without columns");

  const int64_t n = c->n_rows;
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t parts = std::min<int64_t>(hw, std::max<int64_t>(1, c->nnz / (1 << 22)));
  std::vector<int> code(parts, DOSE_OK);
  std::vector<std::string> msg(parts);
  auto work = [&](int64_t part) {
    const int64_t r0 = n * part / parts, r1 = n * (part + 1) / parts;
    for (int64_t i = r0; i < r1; ++i) {
      const int64_t b = c->row_ptr[i], e = c->row_ptr[i + 1];
      if (e < b || b < 0 || e > c->nnz) {
        code[part] = DOSE_ERR_BAD_CSR;
        msg[part] = "row_ptr decreases or leaves [0, nnz] at row " + std::to_string(i);
        return;
      }
      int64_t prev = -1;
      for (int64_t k = b; k < e; ++k) {
        const int64_t j = c->col_idx[k];
        if (j < 0 || j >= c->n_cols) {
          code[part] = DOSE_ERR_BAD_CSR;
          msg[part] = "column out of range at entry " + std::to_string(k);
          return;
        }
        if (j <= prev) {
          code[part] = DOSE_ERR_BAD_CSR;
          msg[part] = "columns not strictly ascending in row " + std::to_string(i);
          return;
        }
        prev = j;
        const float v = c->values[k];
        if (!std::isfinite(v)) {
          code[part] = DOSE_ERR_BAD_CSR;
          msg[part] = "non-finite value at entry " + std::to_string(k);
          return;
        }
        if (overflows(vf, v)) {
          code[part] = DOSE_ERR_UNSUPPORTED;
          msg[part] = "value at entry " + std::to_string(k) + " overflows the format";
          return;
        }
      }
    }
  };
  if (parts == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int64_t p = 0; p < parts; ++p) th.emplace_back(work, p);
    for (auto& t : th) t.join();
  }
  for (int64_t p = 0; p < parts; ++p)
    if (code[p] != DOSE_OK) fail(code[p], msg[p]);
}

// -------------------------------------------------------------- partition
// Row groups: runs of whole rows holding about group_nnz entries (a longer
// row forms a group of its own), at most kMaxGroupRows rows, each split into
// kGroupWaves contiguous shares of nearly equal cost (entries plus 16 per
// row: an empty row still costs an offset load and a store).  The partition
// only decides which wave computes which row; it never changes the order in
// which a row is summed.  brk (optional, one flag per row): a group never
// runs across a row whose flag is set (it starts a new group).
std::vector<GroupDesc> build_partition(const int64_t* rp, int64_t n_rows, int group_nnz,
                                       const uint8_t* brk = nullptr) {
  std::vector<GroupDesc> G;
  G.reserve(static_cast<size_t>(rp[n_rows] / group_nnz + n_rows / kMaxGroupRows + 16));
  const int64_t kRowCost = 16;
  // rows longer than one wave's share become split groups of their own
  const int64_t long_row = std::max<int64_t>(group_nnz / kGroupWaves, kSplitMinNnz);
  int64_t r = 0;
  while (r < n_rows) {
    const int64_t start = r;
    GroupDesc g{};
    g.nnz_base = static_cast<uint64_t>(rp[start]);
    if (rp[r + 1] - rp[r] > long_row) {
      if (rp[r + 1] - rp[r] >= kMaxRowNnz) fail(DOSE_ERR_UNSUPPORTED, "a row holds 2^28 or more entries");
      g.split = 1;
      g.row[0] = static_cast<uint32_t>(r);
      for (int w = 1; w <= kGroupWaves; ++w) g.row[w] = static_cast<uint32_t>(r + 1);
      for (int w = 0; w < kGroupWaves; ++w) g.ent[w] = static_cast<uint32_t>(rp[r + 1] - rp[r]);
      G.push_back(g);
      ++r;
      continue;
    }
    int64_t nnz = 0;
    while (r < n_rows && r - start < kMaxGroupRows) {
      const int64_t l = rp[r + 1] - rp[r];
      if (l > long_row || (r > start && (nnz + l > group_nnz || (brk && brk[r])))) break;
      nnz += l;
      ++r;
    }
    const int64_t total = nnz + kRowCost * (r - start);
    int64_t q = start;
    g.row[0] = static_cast<uint32_t>(start);
    for (int w = 1; w < kGroupWaves; ++w) {
      const int64_t target = total * w / kGroupWaves;
      while (q < r && (rp[q] - rp[start]) + kRowCost * (q - start) < target) ++q;
      g.row[w] = static_cast<uint32_t>(q);
    }
    g.row[kGroupWaves] = static_cast<uint32_t>(r);
    for (int w = 0; w < kGroupWaves; ++w) g.ent[w] = static_cast<uint32_t>(rp[g.row[w + 1]] - rp[start]);
    G.push_back(g);
  }
  return G;
}

// ------------------------------------------------------------- operands
// A row-group partition of one operand: the device descriptors of its groups
// (with their x windows), a host copy (batched plans copy it into their work
// lists) and what the launch needs to know about it.
struct Partition {
  DevBuf groups;
  std::vector<GroupDesc> h_groups;
  int32_t group_nnz = 0;
  int64_t n_groups = 0, n_windowed = 0, n_split = 0;
  int32_t win_floats[3] = {0, 0, 0};  // LDS window size for 1, 2 and 4 vectors
};

struct Operand {
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  std::vector<int64_t> h_row_ptr;
  DevBuf val, col, row_ptr;  // codes, column indices, offsets mod 2^32
  int idx_bytes = 4;         // column index width: 4 (int32) or 2 (uint16)
  Partition part;            // the partition plain products use
  std::vector<uint8_t> h_brk;  // rows that start a row group (A^T in slabs: each slab's first row), or empty
  std::vector<uint32_t> h_row_cbase;  // column of index 0 per row (A^T in slabs: its slab's first voxel), or empty

  uint64_t bytes() const { return val.bytes() + col.bytes() + row_ptr.bytes() + part.groups.bytes(); }
};

int rhs_slot(int n_rhs) { return n_rhs == 1 ? 0 : n_rhs == 2 ? 1 : 2; }

// Cap on one workgroup's LDS x window for one vector, in floats:
// DOSE_LDS_WINDOW_FLOATS (256 .. kWinFloatsMax), default 4096 (16 KB: eight
// workgroups per compute unit, and 99.8% of the clinical beam's groups fit);
// n vectors get n times the cap, up to kWinFloatsMax (row groups) or
// kSellWinFloatsMax (SELL-C-sigma chunks).  A smaller cap lets
// more workgroups share a compute unit; groups whose window exceeds it
// gather x from global memory.
int64_t window_cap_floats() {
  static const int64_t cap = [] {
    const char* e = std::getenv("DOSE_LDS_WINDOW_FLOATS");
    const int64_t v = e ? std::atoll(e) : 4096;
    return std::max<int64_t>(256, std::min<int64_t>(kWinFloatsMax, v));
  }();
  return cap;
}

// The partition of an operand into groups of about group_nnz entries, with
// every group's x window computed on the device.  Synchronous on s.
Partition make_partition(const Operand& op, int group_nnz, hipStream_t s) {
  std::vector<GroupDesc> G =
      build_partition(op.h_row_ptr.data(), op.n_rows, group_nnz, op.h_brk.empty() ? nullptr : op.h_brk.data());
  // a group's rows share one column base (groups never cross a slab)
  if (!op.h_row_cbase.empty())
    for (GroupDesc& g : G) g.cbase = op.h_row_cbase[g.row[0]];
  Partition P;
  P.groups = DevBuf(std::max<size_t>(1, G.size()) * sizeof(GroupDesc));
  if (!G.empty()) {
    HIP_CHECK(hipMemcpyAsync(P.groups.get(), G.data(), G.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s));
    HIP_CHECK(launch_group_windows(P.groups.get<GroupDesc>(), static_cast<int64_t>(G.size()), op.col.get(),
                                   op.idx_bytes, op.row_ptr.get<uint32_t>(), s));
    HIP_CHECK(hipMemcpyAsync(G.data(), P.groups.get(), G.size() * sizeof(GroupDesc), hipMemcpyDeviceToHost, s));
  }
  HIP_CHECK(hipStreamSynchronize(s));
  // LDS per workgroup: the largest window within the cap; groups with larger
  // windows read x from global memory
  const int64_t cap = window_cap_floats();
  int64_t windowed = 0, split = 0;
  int64_t wf[3] = {0, 0, 0};
  const int rhs[3] = {1, 2, 4};
  for (const GroupDesc& g : G) {
    windowed += g.clen > 0 && window_floats(g.clen, 1) <= cap;
    split += g.split;
    for (int i = 0; i < 3; ++i) {
      // the cap scales with the vectors: the same columns fit for 1, 2 and 4
      // (kernels for more vectors hold more registers and fewer workgroups
      // per compute unit, which leaves them the LDS)
      const int64_t f = window_floats(g.clen, rhs[i]);
      if (f <= std::min<int64_t>(cap * rhs[i], kWinFloatsMax)) wf[i] = std::max(wf[i], f);
    }
  }
  P.group_nnz = group_nnz;
  P.n_groups = static_cast<int64_t>(G.size());
  P.h_groups = std::move(G);
  P.n_windowed = windowed;
  P.n_split = split;
  for (int i = 0; i < 3; ++i) P.win_floats[i] = static_cast<int32_t>((wf[i] + 3) / 4 * 4);
  return P;
}

void upload_partition(Operand& op, int group_nnz, hipStream_t s) { op.part = make_partition(op, group_nnz, s); }

void upload_row_ptr32(Operand& op, hipStream_t s) {
  std::vector<uint32_t> rp32(op.h_row_ptr.size());
  for (size_t i = 0; i < rp32.size(); ++i) rp32[i] = static_cast<uint32_t>(op.h_row_ptr[i]);
  op.row_ptr = DevBuf(rp32.size() * sizeof(uint32_t));
  HIP_CHECK(hipMemcpyAsync(op.row_ptr.get(), rp32.data(), rp32.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
}

size_t padded(int64_t nnz) { return static_cast<size_t>(((nnz + kStreamPad + 63) / 64) * 64); }
int pad_entries(int64_t nnz) { return static_cast<int>(static_cast<int64_t>(padded(nnz)) - nnz); }

}  // namespace

struct dose_matrix_s {
  int device = 0;
  int vf = 0, xf = 0;
  bool has_t = false;
  Operand A, AT;
  DevBuf row_scale;  // E4M3: s_i per row of A
  // A^T in voxel slabs (slab > 0: slab width in voxels; AT's rows are the
  // (slab, spot) rows, padding rows included): spot j's rows are
  // comb_rows[comb_ptr[j] .. comb_ptr[j+1]), in ascending slab
  int32_t slab = 0;
  int64_t n_slab_rows = 0, n_slab_pad = 0;  // rows holding entries; padding entries
  DevBuf comb_ptr, comb_rows;
};

namespace {

int scale_mode_A(const dose_matrix_s* m) { return m->vf == kFp8 ? kScaleRow : kScaleNone; }
int scale_mode_AT(const dose_matrix_s* m) { return m->vf == kFp8 ? kScaleCol : kScaleNone; }

// Dies of the chip that workgroups are dealt to in turn (DOSE_XCD_BLOCKS):
// 8, the MI355X's eight XCDs, gives each die a contiguous run of the work
// items so that its L2 sees one part of x (and, for SELL-C-sigma, the rows
// one sigma window writes); 1 keeps the dispatch order.  Only the order in
// which work items are dispatched depends on it, never a result.  Measured:
// CSR products are faster without it (the largest workload's half/double
// product 1.648 ms against 1.690 ms, the clinical beam's adjoint 0.69 ms
// against 0.80 ms: default 1, and never on A^T), SELL-C-sigma products with
// it (the clinical beam, sigma 4096: 0.72 ms against 1.12 ms: default 8).
int xcd_blocks(int dflt) {
  static const int d = [] {
    const char* e = std::getenv("DOSE_XCD_BLOCKS");
    return e ? std::max(1, std::min(64, std::atoi(e))) : 0;
  }();
  return d > 0 ? d : dflt;
}

// n_rhs sizes the LDS window (an FP64 vector takes the window of two FP32 ones).
SpmvArgs make_args(const dose_matrix_s* m, const Operand& op, const Partition& P, int sm, int n_rhs, const void* x,
                   void* y) {
  SpmvArgs a{};
  a.win_floats = P.win_floats[rhs_slot(n_rhs)];
  a.groups = P.groups.get<GroupDesc>();
  a.val = op.val.get();
  a.col = op.col.get();
  a.idx_bytes = op.idx_bytes;
  a.row_ptr = op.row_ptr.get<uint32_t>();
  a.scale = sm == kScaleNone ? nullptr : m->row_scale.get<float>();
  a.x = x;
  a.y = y;
  a.n_groups = P.n_groups;
  a.xcd_blocks = &op == &m->AT && m->slab == 0 ? 1 : xcd_blocks(1);
  return a;
}
SpmvArgs make_args(const dose_matrix_s* m, const Operand& op, int sm, int n_rhs, const void* x, void* y) {
  return make_args(m, op, op.part, sm, n_rhs, x, y);
}

// Encode A's FP32 source values into its code stream, a row range at a time.
void encode_values(dose_matrix_s* m, const dose_csr_host* c, hipStream_t s) {
  Operand& A = m->A;
  if (A.nnz == 0 && m->vf != kFp8) return;
  int64_t max_row = 0;
  for (int64_t i = 0; i < A.n_rows; ++i) max_row = std::max(max_row, A.h_row_ptr[i + 1] - A.h_row_ptr[i]);
  const int64_t stage_n = std::max<int64_t>(std::max<int64_t>(std::min<int64_t>(A.nnz, int64_t{1} << 26), max_row), 1);
  DevBuf stage(static_cast<size_t>(stage_n) * sizeof(float));
  const int vb = value_bytes(m->vf);
  int64_t r0 = 0;
  while (r0 < A.n_rows) {
    // the longest run of rows from r0 that fits the staging buffer
    int64_t lo = r0 + 1, hi = A.n_rows;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (A.h_row_ptr[mid] - A.h_row_ptr[r0] <= stage_n) lo = mid; else hi = mid - 1;
    }
    const int64_t r1 = lo;
    const int64_t k0 = A.h_row_ptr[r0], k1 = A.h_row_ptr[r1];
    if (k1 > k0)
      HIP_CHECK(hipMemcpyAsync(stage.get(), c->values + k0, static_cast<size_t>(k1 - k0) * sizeof(float),
                               hipMemcpyHostToDevice, s));
    HIP_CHECK(launch_encode_rows(m->vf, A.row_ptr.get<uint32_t>() + r0, static_cast<uint32_t>(k0), r1 - r0,
                                 stage.get<float>(), static_cast<uint8_t*>(A.val.get()) + k0 * vb,
                                 m->vf == kFp8 ? m->row_scale.get<float>() + r0 : nullptr, s));
    HIP_CHECK(hipStreamSynchronize(s));  // the staging buffer is reused
    r0 = r1;
  }
}

// A^T on the device: stable radix sort of (column, entry) pairs, so every row
// of A^T lists its entries in ascending row of A.
void build_transpose(dose_matrix_s* m, int group_nnz_t, hipStream_t s) {
  const Operand& A = m->A;
  Operand& T = m->AT;
  if (A.nnz > INT32_MAX) fail(DOSE_ERR_UNSUPPORTED, "transpose needs nnz < 2^31");
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.nnz = A.nnz;
  const int vb = value_bytes(m->vf);
  T.val = DevBuf(padded(T.nnz) * vb);
  T.col = DevBuf(padded(T.nnz) * sizeof(int32_t));
  HIP_CHECK(hipMemsetAsync(T.val.get(), 0, T.val.bytes(), s));
  HIP_CHECK(hipMemsetAsync(T.col.get(), 0, T.col.bytes(), s));
  DevBuf rp64(static_cast<size_t>(T.n_rows + 1) * sizeof(int64_t));
  if (A.nnz > 0) {
    const int64_t n = A.nnz;
    DevBuf rows(static_cast<size_t>(n) * 4), keys_out(static_cast<size_t>(n) * 4), perm_in(static_cast<size_t>(n) * 4),
        perm_out(static_cast<size_t>(n) * 4);
    HIP_CHECK(launch_row_ids(A.row_ptr.get<uint32_t>(), A.n_rows, static_cast<uint64_t>(n), rows.get<uint32_t>(), s));
    HIP_CHECK(launch_iota(perm_in.get<uint32_t>(), n, s));
    int end_bit = 1;
    while (end_bit < 32 && (int64_t{1} << end_bit) < A.n_cols) ++end_bit;
    size_t tmp_bytes = 0;
    // sort keys: A's column indices as uint32
    DevBuf wide;
    const uint32_t* keys_in = reinterpret_cast<const uint32_t*>(A.col.get());
    if (A.idx_bytes == 2) {
      wide = DevBuf(static_cast<size_t>(n) * 4);
      HIP_CHECK(launch_widen_u16(A.col.get<uint16_t>(), wide.get<uint32_t>(), n, s));
      keys_in = wide.get<uint32_t>();
    }
    HIP_CHECK(radix_sort_pairs(nullptr, &tmp_bytes, keys_in,
                               keys_out.get<uint32_t>(), perm_in.get<uint32_t>(), perm_out.get<uint32_t>(), n, end_bit, s));
    DevBuf tmp(tmp_bytes);
    HIP_CHECK(radix_sort_pairs(tmp.get(), &tmp_bytes, keys_in,
                               keys_out.get<uint32_t>(), perm_in.get<uint32_t>(), perm_out.get<uint32_t>(), n, end_bit, s));
    HIP_CHECK(launch_gather_transpose(m->vf, perm_out.get<uint32_t>(), rows.get<uint32_t>(), A.val.get(), T.val.get(),
                                      T.col.get<int32_t>(), n, s));
    HIP_CHECK(launch_fill_pad(T.col.get(), 4, n, pad_entries(n), s));
    HIP_CHECK(launch_row_ptr_from_sorted(keys_out.get<uint32_t>(), n, T.n_rows, rp64.get<int64_t>(), s));
    HIP_CHECK(hipStreamSynchronize(s));
  } else {
    HIP_CHECK(hipMemsetAsync(rp64.get(), 0, rp64.bytes(), s));
  }
  T.h_row_ptr.resize(static_cast<size_t>(T.n_rows + 1));
  HIP_CHECK(hipMemcpyAsync(T.h_row_ptr.data(), rp64.get(), rp64.bytes(), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  upload_row_ptr32(T, s);
  upload_partition(T, group_nnz_t, s);
}

// Slab width of A^T in voxel slabs: the one-vector LDS window cap (so that
// every row group of a slab reads v from LDS), at most kWinFloatsMax / 2
// voxels so that an FP64 seed (two floats a voxel) stays windowed too.
int32_t slab_voxels() {
  const int64_t w = std::min<int64_t>(window_cap_floats(), kWinFloatsMax / 2);
  return static_cast<int32_t>(w / kWinAlign * kWinAlign);
}

// A^T in voxel slabs on the device: A's entries stably sorted by (slab of
// their voxel, spot), one row per distinct pair, entries in ascending voxel,
// each column stored as a 16-bit offset from its slab's first voxel (the
// groups' column base).  Each slab's entries are padded to a whole number of
// 4-entry quarters by a padding row of zero codes at the slab's first voxel,
// whose partial no spot combines: no quarter a row group loads then reaches
// into another slab, and (with the partition starting a group at every
// slab's first row) every group's window lies inside its slab.
void build_transpose_slabs(dose_matrix_s* m, int group_nnz_t, hipStream_t s) {
  const Operand& A = m->A;
  Operand& T = m->AT;
  const int64_t W = slab_voxels();
  const int64_t n_slabs = (A.n_rows + W - 1) / W;
  const int64_t nc = A.n_cols;
  if (n_slabs * nc > int64_t{UINT32_MAX})
    fail(DOSE_ERR_UNSUPPORTED, "slab transpose needs ceil(n_rows / slab) * n_cols < 2^32");
  if (A.nnz + (kQuarterEntries - 1) * n_slabs > INT32_MAX) fail(DOSE_ERR_UNSUPPORTED, "transpose needs nnz < 2^31");
  const int64_t n = A.nnz;
  std::vector<uint32_t> run_key, run_len;
  DevBuf rows, keys_out, perm_out;
  if (n > 0) {
    rows = DevBuf(static_cast<size_t>(n) * 4);
    keys_out = DevBuf(static_cast<size_t>(n) * 4);
    perm_out = DevBuf(static_cast<size_t>(n) * 4);
    DevBuf keys_in(static_cast<size_t>(n) * 4), perm_in(static_cast<size_t>(n) * 4);
    HIP_CHECK(launch_row_ids(A.row_ptr.get<uint32_t>(), A.n_rows, static_cast<uint64_t>(n), rows.get<uint32_t>(), s));
    DevBuf wide;
    const uint32_t* cols = reinterpret_cast<const uint32_t*>(A.col.get());
    if (A.idx_bytes == 2) {
      wide = DevBuf(static_cast<size_t>(n) * 4);
      HIP_CHECK(launch_widen_u16(A.col.get<uint16_t>(), wide.get<uint32_t>(), n, s));
      cols = wide.get<uint32_t>();
    }
    HIP_CHECK(launch_slab_keys(rows.get<uint32_t>(), cols, static_cast<uint32_t>(W), static_cast<uint32_t>(nc), n,
                               keys_in.get<uint32_t>(), s));
    HIP_CHECK(launch_iota(perm_in.get<uint32_t>(), n, s));
    int end_bit = 1;
    while (end_bit < 32 && (int64_t{1} << end_bit) < n_slabs * nc) ++end_bit;
    size_t tmp_bytes = 0;
    HIP_CHECK(radix_sort_pairs(nullptr, &tmp_bytes, keys_in.get<uint32_t>(), keys_out.get<uint32_t>(),
                               perm_in.get<uint32_t>(), perm_out.get<uint32_t>(), n, end_bit, s));
    {
      DevBuf tmp(tmp_bytes);
      HIP_CHECK(radix_sort_pairs(tmp.get(), &tmp_bytes, keys_in.get<uint32_t>(), keys_out.get<uint32_t>(),
                                 perm_in.get<uint32_t>(), perm_out.get<uint32_t>(), n, end_bit, s));
      HIP_CHECK(hipStreamSynchronize(s));
    }
    // the distinct (slab, spot) keys and their entry counts
    const int64_t max_runs = std::min<int64_t>(n, n_slabs * nc);
    DevBuf uniq(static_cast<size_t>(max_runs) * 4), cnt(static_cast<size_t>(max_runs) * 4), n_runs(4);
    size_t rle_bytes = 0;
    HIP_CHECK(run_length_encode(nullptr, &rle_bytes, keys_out.get<uint32_t>(), uniq.get<uint32_t>(),
                                cnt.get<uint32_t>(), n_runs.get<uint32_t>(), n, s));
    DevBuf rle_tmp(std::max<size_t>(rle_bytes, 1));
    HIP_CHECK(run_length_encode(rle_tmp.get(), &rle_bytes, keys_out.get<uint32_t>(), uniq.get<uint32_t>(),
                                cnt.get<uint32_t>(), n_runs.get<uint32_t>(), n, s));
    uint32_t h_runs = 0;
    HIP_CHECK(hipMemcpyAsync(&h_runs, n_runs.get(), 4, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (h_runs == 0 || h_runs > max_runs) fail(DOSE_ERR_INTERNAL, "slab transpose: bad run count");
    run_key.resize(h_runs);
    run_len.resize(h_runs);
    HIP_CHECK(hipMemcpyAsync(run_key.data(), uniq.get(), size_t{h_runs} * 4, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(run_len.data(), cnt.get(), size_t{h_runs} * 4, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  }
  // rows of the slab form (host): offsets, slab starts, padding, and the
  // spot each row belongs to
  std::vector<int64_t>& rp = T.h_row_ptr;
  std::vector<uint8_t>& brk = T.h_brk;
  rp.assign(1, 0);
  brk.clear();
  std::vector<uint32_t> slab_off(static_cast<size_t>(std::max<int64_t>(n_slabs, 1)), 0), row_spot;
  std::vector<uint32_t>& cbase = T.h_row_cbase;
  cbase.clear();
  int64_t pads = 0;
  for (size_t i = 0; i < run_key.size();) {
    const uint32_t t = run_key[i] / static_cast<uint32_t>(nc);
    slab_off[t] = static_cast<uint32_t>(pads);
    int64_t tot = 0;
    for (bool first = true; i < run_key.size() && run_key[i] / static_cast<uint32_t>(nc) == t; ++i, first = false) {
      brk.push_back(first ? 1 : 0);
      rp.push_back(rp.back() + run_len[i]);
      row_spot.push_back(run_key[i] % static_cast<uint32_t>(nc));
      cbase.push_back(static_cast<uint32_t>(t * W));
      tot += run_len[i];
    }
    // the padding entries keep the zero codes and zero offsets (the slab's
    // first voxel) of the cleared streams
    const int64_t p = (kQuarterEntries - tot % kQuarterEntries) % kQuarterEntries;
    if (p > 0) {
      brk.push_back(0);
      rp.push_back(rp.back() + p);
      row_spot.push_back(UINT32_MAX);
      cbase.push_back(static_cast<uint32_t>(t * W));
      pads += p;
    }
  }
  T.n_rows = static_cast<int64_t>(rp.size()) - 1;
  T.n_cols = A.n_rows;
  T.nnz = n + pads;
  m->slab = static_cast<int32_t>(W);
  m->n_slab_pad = pads;
  m->n_slab_rows = T.n_rows - static_cast<int64_t>(std::count(row_spot.begin(), row_spot.end(), UINT32_MAX));
  // spot j's rows in ascending slab (rows are in ascending slab)
  std::vector<uint32_t> cptr(static_cast<size_t>(nc) + 1, 0), crows(static_cast<size_t>(std::max<int64_t>(m->n_slab_rows, 1)));
  for (uint32_t j : row_spot)
    if (j != UINT32_MAX) ++cptr[j + 1];
  for (int64_t j = 0; j < nc; ++j) cptr[j + 1] += cptr[j];
  {
    std::vector<uint32_t> fill(cptr.begin(), cptr.end() - 1);
    for (size_t r = 0; r < row_spot.size(); ++r)
      if (row_spot[r] != UINT32_MAX) crows[fill[row_spot[r]]++] = static_cast<uint32_t>(r);
  }
  const int vb = value_bytes(m->vf);
  T.val = DevBuf(padded(T.nnz) * vb);
  T.col = DevBuf(padded(T.nnz) * sizeof(uint16_t));
  T.idx_bytes = 2;
  HIP_CHECK(hipMemsetAsync(T.val.get(), 0, T.val.bytes(), s));
  HIP_CHECK(hipMemsetAsync(T.col.get(), 0, T.col.bytes(), s));
  DevBuf d_off;
  if (n > 0) {
    d_off = DevBuf(slab_off.size() * 4);
    HIP_CHECK(hipMemcpyAsync(d_off.get(), slab_off.data(), slab_off.size() * 4, hipMemcpyHostToDevice, s));
    HIP_CHECK(launch_slab_gather(m->vf, perm_out.get<uint32_t>(), rows.get<uint32_t>(), keys_out.get<uint32_t>(),
                                 static_cast<uint32_t>(nc), static_cast<uint32_t>(W), d_off.get<uint32_t>(),
                                 A.val.get(), T.val.get(), T.col.get<uint16_t>(), n, s));
  }
  HIP_CHECK(launch_fill_pad(T.col.get(), 2, T.nnz, pad_entries(T.nnz), s));
  m->comb_ptr = DevBuf(cptr.size() * 4);
  m->comb_rows = DevBuf(crows.size() * 4);
  HIP_CHECK(hipMemcpyAsync(m->comb_ptr.get(), cptr.data(), cptr.size() * 4, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpyAsync(m->comb_rows.get(), crows.data(), crows.size() * 4, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
  upload_row_ptr32(T, s);
  upload_partition(T, group_nnz_t, s);
}

void check_group_nnz(int32_t g) {
  if (!is_pow2(g) || g < kMinGroupNnz || g > kMaxGroupNnz)
    fail(DOSE_ERR_INVALID_ARGUMENT, "group_nnz must be a power of two in [1024, 2^20]");
}

// Default row-group size: large enough that staging a group's x window is a
// small fraction of its stream, small enough for many groups per compute
// unit.  32K entries when the launch runs at least 24 rounds of resident
// workgroups (eight per compute unit), so that the last, partial round costs
// little; 16K otherwise; halved, down to 1K, for matrices with fewer groups
// than resident workgroups (a cache-resident matrix of 806K entries: 7.6 us
// per product with 1K groups, 13.1 us with 4K).
int default_group_nnz(int64_t nnz, int device) {
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
  const int64_t resident = int64_t{cus} * 8;
  int g = nnz / 32768 >= 24 * resident ? 32768 : 16384;
  while (g > kMinGroupNnz && nnz / g < resident) g >>= 1;
  return g;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return na > 0 && nb > 0 && pa < pb + nb && pb < pa + na;
}

void run_product(const dose_matrix_s* m, const Operand& op, int sm, int n_rhs, const float* x, float* y,
                 hipStream_t s) {
  HIP_CHECK(launch_spmv(m->vf, sm, n_rhs, make_args(m, op, sm, n_rhs, x, y), s));
}

// ------------------------------------------------------------ tuning cache
std::mutex g_tune_mu;

std::string tune_key(const dose_matrix_s* m, const Operand& op, int n_rhs) {
  std::ostringstream k;
  k << "v2:" << op.n_rows << "x" << op.n_cols << ":" << op.nnz << ":f" << m->vf << ":r" << n_rhs;
  return k.str();
}

int tune_lookup(const std::string& key) {
  const char* path = std::getenv("DOSE_TUNE_CACHE");
  if (!path) return 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::ifstream f(path);
  std::string k;
  int v = 0, found = 0;
  while (f >> k >> v)
    if (k == key) found = v;
  return found;
}

void tune_store(const std::string& key, int v) {
  const char* path = std::getenv("DOSE_TUNE_CACHE");
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::ofstream f(path, std::ios::app);
  f << key << " " << v << "\n";
}

}  // namespace

// ------------------------------------------------------------ batch plans
// One launch of a plan: the arguments of its items and the groups of all of
// them (a work list of descriptor copies naming their item).
struct PlanLayer {
  int lds_floats = 0;
  int accumulate = 0;  // 1: the launch adds its items' products to what their y hold
  int64_t n_work = 0;
  DevBuf args, work;
};

// The launch of a SELL-C-sigma plan: its items' arguments and (item, chunk)
// work lists.
struct SellPlanLayer {
  int64_t n_work = 0, n_zero = 0;
  size_t lds_bytes = 0;
  int xcd = 1;
  DevBuf args, work, zero;
};

// Adjoint plans: an item's E4M3 seed scaling (u = fl32(s v)) before the
// launch, and its slab combine (g from the slab rows' partials) after it.
struct PlanScale {
  int64_t n = 0;
  const float *scale = nullptr, *v = nullptr;
  float* u = nullptr;
};
struct PlanCombine {
  const float* part = nullptr;
  const uint32_t *ptr = nullptr, *rows = nullptr;
  float* g = nullptr;
  int64_t n_cols = 0;
};

struct dose_batch_plan_s {
  int device = 0;
  int vf = 0, sm = 0, n_rhs = 0, idx_bytes = 4;
  std::vector<PlanScale> pre;     // adjoint plans: seed scaling before the layers
  DevBuf pre_items;               // the same as one table (one launch for all of them)
  int64_t pre_max_n = 0;
  std::vector<PlanLayer> layers;  // launched one after another (one layer for a batch plan)
  std::vector<SellPlanLayer> sell_layers;  // a SELL-C-sigma plan's launch (then layers is empty)
  std::vector<PlanCombine> post;  // adjoint plans: slab combines after the layers
  DevBuf post_groups, post_items;  // the same as output groups and items (one launch for all of them)
  int32_t n_post_groups = 0;
  int64_t post_max_cols = 0;
  DevBuf scratch;                 // adjoint plans: the scaled seeds and slab partials
  std::vector<std::unique_ptr<Partition>> parts;  // autotuned partitions the work lists were built from
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~dose_batch_plan_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

void check_items(const dose_batch_item* items, int32_t n_items) {
  if (!items || n_items <= 0) fail(DOSE_ERR_INVALID_ARGUMENT, "no items");
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_batch_item& it = items[i];
    if (!it.A) fail(DOSE_ERR_INVALID_ARGUMENT, "item without matrix");
    if (it.n_rhs != 1 && it.n_rhs != 2 && it.n_rhs != 4) fail(DOSE_ERR_UNSUPPORTED, "n_rhs must be 1, 2 or 4");
    if (it.ldx != it.n_rhs || it.ldy != it.n_rhs) fail(DOSE_ERR_UNSUPPORTED, "ldx and ldy must equal n_rhs");
    if ((it.A->A.n_cols > 0 && !it.x) || (it.A->A.n_rows > 0 && !it.y)) fail(DOSE_ERR_INVALID_ARGUMENT, "null x or y");
    if (it.A->vf != items[0].A->vf) fail(DOSE_ERR_UNSUPPORTED, "items mix value formats");
    if (it.A->A.idx_bytes != items[0].A->A.idx_bytes) fail(DOSE_ERR_UNSUPPORTED, "items mix index formats");
    if (it.n_rhs != items[0].n_rhs) fail(DOSE_ERR_UNSUPPORTED, "items mix n_rhs");
    if (it.A->device != items[0].A->device) fail(DOSE_ERR_INVALID_ARGUMENT, "items on different devices");
    if (overlaps(it.x, it.A->A.n_cols * it.n_rhs * 4, it.y, it.A->A.n_rows * it.n_rhs * 4))
      fail(DOSE_ERR_INVALID_ARGUMENT, "x and y overlap");
    if ((reinterpret_cast<uintptr_t>(it.x) | reinterpret_cast<uintptr_t>(it.y)) % (4 * it.n_rhs) != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "x and y must be aligned to n_rhs floats");
    for (int32_t j = 0; j < i; ++j)
      if (overlaps(items[j].y, items[j].A->A.n_rows * items[j].n_rhs * 4, it.y, it.A->A.n_rows * it.n_rhs * 4))
        fail(DOSE_ERR_INVALID_ARGUMENT, "items share outputs");
  }
}

// Median time of the plain product of one operand under partition P.
double time_partition(dose_matrix_s* m, const Operand& op, const Partition& P, int sm, int n_rhs, const float* x,
                      float* y, hipStream_t s) {
  const SpmvArgs a = make_args(m, op, P, sm, n_rhs, x, y);
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  std::vector<float> ts;
  for (int rep = 0; rep < 7; ++rep) {
    HIP_CHECK(hipEventRecord(e0, s));
    HIP_CHECK(launch_spmv(m->vf, sm, n_rhs, a, s));
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0) ts.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(ts.begin(), ts.end());
  return ts[ts.size() / 2];
}

// The fastest row-group size for a matrix's products with n_rhs vectors,
// found by timing candidate partitions built for this purpose (the result
// does not depend on the partition: every row is summed in the same order
// under any of them).  The matrix itself is left as it is, so products on
// other streams may use it meanwhile.  Returns the chosen partition, or null
// when the matrix's own partition already has the chosen size.
std::unique_ptr<Partition> autotune_operand(dose_matrix_s* m, const Operand& op, int sm, int n_rhs, const float* x,
                                            float* y, hipStream_t s) {
  const std::string key = tune_key(m, op, n_rhs);
  int best = tune_lookup(key);
  std::unique_ptr<Partition> best_p;
  if (best == 0) {
    double best_t = 1e30;
    for (int g = 8192; g <= 65536; g *= 2) {
      auto P = std::make_unique<Partition>(make_partition(op, g, s));
      const double t = time_partition(m, op, *P, sm, n_rhs, x, y, s);
      if (t < best_t) best_t = t, best = g, best_p = std::move(P);
    }
    tune_store(key, best);
  }
  if (op.part.group_nnz == best) return nullptr;
  if (!best_p) best_p = std::make_unique<Partition>(make_partition(op, best, s));
  return best_p;
}

std::unique_ptr<Partition> autotune_matrix(dose_matrix_s* m, int n_rhs, const float* x, float* y, hipStream_t s) {
  return autotune_operand(m, m->A, scale_mode_A(m), n_rhs, x, y, s);
}

// The partition each distinct matrix of the items runs under in a plan: its
// own, or with DOSE_PLAN_AUTOTUNE a tuned copy the plan keeps.
std::map<const dose_matrix_s*, const Partition*> plan_partitions(dose_batch_plan_s* plan,
                                                                 const dose_batch_item* items, int32_t n_items,
                                                                 uint32_t flags, hipStream_t s) {
  std::map<const dose_matrix_s*, const Partition*> part_of;
  for (int32_t i = 0; i < n_items; ++i) {
    dose_matrix_s* m = items[i].A;
    if (part_of.count(m)) continue;
    const Partition* P = &m->A.part;
    if (flags & DOSE_PLAN_AUTOTUNE) {
      std::unique_ptr<Partition> tuned = autotune_matrix(m, items[i].n_rhs, items[i].x, items[i].y, s);
      if (tuned) {
        P = tuned.get();
        plan->parts.push_back(std::move(tuned));
      }
    }
    part_of[m] = P;
  }
  return part_of;
}

// One launch over the groups of all items; with accumulate, each item's
// products are added to what its y holds.
PlanLayer make_layer(const dose_batch_plan_s* plan, const dose_batch_item* items, int32_t n_items,
                     const std::map<const dose_matrix_s*, const Partition*>& part_of, int accumulate,
                     hipStream_t s) {
  PlanLayer L;
  L.accumulate = accumulate;
  std::vector<SpmvArgs> args(static_cast<size_t>(n_items));
  std::vector<GroupDesc> work;
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_matrix_s* m = items[i].A;
    const Partition& P = *part_of.at(m);
    args[i] = make_args(m, m->A, P, plan->sm, plan->n_rhs, items[i].x, items[i].y);
    L.lds_floats = std::max(L.lds_floats, args[i].win_floats);
    for (GroupDesc g : P.h_groups) {
      g.item = static_cast<uint32_t>(i);
      work.push_back(g);
    }
  }
  L.n_work = static_cast<int64_t>(work.size());
  if (L.n_work > int64_t{0x7fffffff}) fail(DOSE_ERR_UNSUPPORTED, "too many row groups for one launch");
  L.args = DevBuf(args.size() * sizeof(SpmvArgs));
  L.work = DevBuf(std::max<size_t>(1, work.size()) * sizeof(GroupDesc));
  HIP_CHECK(hipMemcpyAsync(L.args.get(), args.data(), args.size() * sizeof(SpmvArgs), hipMemcpyHostToDevice, s));
  if (!work.empty())
    HIP_CHECK(hipMemcpyAsync(L.work.get(), work.data(), work.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return L;
}

std::unique_ptr<dose_batch_plan_s> new_plan(const dose_batch_item* items) {
  auto plan = std::make_unique<dose_batch_plan_s>();
  const dose_matrix_s* m0 = items[0].A;
  plan->device = m0->device;
  plan->vf = m0->vf;
  plan->sm = scale_mode_A(m0);
  plan->n_rhs = items[0].n_rhs;
  plan->idx_bytes = m0->A.idx_bytes;
  return plan;
}

dose_batch_plan_s* build_plan(const dose_batch_item* items, int32_t n_items, uint32_t flags, hipStream_t s) {
  check_items(items, n_items);
  auto plan = new_plan(items);
  const auto part_of = plan_partitions(plan.get(), items, n_items, flags, s);
  plan->layers.push_back(make_layer(plan.get(), items, n_items, part_of, 0, s));
  return plan.release();
}

void enqueue_plan(const dose_batch_plan_s* p, hipStream_t s) {
  if (p->pre_items.get())
    HIP_CHECK(launch_scale_items(p->pre_items.get<ScaleItem>(), static_cast<int32_t>(p->pre.size()), p->pre_max_n, s));
  else
    for (const PlanScale& c : p->pre) HIP_CHECK(launch_scale_vec(c.n, c.scale, c.v, c.u, s));
  for (const PlanLayer& L : p->layers) {
    BatchTable t{};
    t.args = L.args.get<SpmvArgs>();
    t.work = L.work.get<GroupDesc>();
    HIP_CHECK(launch_spmv_batched(p->vf, p->sm, p->n_rhs, L.accumulate, p->idx_bytes, t, L.n_work, L.lds_floats, s));
  }
  for (const SellPlanLayer& L : p->sell_layers) {
    SellBatchTable t{};
    t.args = L.args.get<SellArgs>();
    t.work = L.work.get<uint2>();
    t.zero = L.zero.get<uint2>();
    t.n_work = L.n_work;
    t.n_zero = L.n_zero;
    t.xcd_blocks = L.xcd;
    HIP_CHECK(launch_sell_batched(p->vf, p->sm, p->n_rhs, p->idx_bytes, t, L.lds_bytes, s));
  }
  if (p->post_groups.get())
    HIP_CHECK(launch_slab_combine_groups(p->post_groups.get<SlabCombineGroup>(), p->n_post_groups,
                                         p->post_items.get<SlabCombineItem>(), p->post_max_cols, s));
  else
    for (const PlanCombine& c : p->post)
      HIP_CHECK(launch_slab_combine(false, c.part, c.ptr, c.rows, c.g, c.n_cols, s));
}

// The adjoint items of a plan: every matrix with a transpose of the same
// layout (spot rows or voxel slabs), value format and device; v and g of an
// item apart, no g overlapping another item's v, and no g shared or
// overlapping another item's g, except (accumulate, voxel slabs) the very
// same g of items with as many spots.  v may be shared.
void check_adjoint_items(const dose_adjoint_item* items, int32_t n_items, bool accumulate) {
  if (!items || n_items <= 0) fail(DOSE_ERR_INVALID_ARGUMENT, "no items");
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_adjoint_item& it = items[i];
    const dose_matrix_s* m = it.A;
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "item without matrix");
    if (it.reserved != 0) fail(DOSE_ERR_INVALID_ARGUMENT, "reserved must be 0");
    if (!m->has_t) fail(DOSE_ERR_NO_TRANSPOSE, "item matrix was created without a transpose");
    if ((m->A.n_rows > 0 && !it.v) || (m->A.n_cols > 0 && !it.g)) fail(DOSE_ERR_INVALID_ARGUMENT, "null v or g");
    if ((reinterpret_cast<uintptr_t>(it.v) | reinterpret_cast<uintptr_t>(it.g)) % 4 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "v and g must be 4-byte aligned");
    if (overlaps(it.v, m->A.n_rows * 4, it.g, m->A.n_cols * 4)) fail(DOSE_ERR_INVALID_ARGUMENT, "v and g overlap");
    const dose_matrix_s* m0 = items[0].A;
    if (m->vf != m0->vf) fail(DOSE_ERR_UNSUPPORTED, "items mix value formats");
    if ((m->slab > 0) != (m0->slab > 0) || m->AT.idx_bytes != m0->AT.idx_bytes)
      fail(DOSE_ERR_UNSUPPORTED, "items mix transpose layouts");
    if (m->device != m0->device) fail(DOSE_ERR_INVALID_ARGUMENT, "items on different devices");
    if (accumulate && m->slab == 0) fail(DOSE_ERR_UNSUPPORTED, "accumulating adjoint plans need voxel slabs");
    for (int32_t j = 0; j < i; ++j) {
      const bool same = accumulate && items[j].g == it.g && items[j].A->A.n_cols == m->A.n_cols;
      if (!same && overlaps(items[j].g, items[j].A->A.n_cols * 4, it.g, m->A.n_cols * 4))
        fail(DOSE_ERR_INVALID_ARGUMENT, "items share outputs");
      if (overlaps(items[j].v, items[j].A->A.n_rows * 4, it.g, m->A.n_cols * 4) ||
          overlaps(it.v, m->A.n_rows * 4, items[j].g, items[j].A->A.n_cols * 4))
        fail(DOSE_ERR_INVALID_ARGUMENT, "an item's g overlaps another item's v");
    }
  }
}

// The adjoints of all items: E4M3 seeds scaled into the plan's scratch, one
// batched launch over the row groups of every item's transpose (writing g,
// or the slab partials into the scratch), then the slab combines (one output
// group per g: with DOSE_ADJOINT_ACCUMULATE, every item writing it).  The row
// groups are sized for the whole launch (a matrix's own are sized to fill the
// chip alone): plan-owned partitions where the sizes differ, the results
// not depending on the partition; with DOSE_PLAN_AUTOTUNE the launch is
// timed under 8K-64K-entry groups and the fastest kept.
dose_batch_plan_s* build_adjoint_plan(const dose_adjoint_item* items, int32_t n_items, uint32_t flags,
                                      hipStream_t s) {
  const bool accumulate = (flags & DOSE_ADJOINT_ACCUMULATE) != 0;
  check_adjoint_items(items, n_items, accumulate);
  auto plan = std::make_unique<dose_batch_plan_s>();
  const dose_matrix_s* m0 = items[0].A;
  const bool fp8 = m0->vf == kFp8, slabs = m0->slab > 0;
  plan->device = m0->device;
  plan->vf = m0->vf;
  plan->sm = fp8 ? kScaleNone : scale_mode_AT(m0);
  plan->n_rhs = 1;
  plan->idx_bytes = m0->AT.idx_bytes;
  // scratch: per item, u (E4M3) then the partials (slabs), each 16-byte aligned
  auto up4 = [](int64_t n) { return (n + 3) / 4 * 4; };
  std::vector<int64_t> off_u(static_cast<size_t>(n_items)), off_p(static_cast<size_t>(n_items));
  int64_t total = 0, nnz_all = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_matrix_s* m = items[i].A;
    off_u[i] = total;
    if (fp8) total += up4(m->A.n_rows);
    off_p[i] = total;
    if (slabs) total += up4(m->AT.n_rows);
    nnz_all += m->AT.nnz;
  }
  if (total > 0) plan->scratch = DevBuf(static_cast<size_t>(total) * 4);
  float* sc = plan->scratch.get<float>();
  // each item's product input and output, its seed scaling and its combine
  std::vector<const float*> xs(static_cast<size_t>(n_items));
  std::vector<float*> ys(static_cast<size_t>(n_items));
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_adjoint_item& it = items[i];
    const dose_matrix_s* m = it.A;
    xs[i] = it.v;
    if (fp8 && m->A.n_rows > 0) {
      PlanScale c;
      c.n = m->A.n_rows, c.scale = m->row_scale.get<float>(), c.v = it.v, c.u = sc + off_u[i];
      plan->pre.push_back(c);
      xs[i] = c.u;
    }
    ys[i] = slabs ? sc + off_p[i] : it.g;
    if (slabs && m->A.n_cols > 0) {
      PlanCombine c;
      c.part = ys[i], c.ptr = m->comb_ptr.get<uint32_t>(), c.rows = m->comb_rows.get<uint32_t>(), c.g = it.g;
      c.n_cols = m->A.n_cols;
      plan->post.push_back(c);
    }
  }
  // the launch under row groups of about g entries (partitions the plan owns
  // go to `parts`)
  auto layer_for = [&](int g, std::vector<std::unique_ptr<Partition>>& parts) {
    std::map<const dose_matrix_s*, const Partition*> part_of;
    PlanLayer L;
    std::vector<SpmvArgs> args(static_cast<size_t>(n_items));
    std::vector<GroupDesc> work;
    for (int32_t i = 0; i < n_items; ++i) {
      const dose_matrix_s* m = items[i].A;
      if (!part_of.count(m)) {
        const Partition* P = &m->AT.part;
        if (P->group_nnz != g && m->AT.nnz > 0) {
          parts.push_back(std::make_unique<Partition>(make_partition(m->AT, g, s)));
          P = parts.back().get();
        }
        part_of[m] = P;
      }
      const Partition& P = *part_of.at(m);
      args[i] = make_args(m, m->AT, P, plan->sm, 1, xs[i], ys[i]);
      L.lds_floats = std::max(L.lds_floats, args[i].win_floats);
      for (GroupDesc gd : P.h_groups) {
        gd.item = static_cast<uint32_t>(i);
        work.push_back(gd);
      }
    }
    L.n_work = static_cast<int64_t>(work.size());
    if (L.n_work > int64_t{0x7fffffff}) fail(DOSE_ERR_UNSUPPORTED, "too many row groups for one launch");
    L.args = DevBuf(args.size() * sizeof(SpmvArgs));
    L.work = DevBuf(std::max<size_t>(1, work.size()) * sizeof(GroupDesc));
    HIP_CHECK(hipMemcpyAsync(L.args.get(), args.data(), args.size() * sizeof(SpmvArgs), hipMemcpyHostToDevice, s));
    if (!work.empty())
      HIP_CHECK(hipMemcpyAsync(L.work.get(), work.data(), work.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return L;
  };
  if (!(flags & DOSE_PLAN_AUTOTUNE)) {
    plan->layers.push_back(layer_for(default_group_nnz(nnz_all, plan->device), plan->parts));
  } else {
    // median of 6 timed launches after one untimed, per candidate size
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    double best_t = 1e30;
    for (int g = 8192; g <= 65536; g *= 2) {
      std::vector<std::unique_ptr<Partition>> parts;
      PlanLayer L = layer_for(g, parts);
      BatchTable t{};
      t.args = L.args.get<SpmvArgs>();
      t.work = L.work.get<GroupDesc>();
      std::vector<float> ts;
      for (int rep = 0; rep < 7; ++rep) {
        HIP_CHECK(hipEventRecord(e0, s));
        HIP_CHECK(launch_spmv_batched(plan->vf, plan->sm, 1, 0, plan->idx_bytes, t, L.n_work, L.lds_floats, s));
        HIP_CHECK(hipEventRecord(e1, s));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) ts.push_back(ms);
      }
      std::sort(ts.begin(), ts.end());
      const double t_med = ts[ts.size() / 2];
      if (t_med < best_t) {
        best_t = t_med;
        plan->layers.clear();
        plan->layers.push_back(std::move(L));
        plan->parts = std::move(parts);
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  // the seed scalings, and the combines, in one launch each (the kernels
  // take up to 65,535 items)
  if (!plan->pre.empty() && plan->pre.size() <= 65535) {
    std::vector<ScaleItem> si;
    for (const PlanScale& c : plan->pre) {
      si.push_back(ScaleItem{c.scale, c.v, c.u, c.n});
      plan->pre_max_n = std::max(plan->pre_max_n, c.n);
    }
    plan->pre_items = DevBuf(si.size() * sizeof(ScaleItem));
    HIP_CHECK(hipMemcpyAsync(plan->pre_items.get(), si.data(), si.size() * sizeof(ScaleItem), hipMemcpyHostToDevice,
                             s));
  }
  // the combines as output groups: the items writing one g, in item order
  // (one item per group unless accumulating)
  std::vector<SlabCombineGroup> cg;
  std::vector<SlabCombineItem> ci;
  {
    std::map<float*, std::vector<size_t>> by_g;
    std::vector<float*> order;
    for (size_t k = 0; k < plan->post.size(); ++k) {
      float* g = plan->post[k].g;
      if (!accumulate || !by_g.count(g)) order.push_back(g);
      by_g[g].push_back(k);
    }
    for (size_t q = 0; q < order.size(); ++q) {
      // without accumulate every g is distinct, so each group is one item
      const std::vector<size_t>& ks = by_g.at(order[q]);
      SlabCombineGroup G{order[q], plan->post[ks[0]].n_cols, static_cast<int32_t>(ci.size()),
                         static_cast<int32_t>(ks.size())};
      for (size_t k : ks) ci.push_back(SlabCombineItem{plan->post[k].part, plan->post[k].ptr, plan->post[k].rows});
      cg.push_back(G);
      plan->post_max_cols = std::max(plan->post_max_cols, G.n_cols);
    }
  }
  if (!cg.empty() && cg.size() <= 65535) {
    plan->n_post_groups = static_cast<int32_t>(cg.size());
    plan->post_groups = DevBuf(cg.size() * sizeof(SlabCombineGroup));
    plan->post_items = DevBuf(ci.size() * sizeof(SlabCombineItem));
    HIP_CHECK(hipMemcpyAsync(plan->post_groups.get(), cg.data(), cg.size() * sizeof(SlabCombineGroup),
                             hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(plan->post_items.get(), ci.data(), ci.size() * sizeof(SlabCombineItem),
                             hipMemcpyHostToDevice, s));
  } else if (accumulate && !cg.empty()) {
    fail(DOSE_ERR_UNSUPPORTED, "an accumulating adjoint plan takes at most 65,535 outputs");
  }
  HIP_CHECK(hipStreamSynchronize(s));
  return plan.release();
}

// Captures a built plan's launches into its HIP graph.
void capture_plan(dose_batch_plan_s* p) {
  hipStream_t cap;
  HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    try {
      enqueue_plan(p, cap);
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(cap, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      (void)hipStreamDestroy(cap);
      throw;
    }
    e = hipStreamEndCapture(cap, &p->graph);
  }
  (void)hipStreamDestroy(cap);
  HIP_CHECK(e);
  HIP_CHECK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
}

// ------------------------------------------------- item tables of batched calls
// dose_spmv_batched hands its items' arguments to the kernel through a table
// in device memory: the first workgroup of every item (n_items + 1 ascending
// entries, the last one the total) followed by the items' SpmvArgs, each
// naming the matrix's own row groups.  The table is written into a slot of a
// pinned host ring and copied to the same slot of a device ring on the
// caller's stream, so the call returns without waiting for the GPU; an event
// recorded after the launch keeps a slot from being reused before its launch
// has finished.  One ring per device, kept until the process ends.
constexpr int kRingSlots = 16;
constexpr size_t kRingSlotBytes = size_t{256} << 10;
constexpr int32_t kMaxCallItems = 2048;
static_assert((kMaxCallItems + 1) * sizeof(uint32_t) + 16 + kMaxCallItems * sizeof(SpmvArgs) <= kRingSlotBytes,
              "a slot holds the table of the largest call");

struct ItemRing {
  std::mutex mu;
  char* host = nullptr;  // pinned
  char* dev = nullptr;
  hipEvent_t done[kRingSlots] = {};
  uint64_t next = 0;
};

std::mutex g_ring_mu;
std::map<int, std::unique_ptr<ItemRing>> g_rings;

ItemRing& ring_for(int device) {
  std::lock_guard<std::mutex> lk(g_ring_mu);
  auto& r = g_rings[device];
  if (!r) {
    auto nr = std::make_unique<ItemRing>();
    const size_t bytes = kRingSlots * kRingSlotBytes;
    if (hipHostMalloc(reinterpret_cast<void**>(&nr->host), bytes, hipHostMallocDefault) != hipSuccess)
      fail(DOSE_ERR_OUT_OF_MEMORY, "pinned item ring");
    try {
      nr->dev = static_cast<char*>(dev_alloc(bytes));
      for (auto& e : nr->done) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    } catch (...) {
      (void)hipHostFree(nr->host);
      if (nr->dev) (void)hipFree(nr->dev);
      throw;
    }
    r = std::move(nr);
  }
  return *r;
}

void launch_items(const dose_batch_item* items, int32_t n_items, hipStream_t s) {
  if (n_items > kMaxCallItems)
    fail(DOSE_ERR_UNSUPPORTED, "more than " + std::to_string(kMaxCallItems) + " items in one call (use a batch plan)");
  const dose_matrix_s* m0 = items[0].A;
  const int sm = scale_mode_A(m0), n_rhs = items[0].n_rhs;
  // table layout: first[n_items + 1] (u32), padded to 16 bytes, then the args
  const size_t args_off = (static_cast<size_t>(n_items + 1) * sizeof(uint32_t) + 15) / 16 * 16;
  const size_t bytes = args_off + static_cast<size_t>(n_items) * sizeof(SpmvArgs);
  std::vector<uint32_t> first(static_cast<size_t>(n_items) + 1);
  std::vector<SpmvArgs> args(static_cast<size_t>(n_items));
  int64_t total = 0;
  int lds = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_matrix_s* m = items[i].A;
    first[i] = static_cast<uint32_t>(total);
    args[i] = make_args(m, m->A, sm, n_rhs, items[i].x, items[i].y);
    lds = std::max(lds, args[i].win_floats);
    total += m->A.part.n_groups;
    if (total > int64_t{0x7fffffff}) fail(DOSE_ERR_UNSUPPORTED, "too many row groups for one launch");
  }
  first[n_items] = static_cast<uint32_t>(total);
  if (total == 0) return;
  ItemRing& R = ring_for(m0->device);
  std::lock_guard<std::mutex> lk(R.mu);
  const int slot = static_cast<int>(R.next++ % kRingSlots);
  HIP_CHECK(hipEventSynchronize(R.done[slot]));  // the slot's previous launch has finished
  char* h = R.host + slot * kRingSlotBytes;
  char* d = R.dev + slot * kRingSlotBytes;
  std::memcpy(h, first.data(), first.size() * sizeof(uint32_t));
  std::memcpy(h + args_off, args.data(), args.size() * sizeof(SpmvArgs));
  HIP_CHECK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  BatchTable t{};
  t.args = reinterpret_cast<const SpmvArgs*>(d + args_off);
  t.first = reinterpret_cast<const uint32_t*>(d);
  t.n_items = n_items;
  const hipError_t e = launch_spmv_batched(m0->vf, sm, n_rhs, 0, m0->A.idx_bytes, t, total, lds, s);
  // recorded even when the launch failed, so that the slot is free again
  const hipError_t er = hipEventRecord(R.done[slot], s);
  HIP_CHECK(e);
  HIP_CHECK(er);
}

constexpr int32_t kMaxScenarios = 65536;  // also the limit on beams per scenario

// Argument checks of the scenario epilogue (both entry points).
void check_scenario_args(int32_t n_scen, int32_t n_beams, int64_t n, const float* part, const float* p, const float* w,
                         const double* prob, const float* d_out, const float* seed, const double* out) {
  if (n_scen < 1 || n_scen > kMaxScenarios || n_beams < 1 || n_beams > kMaxScenarios || n < 0 || !out)
    fail(DOSE_ERR_INVALID_ARGUMENT, "bad scenario count, beam count, size or null output");
  if (n > INT64_MAX / 4 / n_scen / n_beams) fail(DOSE_ERR_INVALID_ARGUMENT, "beam doses too large");
  if (n > 0 && (!part || !p || !w)) fail(DOSE_ERR_INVALID_ARGUMENT, "null input");
  const uintptr_t a4 = reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(p) |
                       reinterpret_cast<uintptr_t>(w) | reinterpret_cast<uintptr_t>(d_out) |
                       reinterpret_cast<uintptr_t>(seed);
  const uintptr_t a8 = reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(prob);
  if (a4 % 4 != 0 || a8 % 8 != 0)
    fail(DOSE_ERR_INVALID_ARGUMENT, "float arrays must be 4-byte and double arrays 8-byte aligned");
  const size_t sn = static_cast<size_t>(n_scen) * static_cast<size_t>(n) * 4;
  const struct {
    const void* ptr;
    size_t bytes;
  } in[4] = {{part, sn * static_cast<size_t>(n_beams)}, {p, static_cast<size_t>(n) * 4},
             {w, static_cast<size_t>(n) * 4}, {prob, prob ? static_cast<size_t>(n_scen) * 8 : 0}},
    outs[3] = {{d_out, d_out ? sn : 0}, {seed, seed ? sn : 0}, {out, static_cast<size_t>(n_scen + 3) * 8}};
  for (int i = 0; i < 3; ++i) {
    if (!outs[i].ptr || outs[i].bytes == 0) continue;
    for (int j = 0; j < 4; ++j)
      if (in[j].ptr && in[j].bytes && overlaps(outs[i].ptr, outs[i].bytes, in[j].ptr, in[j].bytes))
        fail(DOSE_ERR_INVALID_ARGUMENT, "outputs must not overlap inputs");
    for (int j = i + 1; j < 3; ++j)
      if (outs[j].ptr && outs[j].bytes && overlaps(outs[i].ptr, outs[i].bytes, outs[j].ptr, outs[j].bytes))
        fail(DOSE_ERR_INVALID_ARGUMENT, "outputs must not overlap each other");
  }
}

int n_partial_for(int64_t n) { return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(1024, (n + 4095) / 4096))); }

}  // namespace

namespace {
// A's streams on the current device: validated host CSR uploaded, codes
// encoded, indices padded; no partition yet.  Synchronous on s.
std::unique_ptr<dose_matrix_s> upload_encode_A(const dose_csr_host* csr, int32_t vf, int32_t xf,
                                               hipStream_t s) {
  auto m = std::make_unique<dose_matrix_s>();
  HIP_CHECK(hipGetDevice(&m->device));
  m->vf = vf;
  m->xf = xf;
  Operand& A = m->A;
  A.n_rows = csr->n_rows;
  A.n_cols = csr->n_cols;
  A.nnz = csr->nnz;
  A.h_row_ptr.assign(csr->row_ptr, csr->row_ptr + csr->n_rows + 1);
  const int vb = value_bytes(vf);
  A.val = DevBuf(padded(A.nnz) * vb);
  A.idx_bytes = xf == DOSE_IDX_U16 ? 2 : 4;
  A.col = DevBuf(padded(A.nnz) * A.idx_bytes);
  if (m->vf == kFp8) m->row_scale = DevBuf(static_cast<size_t>(std::max<int64_t>(A.n_rows, 1)) * sizeof(float));
  HIP_CHECK(hipMemsetAsync(A.val.get(), 0, A.val.bytes(), s));
  HIP_CHECK(hipMemsetAsync(A.col.get(), 0, A.col.bytes(), s));
  upload_row_ptr32(A, s);
  if (A.nnz > 0 && A.idx_bytes == 4)
    HIP_CHECK(hipMemcpyAsync(A.col.get(), csr->col_idx, static_cast<size_t>(A.nnz) * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
  if (A.nnz > 0 && A.idx_bytes == 2) {
    // narrowed on the host in chunks (the indices were validated < 65536)
    const int64_t chunk = int64_t{1} << 24;
    std::vector<uint16_t> h(static_cast<size_t>(std::min<int64_t>(chunk, A.nnz)));
    for (int64_t k0 = 0; k0 < A.nnz; k0 += chunk) {
      const int64_t n = std::min<int64_t>(chunk, A.nnz - k0);
      for (int64_t k = 0; k < n; ++k) h[k] = static_cast<uint16_t>(csr->col_idx[k0 + k]);
      HIP_CHECK(hipMemcpyAsync(A.col.get<uint16_t>() + k0, h.data(), static_cast<size_t>(n) * 2,
                               hipMemcpyHostToDevice, s));
      HIP_CHECK(hipStreamSynchronize(s));  // h is reused
    }
  }
  HIP_CHECK(launch_fill_pad(A.col.get(), A.idx_bytes, A.nnz, pad_entries(A.nnz), s));
  encode_values(m.get(), csr, s);
  return m;
}
}  // namespace

namespace {

// ------------------------------------------------------------ SELL-C-sigma
// Host layout of SELL-C-sigma (C = 64): the sigma-sorted row order and the
// chunks' widths, as Kreutzer et al. define them: rows in consecutive windows
// of sigma rows, each window ordered by descending length (equal lengths keep
// ascending row order), the sequence cut into chunks of 64 positions.
struct SellLayout {
  std::vector<uint32_t> perm;  // row at each position
  std::vector<int64_t> width;  // longest row of each chunk
};

SellLayout sell_layout(const int64_t* rp, int64_t n_rows, int64_t sigma) {
  SellLayout L;
  L.perm.resize(static_cast<size_t>(n_rows));
  const int64_t n_win = sigma > 0 ? (n_rows + sigma - 1) / sigma : 0;
  auto work = [&](int64_t w_begin, int64_t w_end) {
    for (int64_t w = w_begin; w < w_end; ++w) {
      const int64_t r0 = w * sigma, r1 = std::min(n_rows, r0 + sigma);
      for (int64_t r = r0; r < r1; ++r) L.perm[r] = static_cast<uint32_t>(r);
      std::stable_sort(L.perm.begin() + r0, L.perm.begin() + r1, [&](uint32_t a, uint32_t b) {
        return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
      });
    }
  };
  const int64_t parts = std::max<int64_t>(1, std::min<int64_t>(16, n_win / 64));
  if (parts == 1) {
    work(0, n_win);
  } else {
    std::vector<std::thread> th;
    for (int64_t p = 0; p < parts; ++p) th.emplace_back(work, n_win * p / parts, n_win * (p + 1) / parts);
    for (auto& t : th) t.join();
  }
  const int64_t n_chunks = (n_rows + kSellC - 1) / kSellC;
  L.width.assign(static_cast<size_t>(n_chunks), 0);
  for (int64_t i = 0; i < n_rows; ++i) {
    const uint32_t r = L.perm[i];
    L.width[i / kSellC] = std::max(L.width[i / kSellC], rp[r + 1] - rp[r]);
  }
  return L;
}

// Most runs of one chunk of 64 row positions with run-length indices (the
// chunk's runs are staged in LDS: 8 B each).
constexpr int64_t kSellMaxGroupRuns = 1024;

void check_sigma(int64_t sigma) {
  if (sigma < 1 || sigma > INT32_MAX) fail(DOSE_ERR_INVALID_ARGUMENT, "sigma must be in [1, 2^31)");
}

}  // namespace

struct dose_sell_s {
  int device = 0;
  int vf = 0, xf = 0;
  int32_t sigma = 1;
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  int64_t n_chunks = 0;  // ceil(n_rows / 64)
  int64_t n_groups = 0;  // ceil(n_chunks / 4); the chunk and position arrays are padded to whole groups
  int64_t n_slices = 0, n_windowed = 0;
  int64_t std_slots = 0;  // 64 * sum of the chunks' widths (Kreutzer's layout)
  int32_t win_floats[3] = {0, 0, 0};  // LDS window floats for 1, 2 and 4 vectors
  int32_t idx_bytes = 4;               // 0: run-length indices
  int64_t n_runs = 0;
  int32_t lds_runs = 0;  // most runs of one group
  int64_t n_work = 0, n_zero = 0;  // chunks with entries, chunks without
  std::vector<SellChunk> h_chunks;
  std::vector<uint32_t> h_perm, h_len;
  std::vector<int64_t> h_width;
  DevBuf val, col, chunks, win, perm, len, row_scale, run_ptr, runs, work;
};

namespace {

// n_rhs selects the LDS window (2 for one FP64 vector: 8 bytes a column).
SellArgs sell_args(const dose_sell_s* m, int n_rhs, const void* x, void* y) {
  SellArgs a{};
  a.chunks = m->chunks.get<SellChunk>();
  a.win = m->win.get<uint32_t>();
  a.val = m->val.get();
  a.col = m->col.get();
  a.perm = m->perm.get<uint32_t>();
  a.len = m->len.get<uint32_t>();
  a.scale = m->vf == kFp8 ? m->row_scale.get<float>() : nullptr;
  a.run_ptr = m->run_ptr.get<uint32_t>();
  a.runs = m->runs.get<SellRun>();
  a.work = m->work.get<uint32_t>();
  a.zero = m->work.get<uint32_t>() + m->n_work;
  a.x = x;
  a.y = y;
  a.n_groups = m->n_work;
  a.n_zero = m->n_zero;
  a.win_floats = m->win_floats[rhs_slot(n_rhs)];
  a.idx_bytes = m->idx_bytes;
  a.xcd_blocks = xcd_blocks(8);
  a.lds_runs = m->lds_runs;
  a.n_cols = static_cast<int32_t>(std::min<int64_t>(m->n_cols, INT32_MAX));
  return a;
}

// Arguments of a SELL-C-sigma product with n_rhs row-major vectors.
void check_sell_product(const dose_sell_s* m, int32_t n_rhs, const float* x, const float* y) {
  if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
  if (n_rhs != 1 && n_rhs != 2 && n_rhs != 4) fail(DOSE_ERR_UNSUPPORTED, "n_rhs must be 1, 2 or 4");
  if ((m->n_cols > 0 && !x) || (m->n_rows > 0 && !y)) fail(DOSE_ERR_INVALID_ARGUMENT, "null x or y");
  if (m->n_cols > INT32_MAX / n_rhs) fail(DOSE_ERR_UNSUPPORTED, "n_cols * n_rhs must stay below 2^31");
  if (overlaps(x, m->n_cols * n_rhs * 4, y, m->n_rows * n_rhs * 4))
    fail(DOSE_ERR_INVALID_ARGUMENT, "x and y overlap");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % (4 * static_cast<uintptr_t>(n_rhs)) != 0)
    fail(DOSE_ERR_INVALID_ARGUMENT, "x and y must be aligned to n_rhs floats");
}

void check_sell_items(const dose_sell_batch_item* items, int32_t n_items) {
  if (!items || n_items <= 0) fail(DOSE_ERR_INVALID_ARGUMENT, "no items");
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_sell_batch_item& it = items[i];
    if (!it.S) fail(DOSE_ERR_INVALID_ARGUMENT, "item without matrix");
    if (it.ldx != it.n_rhs || it.ldy != it.n_rhs) fail(DOSE_ERR_UNSUPPORTED, "ldx and ldy must equal n_rhs");
    check_sell_product(it.S, it.n_rhs, it.x, it.y);
    const dose_sell_s* m0 = items[0].S;
    if (it.S->vf != m0->vf) fail(DOSE_ERR_UNSUPPORTED, "items mix value formats");
    if (it.S->idx_bytes != m0->idx_bytes) fail(DOSE_ERR_UNSUPPORTED, "items mix index formats");
    if (it.n_rhs != items[0].n_rhs) fail(DOSE_ERR_UNSUPPORTED, "items mix n_rhs");
    if (it.S->device != m0->device) fail(DOSE_ERR_INVALID_ARGUMENT, "items on different devices");
    const int64_t yb = it.S->n_rows * it.n_rhs * 4;
    for (int32_t j = 0; j < n_items; ++j) {
      const dose_sell_batch_item& o = items[j];
      if (!o.S) continue;
      // one launch reads every x while it writes every y
      if (overlaps(o.x, o.S->n_cols * o.n_rhs * 4, it.y, yb)) fail(DOSE_ERR_INVALID_ARGUMENT, "a y overlaps an x");
      if (j < i && overlaps(o.y, o.S->n_rows * o.n_rhs * 4, it.y, yb))
        fail(DOSE_ERR_INVALID_ARGUMENT, "items share outputs");
    }
  }
}

// One launch over the chunks of all items: those holding entries, item by
// item in chunk order, then those without (their rows get +0).
dose_batch_plan_s* build_sell_plan(const dose_sell_batch_item* items, int32_t n_items, hipStream_t s) {
  auto plan = std::make_unique<dose_batch_plan_s>();
  const dose_sell_s* m0 = items[0].S;
  plan->device = m0->device;
  plan->vf = m0->vf;
  plan->sm = m0->vf == kFp8 ? kScaleRow : kScaleNone;
  plan->n_rhs = items[0].n_rhs;
  plan->idx_bytes = m0->idx_bytes;
  SellPlanLayer L;
  std::vector<SellArgs> args(static_cast<size_t>(n_items));
  std::vector<uint2> work, zero;
  for (int32_t i = 0; i < n_items; ++i) {
    const dose_sell_s* m = items[i].S;
    args[i] = sell_args(m, plan->n_rhs, items[i].x, items[i].y);
    L.lds_bytes = std::max(L.lds_bytes, sell_launch_lds_bytes(args[i]));
    for (size_t c = 0; c < m->h_chunks.size(); ++c)
      (m->h_chunks[c].n_slices > 0 ? work : zero).push_back(make_uint2(static_cast<uint32_t>(i),
                                                                       static_cast<uint32_t>(c)));
  }
  L.n_work = static_cast<int64_t>(work.size());
  L.n_zero = static_cast<int64_t>(zero.size());
  if (L.n_work + (L.n_zero + kGroupWaves - 1) / kGroupWaves > int64_t{0x7fffffff})
    fail(DOSE_ERR_UNSUPPORTED, "too many chunks for one launch");
  L.xcd = xcd_blocks(8);
  L.args = DevBuf(args.size() * sizeof(SellArgs));
  L.work = DevBuf(std::max<size_t>(1, work.size()) * sizeof(uint2));
  L.zero = DevBuf(std::max<size_t>(1, zero.size()) * sizeof(uint2));
  HIP_CHECK(hipMemcpyAsync(L.args.get(), args.data(), args.size() * sizeof(SellArgs), hipMemcpyHostToDevice, s));
  if (!work.empty())
    HIP_CHECK(hipMemcpyAsync(L.work.get(), work.data(), work.size() * sizeof(uint2), hipMemcpyHostToDevice, s));
  if (!zero.empty())
    HIP_CHECK(hipMemcpyAsync(L.zero.get(), zero.data(), zero.size() * sizeof(uint2), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));
  plan->sell_layers.push_back(std::move(L));
  return plan.release();
}

}  // namespace

// ------------------------------------------------ static scratch (no allocation)
// The partial sums of dose_scenario_objective_noalloc live in this array:
// each device that runs the library holds its own copy until the process
// ends.  Host code must not pass the array's name to a kernel (on the host
// it is a stand-in, not a device address): its address on each device comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t kScratchDoubles = 65536;  // 512 KB: 64 scenarios x 1024 partial sums
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (looked up once per
// device; the lookup allocates nothing).
double* scratch_on_current_device() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(DOSE_ERR_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(DOSE_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// ================================================================== C ABI
extern "C" {

const char* dose_status_string(dose_status s) {
  switch (s) {
    case DOSE_OK: return "ok";
    case DOSE_ERR_INVALID_ARGUMENT: return "invalid argument";
    case DOSE_ERR_BAD_CSR: return "malformed CSR matrix";
    case DOSE_ERR_UNSUPPORTED: return "unsupported";
    case DOSE_ERR_NO_TRANSPOSE: return "matrix has no transpose";
    case DOSE_ERR_OUT_OF_MEMORY: return "out of memory";
    case DOSE_ERR_HIP: return "HIP runtime error";
    case DOSE_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* dose_last_error(void) { return g_last_error.c_str(); }

dose_status dose_csr_validate(const dose_csr_host* csr, int32_t vf, int32_t xf) {
  return guarded([&] { validate_csr(csr, vf, xf); });
}

dose_status dose_partition_preview(const int64_t* row_ptr, int64_t n_rows, int32_t group_nnz, int64_t* groups,
                                   int64_t cap, int64_t* n_groups) {
  return guarded([&] {
    if (!row_ptr || !n_groups || n_rows < 0 || (cap > 0 && !groups)) fail(DOSE_ERR_INVALID_ARGUMENT, "bad argument");
    check_group_nnz(group_nnz);
    std::vector<GroupDesc> G = build_partition(row_ptr, n_rows, group_nnz);
    *n_groups = static_cast<int64_t>(G.size());
    for (int64_t i = 0; i < std::min<int64_t>(cap, *n_groups); ++i) {
      const GroupDesc& g = G[i];
      int64_t* o = groups + i * (kGroupWaves + 2);
      for (int w = 0; w <= kGroupWaves; ++w) o[w] = g.row[w];
      o[kGroupWaves + 1] = g.split;
    }
  });
}

dose_status dose_matrix_create(const dose_csr_host* csr, int32_t vf, int32_t xf, uint32_t flags,
                               void* hip_stream, dose_matrix* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    if (xf == DOSE_IDX_RUNS) fail(DOSE_ERR_UNSUPPORTED, "run-length indices are a SELL-C-sigma format (dose_sell_create)");
    if (flags & ~static_cast<uint32_t>(DOSE_CREATE_TRANSPOSE | DOSE_CREATE_AUTOTUNE | DOSE_CREATE_TRANSPOSE_SLABS))
      fail(DOSE_ERR_INVALID_ARGUMENT, "unknown flags");
    validate_csr(csr, vf, xf);
    hipStream_t s = as_stream(hip_stream);
    auto m = upload_encode_A(csr, vf, xf, s);
    Operand& A = m->A;
    upload_partition(A, default_group_nnz(A.nnz, m->device), s);
    if (flags & DOSE_CREATE_TRANSPOSE_SLABS) {
      build_transpose_slabs(m.get(), default_group_nnz(A.nnz, m->device), s);
      m->has_t = true;
    } else if (flags & DOSE_CREATE_TRANSPOSE) {
      build_transpose(m.get(), default_group_nnz(A.nnz, m->device), s);
      m->has_t = true;
    }
    if (flags & DOSE_CREATE_AUTOTUNE) {
      // the plain one-vector products timed under candidate row-group sizes
      // (the paper's block-size sweep, Sec. V-A), on scratch vectors of zeros
      const int64_t nr = std::max<int64_t>(A.n_rows, 1), nc = std::max<int64_t>(A.n_cols, 1);
      DevBuf xa(static_cast<size_t>(nc) * 4), ya(static_cast<size_t>(nr) * 4);
      HIP_CHECK(hipMemsetAsync(xa.get(), 0, xa.bytes(), s));
      HIP_CHECK(hipMemsetAsync(ya.get(), 0, ya.bytes(), s));
      if (A.nnz > 0) {
        auto P = autotune_operand(m.get(), A, scale_mode_A(m.get()), 1, xa.get<float>(), ya.get<float>(), s);
        if (P) A.part = std::move(*P);
        if (m->has_t && m->AT.nnz > 0) {
          // the mode dose_spmv_adjoint runs (E4M3: its seed carries the row
          // scales); the slab form writes one partial per row
          const int smt = m->vf == kFp8 ? kScaleNone : scale_mode_AT(m.get());
          DevBuf part;
          float* yt = xa.get<float>();
          if (m->slab > 0) {
            part = DevBuf(static_cast<size_t>(std::max<int64_t>(m->AT.n_rows, 1)) * 4);
            yt = part.get<float>();
          }
          auto PT = autotune_operand(m.get(), m->AT, smt, 1, ya.get<float>(), yt, s);
          if (PT) m->AT.part = std::move(*PT);
        }
      }
    }
    HIP_CHECK(hipStreamSynchronize(s));
    *out = m.release();
  });
}

dose_status dose_matrix_set_partition(dose_matrix m, int32_t group_nnz, int32_t group_nnz_t) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    check_group_nnz(group_nnz);
    if (m->has_t) check_group_nnz(group_nnz_t);
    DeviceGuard g(m->device);
    HIP_CHECK(hipDeviceSynchronize());
    upload_partition(m->A, group_nnz, nullptr);
    if (m->has_t) upload_partition(m->AT, group_nnz_t, nullptr);
  });
}

dose_status dose_matrix_decode(dose_matrix m, int32_t part, int64_t row_begin, int64_t row_end, int64_t* row_ptr_out,
                               int32_t* col_out, float* val_out) {
  return guarded([&] {
    if (!m || !row_ptr_out) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    if (part != DOSE_PART_A && part != DOSE_PART_AT) fail(DOSE_ERR_INVALID_ARGUMENT, "unknown part");
    if (part == DOSE_PART_AT && !m->has_t) fail(DOSE_ERR_NO_TRANSPOSE, "matrix has no transpose");
    if (part == DOSE_PART_AT && m->slab > 0)
      fail(DOSE_ERR_UNSUPPORTED, "A^T is stored in voxel slabs, not one row per spot (decode A instead)");
    const Operand& op = part == DOSE_PART_A ? m->A : m->AT;
    if (row_begin < 0 || row_end < row_begin || row_end > op.n_rows) fail(DOSE_ERR_INVALID_ARGUMENT, "row range");
    DeviceGuard g(m->device);
    const int64_t nb = op.h_row_ptr[row_begin], ne = op.h_row_ptr[row_end], n = ne - nb;
    for (int64_t i = row_begin; i <= row_end; ++i) row_ptr_out[i - row_begin] = op.h_row_ptr[i] - nb;
    if (n == 0) return;
    if (col_out && op.idx_bytes == 4)
      HIP_CHECK(hipMemcpy(col_out, op.col.get<int32_t>() + nb, static_cast<size_t>(n) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (col_out && op.idx_bytes == 2) {
      std::vector<uint16_t> h(static_cast<size_t>(n));
      HIP_CHECK(hipMemcpy(h.data(), op.col.get<uint16_t>() + nb, static_cast<size_t>(n) * 2, hipMemcpyDeviceToHost));
      for (int64_t k = 0; k < n; ++k) col_out[k] = h[k];
    }
    if (val_out) {
      DevBuf tmp(static_cast<size_t>(n) * sizeof(float));
      const int sm = part == DOSE_PART_A ? scale_mode_A(m) : scale_mode_AT(m);
      // the column scale mode (E4M3 A^T) reads the int32 columns of A^T
      HIP_CHECK(launch_decode(m->vf, sm, op.val.get(), op.idx_bytes == 4 ? op.col.get<int32_t>() : nullptr,
                              m->row_scale.get<float>(),
                              op.row_ptr.get<uint32_t>(), row_begin, row_end - row_begin, static_cast<uint64_t>(nb), n,
                              tmp.get<float>(), nullptr));
      HIP_CHECK(hipDeviceSynchronize());
      HIP_CHECK(hipMemcpy(val_out, tmp.get(), static_cast<size_t>(n) * sizeof(float), hipMemcpyDeviceToHost));
    }
  });
}

dose_status dose_matrix_info(dose_matrix m, dose_matrix_info_t* info) {
  return guarded([&] {
    if (!m || !info) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    std::memset(info, 0, sizeof(*info));
    const Operand& A = m->A;
    info->n_rows = A.n_rows;
    info->n_cols = A.n_cols;
    info->nnz = A.nnz;
    info->value_format = m->vf;
    info->index_format = m->xf;
    info->has_transpose = m->has_t ? 1 : 0;
    info->group_nnz = A.part.group_nnz;
    info->n_groups = A.part.n_groups;
    info->n_groups_windowed = A.part.n_windowed;
    info->group_nnz_t = m->has_t ? m->AT.part.group_nnz : 0;
    info->n_groups_t = m->has_t ? m->AT.part.n_groups : 0;
    info->n_groups_windowed_t = m->has_t ? m->AT.part.n_windowed : 0;
    info->device_bytes = A.bytes() + m->row_scale.bytes() + (m->has_t ? m->AT.bytes() : 0) + m->comb_ptr.bytes() +
                         m->comb_rows.bytes();
    info->slab_voxels = m->slab;
    const uint64_t per_nnz = static_cast<uint64_t>(value_bytes(m->vf)) + static_cast<uint64_t>(A.idx_bytes);
    const uint64_t per_nnz_t = static_cast<uint64_t>(value_bytes(m->vf)) + 4;
    const uint64_t scale_b = m->vf == kFp8 ? 4 : 0;
    info->spmv_bytes = A.nnz * per_nnz + (A.n_rows + 1) * 4 + A.n_rows * scale_b + 4 * A.n_cols + 4 * A.n_rows;
    // A^T reads the scale of A's rows through its columns: 4 B per column of A^T
    info->n_groups_split = A.part.n_split;
    info->n_groups_split_t = m->has_t ? m->AT.part.n_split : 0;
    info->adjoint_bytes = m->has_t ? A.nnz * per_nnz_t + (A.n_cols + 1) * 4 + A.n_rows * scale_b + 4 * A.n_rows + 4 * A.n_cols : 0;
    if (m->slab > 0) {
      // voxel slabs: 16-bit indices, the padding entries, one offset per
      // slab row instead of per spot, each row's partial written and read
      // back, the combine map
      const uint64_t rows_t = static_cast<uint64_t>(m->AT.n_rows), rows_real = static_cast<uint64_t>(m->n_slab_rows);
      const uint64_t per_nnz_s = static_cast<uint64_t>(value_bytes(m->vf)) + 2;
      info->adjoint_bytes = (A.nnz + m->n_slab_pad) * per_nnz_s + (rows_t + 1) * 4 + A.n_rows * scale_b +
                            4 * A.n_rows + 8 * rows_t + (A.n_cols + 1) * 4 + 4 * rows_real + 4 * A.n_cols;
    }
  });
}

dose_status dose_matrix_destroy(dose_matrix m) {
  return guarded([&] {
    if (!m) return;
    DeviceGuard g(m->device);
    (void)hipDeviceSynchronize();
    delete m;
  });
}

dose_status dose_spmv(dose_matrix m, const float* x, float* y, void* hip_stream) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    if ((m->A.n_cols > 0 && !x) || (m->A.n_rows > 0 && !y)) fail(DOSE_ERR_INVALID_ARGUMENT, "null x or y");
    if (overlaps(x, m->A.n_cols * 4, y, m->A.n_rows * 4)) fail(DOSE_ERR_INVALID_ARGUMENT, "x and y overlap");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 4 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "x and y must be 4-byte aligned");
    DeviceGuard g(m->device);
    run_product(m, m->A, scale_mode_A(m), 1, x, y, as_stream(hip_stream));
  });
}

dose_status dose_spmv_f64(dose_matrix m, const double* x, double* y, void* hip_stream) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    if ((m->A.n_cols > 0 && !x) || (m->A.n_rows > 0 && !y)) fail(DOSE_ERR_INVALID_ARGUMENT, "null x or y");
    if (overlaps(x, m->A.n_cols * 8, y, m->A.n_rows * 8)) fail(DOSE_ERR_INVALID_ARGUMENT, "x and y overlap");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 8 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "x and y must be 8-byte aligned");
    DeviceGuard g(m->device);
    const int sm = scale_mode_A(m);
    HIP_CHECK(launch_spmv_f64(m->vf, sm, make_args(m, m->A, sm, 2, x, y), as_stream(hip_stream)));
  });
}

dose_status dose_spmv_adjoint_f64(dose_matrix m, const double* v, double* gout, void* hip_stream) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    if (!m->has_t) fail(DOSE_ERR_NO_TRANSPOSE, "matrix was created without DOSE_CREATE_TRANSPOSE");
    if ((m->A.n_rows > 0 && !v) || (m->A.n_cols > 0 && !gout)) fail(DOSE_ERR_INVALID_ARGUMENT, "null v or g");
    if (overlaps(v, m->A.n_rows * 8, gout, m->A.n_cols * 8)) fail(DOSE_ERR_INVALID_ARGUMENT, "v and g overlap");
    if ((reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(gout)) % 8 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "v and g must be 8-byte aligned");
    DeviceGuard g(m->device);
    const int sm = scale_mode_AT(m);
    hipStream_t s = as_stream(hip_stream);
    if (m->slab == 0) {
      HIP_CHECK(launch_spmv_f64(m->vf, sm, make_args(m, m->AT, sm, 2, v, gout), s));
      return;
    }
    // voxel slabs: the rows' FP64 partials, then each spot's sum over its
    // slabs in ascending order
    double* part = nullptr;
    if (m->AT.n_rows > 0)
      HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&part), static_cast<size_t>(m->AT.n_rows) * 8, s));
    hipError_t e = launch_spmv_f64(m->vf, sm, make_args(m, m->AT, sm, 2, v, part), s);
    if (e == hipSuccess)
      e = launch_slab_combine(true, part, m->comb_ptr.get<uint32_t>(), m->comb_rows.get<uint32_t>(), gout,
                              m->A.n_cols, s);
    if (part) (void)hipFreeAsync(part, s);
    HIP_CHECK(e);
  });
}

dose_status dose_spmv_adjoint(dose_matrix m, const float* v, float* gout, void* hip_stream) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    if (!m->has_t) fail(DOSE_ERR_NO_TRANSPOSE, "matrix was created without DOSE_CREATE_TRANSPOSE");
    if ((m->A.n_rows > 0 && !v) || (m->A.n_cols > 0 && !gout)) fail(DOSE_ERR_INVALID_ARGUMENT, "null v or g");
    if (overlaps(v, m->A.n_rows * 4, gout, m->A.n_cols * 4)) fail(DOSE_ERR_INVALID_ARGUMENT, "v and g overlap");
    if ((reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(gout)) % 4 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "v and g must be 4-byte aligned");
    DeviceGuard g(m->device);
    hipStream_t s = as_stream(hip_stream);
    if (m->vf != kFp8 && m->slab == 0) {
      run_product(m, m->AT, scale_mode_AT(m), 1, v, gout, s);
      return;
    }
    // E4M3: the row scales go into the seed first (u_i = fl32(s_i v_i)), so
    // that each entry of A^T gathers one value; its term is fl32(q u_i).
    // Voxel slabs: the rows' partials, then each spot's sum over its slabs in
    // ascending order.  One stream-ordered allocation holds u and the partials.
    const bool fp8 = m->vf == kFp8;
    const int64_t n_u = fp8 ? m->A.n_rows : 0, n_p = m->slab > 0 ? m->AT.n_rows : 0;
    float* buf = nullptr;
    if (n_u + n_p > 0)
      HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&buf), static_cast<size_t>(n_u + n_p) * 4, s));
    float* u = fp8 ? buf : nullptr;
    float* part = m->slab > 0 ? buf + n_u : nullptr;
    hipError_t e = hipSuccess;
    if (fp8) e = launch_scale_vec(n_u, m->row_scale.get<float>(), v, u, s);
    const float* x = fp8 ? u : v;
    const int sm = fp8 ? kScaleNone : scale_mode_AT(m);
    if (e == hipSuccess) e = launch_spmv(m->vf, sm, 1, make_args(m, m->AT, sm, 1, x, m->slab > 0 ? part : gout), s);
    if (e == hipSuccess && m->slab > 0)
      e = launch_slab_combine(false, part, m->comb_ptr.get<uint32_t>(), m->comb_rows.get<uint32_t>(), gout,
                              m->A.n_cols, s);
    if (buf) (void)hipFreeAsync(buf, s);
    HIP_CHECK(e);
  });
}

dose_status dose_spmv_batched(const dose_batch_item* items, int32_t n_items, void* hip_stream) {
  return guarded([&] {
    check_items(items, n_items);
    DeviceGuard g(items[0].A->device);
    launch_items(items, n_items, as_stream(hip_stream));
  });
}

dose_status dose_batch_plan_create(const dose_batch_item* items, int32_t n_items, uint32_t flags, void* hip_stream,
                                   dose_batch_plan* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    check_items(items, n_items);
    DeviceGuard g(items[0].A->device);
    std::unique_ptr<dose_batch_plan_s> p(build_plan(items, n_items, flags, as_stream(hip_stream)));
    capture_plan(p.get());
    *out = p.release();
  });
}

dose_status dose_adjoint_plan_create(const dose_adjoint_item* items, int32_t n_items, uint32_t flags,
                                     void* hip_stream, dose_batch_plan* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    if (flags & ~static_cast<uint32_t>(DOSE_PLAN_AUTOTUNE | DOSE_ADJOINT_ACCUMULATE))
      fail(DOSE_ERR_INVALID_ARGUMENT, "unknown flags");
    check_adjoint_items(items, n_items, (flags & DOSE_ADJOINT_ACCUMULATE) != 0);
    DeviceGuard g(items[0].A->device);
    std::unique_ptr<dose_batch_plan_s> p(build_adjoint_plan(items, n_items, flags, as_stream(hip_stream)));
    capture_plan(p.get());
    *out = p.release();
  });
}

dose_status dose_scenario_plan_create(const dose_matrix* mats, const float* const* x, int32_t n_scen,
                                      int32_t n_beams, float* d, uint32_t flags, void* hip_stream,
                                      dose_batch_plan* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    if (!mats || !x || n_scen < 1 || n_beams < 1 || n_scen > kMaxScenarios || n_beams > kMaxScenarios)
      fail(DOSE_ERR_INVALID_ARGUMENT, "bad matrices, spot weights or counts");
    const int64_t n_items = static_cast<int64_t>(n_scen) * n_beams;
    if (n_items > INT32_MAX) fail(DOSE_ERR_INVALID_ARGUMENT, "too many items");
    for (int64_t i = 0; i < n_items; ++i)
      if (!mats[i]) fail(DOSE_ERR_INVALID_ARGUMENT, "null matrix");
    const int64_t n = mats[0]->A.n_rows;
    if (n > 0 && !d) fail(DOSE_ERR_INVALID_ARGUMENT, "d is null");
    const size_t d_bytes = static_cast<size_t>(n_scen) * static_cast<size_t>(n) * 4;
    // items of beam b: (scenario s, beam b) for every s, writing scenario s's dose
    std::vector<dose_batch_item> items(static_cast<size_t>(n_items));
    for (int32_t s = 0; s < n_scen; ++s)
      for (int32_t b = 0; b < n_beams; ++b) {
        const int64_t i = static_cast<int64_t>(s) * n_beams + b;
        if (mats[i]->A.n_rows != n) fail(DOSE_ERR_INVALID_ARGUMENT, "beam matrices of different dose grids");
        if (overlaps(x[i], mats[i]->A.n_cols * 4, d, d_bytes)) fail(DOSE_ERR_INVALID_ARGUMENT, "x overlaps d");
        dose_batch_item& it = items[static_cast<size_t>(b) * n_scen + s];
        it = dose_batch_item{};
        it.A = mats[i];
        it.n_rhs = 1;
        it.x = x[i];
        it.ldx = 1;
        it.y = d + static_cast<int64_t>(s) * n;
        it.ldy = 1;
      }
    for (int32_t b = 0; b < n_beams; ++b) check_items(items.data() + static_cast<size_t>(b) * n_scen, n_scen);
    for (int64_t i = 0; i < n_items; ++i)
      if (mats[i]->vf != mats[0]->vf || mats[i]->A.idx_bytes != mats[0]->A.idx_bytes ||
          mats[i]->device != mats[0]->device)
        fail(DOSE_ERR_UNSUPPORTED, "beam matrices mix formats or devices");
    DeviceGuard g(items[0].A->device);
    hipStream_t s = as_stream(hip_stream);
    auto plan = new_plan(items.data());
    const auto part_of = plan_partitions(plan.get(), items.data(), static_cast<int32_t>(n_items), flags, s);
    // one launch per beam, in ascending beam order: the first stores, the
    // others add, so that each voxel's dose is the FP32 sum of its beam doses
    // in ascending beam order
    for (int32_t b = 0; b < n_beams; ++b)
      plan->layers.push_back(make_layer(plan.get(), items.data() + static_cast<size_t>(b) * n_scen, n_scen, part_of,
                                        b > 0 ? 1 : 0, s));
    capture_plan(plan.get());
    *out = plan.release();
  });
}

dose_status dose_batch_plan_launch(dose_batch_plan p, void* hip_stream) {
  return guarded([&] {
    if (!p || !p->exec) fail(DOSE_ERR_INVALID_ARGUMENT, "plan is null");
    DeviceGuard g(p->device);
    HIP_CHECK(hipGraphLaunch(p->exec, as_stream(hip_stream)));
  });
}

dose_status dose_batch_plan_destroy(dose_batch_plan p) {
  return guarded([&] {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    delete p;
  });
}

dose_status dose_objective(int64_t n, const float* d, const float* p, const float* w, float* seed, double* f_out,
                           void* hip_stream) {
  return guarded([&] {
    if (n < 0 || !f_out || (n > 0 && (!d || !p || !w))) fail(DOSE_ERR_INVALID_ARGUMENT, "bad argument");
    hipStream_t s = as_stream(hip_stream);
    const int np = n_partial_for(n);
    double* partial = nullptr;
    HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial), np * sizeof(double), s));
    hipError_t e = launch_objective(n, d, p, w, seed, partial, np, f_out, s);
    (void)hipFreeAsync(partial, s);
    HIP_CHECK(e);
  });
}

dose_status dose_scenario_objective(int32_t n_scen, int32_t n_beams, int64_t n, const float* part, const float* p,
                                    const float* w, const double* prob, float* d_out, float* seed, double* out,
                                    void* hip_stream) {
  return guarded([&] {
    check_scenario_args(n_scen, n_beams, n, part, p, w, prob, d_out, seed, out);
    hipStream_t s = as_stream(hip_stream);
    const int np = n_partial_for(n);
    double* partial = nullptr;
    HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial), static_cast<size_t>(np) * n_scen * sizeof(double), s));
    hipError_t e = launch_scenario(n_scen, n_beams, n, part, p, w, prob, d_out, seed, partial, np, out, s);
    (void)hipFreeAsync(partial, s);
    HIP_CHECK(e);
  });
}

dose_status dose_scenario_objective_noalloc(int32_t n_scen, int32_t n_beams, int64_t n, const float* part,
                                            const float* p, const float* w, const double* prob, float* d_out,
                                            float* seed, double* out, void* hip_stream) {
  return guarded([&] {
    check_scenario_args(n_scen, n_beams, n, part, p, w, prob, d_out, seed, out);
    const int np = n_partial_for(n);
    if (static_cast<int64_t>(np) * n_scen > kScratchDoubles)
      fail(DOSE_ERR_INVALID_ARGUMENT, "n_scen * partial sums exceed the static scratch (65,536 doubles: at most 64 "
                                      "scenarios, or more when n is small)");
    double* partial = scratch_on_current_device();
    // every partial sum the second pass reads is written by the first, so
    // nothing needs clearing between calls
    HIP_CHECK(launch_scenario(n_scen, n_beams, n, part, p, w, prob, d_out, seed, partial, np, out,
                              as_stream(hip_stream)));
  });
}

dose_status dose_robust_seed(int32_t n_scen, int64_t n, int32_t mode, const double* out, const double* prob,
                             const double* grad_scale, const float* seed, float* wseed, void* hip_stream) {
  return guarded([&] {
    if (n_scen < 1 || n_scen > kMaxScenarios || n < 0) fail(DOSE_ERR_INVALID_ARGUMENT, "bad scenario count or size");
    if (mode != DOSE_ROBUST_EXPECTED && mode != DOSE_ROBUST_WORST) fail(DOSE_ERR_INVALID_ARGUMENT, "unknown mode");
    if (mode == DOSE_ROBUST_WORST && !out) fail(DOSE_ERR_INVALID_ARGUMENT, "the worst case needs out");
    if (n > 0 && (!seed || !wseed)) fail(DOSE_ERR_INVALID_ARGUMENT, "null seed or wseed");
    if (n > INT64_MAX / 4 / n_scen) fail(DOSE_ERR_INVALID_ARGUMENT, "seeds too large");
    const uintptr_t a4 = reinterpret_cast<uintptr_t>(seed) | reinterpret_cast<uintptr_t>(wseed);
    const uintptr_t a8 = reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(prob) |
                         reinterpret_cast<uintptr_t>(grad_scale);
    if (a4 % 4 != 0 || a8 % 8 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "float arrays must be 4-byte and double arrays 8-byte aligned");
    const size_t sn = static_cast<size_t>(n_scen) * static_cast<size_t>(n) * 4;
    if (seed != wseed && overlaps(seed, sn, wseed, sn))
      fail(DOSE_ERR_INVALID_ARGUMENT, "wseed overlaps seed without being seed");
    const struct {
      const void* ptr;
      size_t bytes;
    } in[3] = {{out, out ? static_cast<size_t>(n_scen + 3) * 8 : 0},
               {prob, prob ? static_cast<size_t>(n_scen) * 8 : 0},
               {grad_scale, grad_scale ? size_t{8} : 0}};
    for (const auto& i : in)
      if (i.ptr && overlaps(wseed, sn, i.ptr, i.bytes)) fail(DOSE_ERR_INVALID_ARGUMENT, "wseed overlaps an input");
    HIP_CHECK(launch_robust_seed(n_scen, n, mode == DOSE_ROBUST_WORST ? 1 : 0, out, prob, grad_scale, seed, wseed,
                                 as_stream(hip_stream)));
  });
}

dose_status dose_norm2(int64_t n, const float* gv, double* out, void* hip_stream) {
  return guarded([&] {
    if (n < 0 || !out || (n > 0 && !gv)) fail(DOSE_ERR_INVALID_ARGUMENT, "bad argument");
    hipStream_t s = as_stream(hip_stream);
    const int np = n_partial_for(n);
    double* partial = nullptr;
    HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&partial), np * sizeof(double), s));
    hipError_t e = launch_norm2(n, gv, partial, np, out, s);
    (void)hipFreeAsync(partial, s);
    HIP_CHECK(e);
  });
}

dose_status dose_probe_stream_read(const void* buf, uint64_t bytes, float* sink, void* hip_stream) {
  return guarded([&] {
    if (!buf || !sink) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    HIP_CHECK(launch_probe_read(buf, bytes, sink, as_stream(hip_stream)));
  });
}

dose_status dose_probe_copy(const void* src, void* dst, uint64_t bytes, void* hip_stream) {
  return guarded([&] {
    if (!src || !dst) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    if (overlaps(src, bytes, dst, bytes)) fail(DOSE_ERR_INVALID_ARGUMENT, "src and dst overlap");
    HIP_CHECK(launch_probe_copy(src, dst, bytes, as_stream(hip_stream)));
  });
}

dose_status dose_sell_layout(const int64_t* row_ptr, int64_t n_rows, int32_t sigma, int64_t* perm, int64_t* width) {
  return guarded([&] {
    if (!row_ptr || n_rows < 0 || (n_rows > 0 && (!perm || !width))) fail(DOSE_ERR_INVALID_ARGUMENT, "bad argument");
    check_sigma(sigma);
    if (n_rows > int64_t{0xFFFFFFFE}) fail(DOSE_ERR_UNSUPPORTED, "more than 2^32 - 2 rows");
    for (int64_t i = 0; i < n_rows; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) fail(DOSE_ERR_BAD_CSR, "row_ptr decreases at row " + std::to_string(i));
    SellLayout L = sell_layout(row_ptr, n_rows, sigma);
    for (int64_t i = 0; i < n_rows; ++i) perm[i] = L.perm[i];
    for (size_t c = 0; c < L.width.size(); ++c) width[c] = L.width[c];
  });
}

dose_status dose_sell_create(const dose_csr_host* csr, int32_t vf, int32_t xf, int32_t sigma,
                             void* hip_stream, dose_sell* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    check_sigma(sigma);
    validate_csr(csr, vf, xf);
    const bool runs = xf == DOSE_IDX_RUNS;
    hipStream_t s = as_stream(hip_stream);
    const int64_t* rp = csr->row_ptr;
    auto m = std::make_unique<dose_sell_s>();
    HIP_CHECK(hipGetDevice(&m->device));
    m->vf = vf;
    m->xf = xf;
    m->sigma = sigma;
    m->n_rows = csr->n_rows;
    m->n_cols = csr->n_cols;
    m->nnz = csr->nnz;
    m->idx_bytes = runs ? 0 : xf == DOSE_IDX_U16 ? 2 : 4;
    SellLayout L = sell_layout(rp, csr->n_rows, sigma);
    m->n_chunks = static_cast<int64_t>(L.width.size());
    m->n_groups = (m->n_chunks + kSellGroupChunks - 1) / kSellGroupChunks;
    if (m->n_groups > INT32_MAX) fail(DOSE_ERR_UNSUPPORTED, "too many chunks");
    const int64_t n_pos = m->n_groups * kSellGroupRows, n_ch = m->n_groups * kSellGroupChunks;
    // positions: row, length and first entry (padding positions: no row)
    m->h_perm.assign(static_cast<size_t>(n_pos), 0xFFFFFFFFu);
    m->h_len.assign(static_cast<size_t>(n_pos), 0u);
    std::vector<uint64_t> start(static_cast<size_t>(n_pos), 0);
    for (int64_t i = 0; i < m->n_rows; ++i) {
      const uint32_t r = L.perm[i];
      m->h_perm[i] = r;
      m->h_len[i] = static_cast<uint32_t>(rp[r + 1] - rp[r]);
      start[i] = static_cast<uint64_t>(rp[r]);
    }
    // chunks: slices and shortest row
    m->h_chunks.assign(static_cast<size_t>(n_ch), SellChunk{});
    m->h_width = L.width;
    uint64_t slices = 0;
    for (int64_t c = 0; c < n_ch; ++c) {
      SellChunk& ch = m->h_chunks[c];
      const int64_t w = c < m->n_chunks ? L.width[c] : 0;
      m->std_slots += kSellC * w;
      ch.slice0 = static_cast<uint32_t>(slices);
      ch.n_slices = static_cast<uint32_t>((w + kSellLaneEntries - 1) / kSellLaneEntries);
      uint32_t mn = 0xFFFFFFFFu;
      for (int i = 0; i < kSellC; ++i) mn = std::min(mn, m->h_len[c * kSellC + i]);
      ch.min_len = mn;
      slices += ch.n_slices;
      if (slices >= uint64_t{0xFFFFFFFF}) fail(DOSE_ERR_UNSUPPORTED, "SELL storage beyond 2^32 slices");
    }
    m->n_slices = static_cast<int64_t>(slices);
    // group windows: every entry's column lies in [first column, last column]
    // of its row (columns ascend), so the rows' ends bound the window
    std::vector<uint32_t> win(static_cast<size_t>(2 * m->n_groups), 0u), pad_col(static_cast<size_t>(m->n_groups), 0u);
    const int64_t cap = window_cap_floats();
    int64_t wf[3] = {0, 0, 0};
    for (int64_t g = 0; g < m->n_groups; ++g) {
      int64_t lo = INT64_MAX, hi = -1;
      for (int64_t i = g * kSellGroupRows; i < (g + 1) * kSellGroupRows; ++i) {
        if (m->h_len[i] == 0) continue;
        const uint32_t r = m->h_perm[i];
        lo = std::min<int64_t>(lo, csr->col_idx[rp[r]]);
        hi = std::max<int64_t>(hi, csr->col_idx[rp[r + 1] - 1]);
      }
      if (hi < 0) continue;
      const int64_t cmin = lo & ~int64_t{kWinAlign - 1};
      const int64_t clen = hi - cmin + 1;
      win[2 * g] = static_cast<uint32_t>(cmin);
      win[2 * g + 1] = static_cast<uint32_t>(clen);
      pad_col[g] = static_cast<uint32_t>(cmin);
      if (clen <= cap) ++m->n_windowed;
      // as for CSR row groups, the cap scales with the vectors, up to the
      // largest SELL window (a launch's LDS is sized for its widest window)
      for (int i = 0; i < 3; ++i) {
        const int64_t f = clen << i;
        if (f <= std::min<int64_t>(cap << i, kSellWinFloatsMax)) wf[i] = std::max(wf[i], f);
      }
    }
    for (int i = 0; i < 3; ++i) m->win_floats[i] = static_cast<int32_t>((wf[i] + 3) / 4 * 4);
    // run-length indices: every position's maximal runs of consecutive
    // columns, as (end position in the row, column - position)
    std::vector<uint32_t> h_run_ptr;
    std::vector<SellRun> h_runs;
    if (runs) {
      std::vector<uint64_t> cnt(static_cast<size_t>(n_pos) + 1, 0);
      // rows split among host threads (each position's runs depend on its row only)
      const int64_t parts = std::max<int64_t>(1, std::min<int64_t>(16, m->n_rows / 65536));
      auto in_parallel = [&](auto&& body) {
        if (parts == 1) return body(int64_t{0}, m->n_rows);
        std::vector<std::thread> th;
        for (int64_t q = 0; q < parts; ++q) th.emplace_back(body, m->n_rows * q / parts, m->n_rows * (q + 1) / parts);
        for (auto& t : th) t.join();
      };
      in_parallel([&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
          const uint32_t r = m->h_perm[i];
          uint64_t n = rp[r + 1] > rp[r] ? 1 : 0;
          for (int64_t k = rp[r] + 1; k < rp[r + 1]; ++k) n += csr->col_idx[k] != csr->col_idx[k - 1] + 1;
          cnt[i + 1] = n;
        }
      });
      for (int64_t i = 0; i < n_pos; ++i) cnt[i + 1] += cnt[i];
      if (cnt[n_pos] >= uint64_t{0xFFFFFFFF}) fail(DOSE_ERR_UNSUPPORTED, "more than 2^32 - 2 runs");
      m->n_runs = static_cast<int64_t>(cnt[n_pos]);
      h_run_ptr.assign(cnt.begin(), cnt.end());
      h_runs.resize(static_cast<size_t>(std::max<int64_t>(m->n_runs, 1)));
      in_parallel([&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
          const uint32_t r = m->h_perm[i];
          uint64_t o = cnt[i];
          for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
            const int32_t pos = static_cast<int32_t>(k - rp[r]);
            if (k > rp[r] && csr->col_idx[k] == csr->col_idx[k - 1] + 1) {
              h_runs[o - 1].end = pos + 1;
            } else {
              h_runs[o].end = pos + 1;
              h_runs[o].delta = csr->col_idx[k] - pos;
              ++o;
            }
          }
        }
      });
      for (int64_t g = 0; g < m->n_groups; ++g) {
        const int64_t nr = static_cast<int64_t>(cnt[(g + 1) * kSellGroupRows] - cnt[g * kSellGroupRows]);
        if (nr > kSellMaxGroupRuns)
          fail(DOSE_ERR_UNSUPPORTED, "run-length indices: more than " + std::to_string(kSellMaxGroupRuns) +
                                         " runs in one chunk of 64 rows");
        m->lds_runs = std::max<int32_t>(m->lds_runs, static_cast<int32_t>(nr));
      }
    }
    // device: A's CSR streams, then the scatter into the slice layout
    auto A = upload_encode_A(csr, vf, runs ? DOSE_IDX_I32 : xf, s);
    const int vb = value_bytes(vf);
    const size_t n_ent = static_cast<size_t>(m->n_slices + 1) * kSellSliceEntries;
    m->val = DevBuf(n_ent * vb);
    m->col = DevBuf(n_ent * m->idx_bytes);
    if (runs) {
      m->run_ptr = DevBuf(h_run_ptr.size() * sizeof(uint32_t));
      m->runs = DevBuf(h_runs.size() * sizeof(SellRun));
      HIP_CHECK(hipMemcpyAsync(m->run_ptr.get(), h_run_ptr.data(), m->run_ptr.bytes(), hipMemcpyHostToDevice, s));
      HIP_CHECK(hipMemcpyAsync(m->runs.get(), h_runs.data(), m->runs.bytes(), hipMemcpyHostToDevice, s));
    }
    m->chunks = DevBuf(m->h_chunks.size() * sizeof(SellChunk));
    // the launch's work: chunks holding entries, then those without
    std::vector<uint32_t> work;
    work.reserve(static_cast<size_t>(n_ch));
    for (int64_t c = 0; c < n_ch; ++c)
      if (m->h_chunks[c].n_slices > 0) work.push_back(static_cast<uint32_t>(c));
    m->n_work = static_cast<int64_t>(work.size());
    for (int64_t c = 0; c < n_ch; ++c)
      if (m->h_chunks[c].n_slices == 0) work.push_back(static_cast<uint32_t>(c));
    m->n_zero = n_ch - m->n_work;
    m->work = DevBuf(std::max<size_t>(work.size(), 1) * sizeof(uint32_t));
    if (!work.empty())
      HIP_CHECK(hipMemcpyAsync(m->work.get(), work.data(), work.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    m->win = DevBuf(win.size() * sizeof(uint32_t));
    m->perm = DevBuf(static_cast<size_t>(n_pos) * sizeof(uint32_t));
    m->len = DevBuf(static_cast<size_t>(n_pos) * sizeof(uint32_t));
    DevBuf d_start(static_cast<size_t>(n_pos) * sizeof(uint64_t)), d_pad(pad_col.size() * sizeof(uint32_t));
    HIP_CHECK(hipMemsetAsync(m->val.get(), 0, m->val.bytes(), s));
    HIP_CHECK(hipMemsetAsync(m->col.get(), 0, m->col.bytes(), s));
    HIP_CHECK(hipMemcpyAsync(m->chunks.get(), m->h_chunks.data(), m->chunks.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(m->win.get(), win.data(), m->win.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(m->perm.get(), m->h_perm.data(), m->perm.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(m->len.get(), m->h_len.data(), m->len.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(d_start.get(), start.data(), d_start.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(d_pad.get(), pad_col.data(), d_pad.bytes(), hipMemcpyHostToDevice, s));
    HIP_CHECK(launch_sell_pack(vf, runs ? 4 : m->idx_bytes, m->chunks.get<SellChunk>(), n_ch, d_start.get<uint64_t>(),
                               m->len.get<uint32_t>(), d_pad.get<uint32_t>(), A->A.val.get(), A->A.col.get(),
                               m->val.get(), runs ? nullptr : m->col.get(), s));
    HIP_CHECK(hipStreamSynchronize(s));
    m->row_scale = std::move(A->row_scale);
    *out = m.release();
  });
}

dose_status dose_sell_info(dose_sell m, dose_sell_info_t* info) {
  return guarded([&] {
    if (!m || !info) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_rows = m->n_rows;
    info->n_cols = m->n_cols;
    info->nnz = m->nnz;
    info->value_format = m->vf;
    info->index_format = m->xf;
    info->chunk_rows = kSellC;
    info->sigma = m->sigma;
    info->n_chunks = m->n_chunks;
    info->n_groups = m->n_groups;
    info->n_groups_windowed = m->n_windowed;
    info->std_slots = m->std_slots;
    info->n_runs = m->n_runs;
    info->stored_slots = m->n_slices * kSellSliceEntries;
    info->device_bytes = m->val.bytes() + m->col.bytes() + m->chunks.bytes() + m->win.bytes() + m->perm.bytes() +
                         m->len.bytes() + m->row_scale.bytes() + m->run_ptr.bytes() + m->runs.bytes() +
                         m->work.bytes();
    const uint64_t per = static_cast<uint64_t>(value_bytes(m->vf)) + static_cast<uint64_t>(m->idx_bytes);
    const uint64_t scale_b = m->vf == kFp8 ? 4 : 0;
    const uint64_t nr = static_cast<uint64_t>(m->n_rows), nc = static_cast<uint64_t>(m->n_cols);
    const uint64_t run_b = 8 * static_cast<uint64_t>(m->n_runs);
    info->spmv_bytes = static_cast<uint64_t>(m->nnz) * per + run_b + (nr + 1) * 4 + nr * scale_b + 4 * nc + 4 * nr;
    info->stream_bytes = static_cast<uint64_t>(info->stored_slots) * per + nr * 8 + (m->idx_bytes ? 0 : run_b + nr * 4) +
                         nr * scale_b + 4 * nc + 4 * nr;
  });
}

dose_status dose_sell_decode(dose_sell m, int64_t* perm, int64_t* width, float* val, int32_t* col) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    if (m->n_rows > 0 && (!perm || !width)) fail(DOSE_ERR_INVALID_ARGUMENT, "null perm or width");
    if (m->std_slots > 0 && (!val || !col)) fail(DOSE_ERR_INVALID_ARGUMENT, "null val or col");
    for (int64_t i = 0; i < m->n_rows; ++i) perm[i] = m->h_perm[i];
    for (int64_t c = 0; c < m->n_chunks; ++c) width[c] = m->h_width[c];
    if (m->std_slots == 0) return;
    DeviceGuard g(m->device);
    const size_t n_ent = static_cast<size_t>(m->n_slices) * kSellSliceEntries;
    DevBuf dec(n_ent * sizeof(float));
    HIP_CHECK(launch_sell_decode(m->vf, m->chunks.get<SellChunk>(), m->n_groups * kSellGroupChunks,
                                 m->perm.get<uint32_t>(), m->len.get<uint32_t>(), m->val.get(),
                                 m->row_scale.get<float>(), dec.get<float>(), nullptr));
    HIP_CHECK(hipDeviceSynchronize());
    std::vector<float> hv(n_ent);
    HIP_CHECK(hipMemcpy(hv.data(), dec.get(), n_ent * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<int32_t> hc(n_ent);
    if (m->idx_bytes == 0) {
      // columns from the device's runs: position + delta of the run holding it
      std::vector<uint32_t> hrp(static_cast<size_t>(m->n_groups) * kSellGroupRows + 1);
      std::vector<SellRun> hr(static_cast<size_t>(std::max<int64_t>(m->n_runs, 1)));
      HIP_CHECK(hipMemcpy(hrp.data(), m->run_ptr.get(), hrp.size() * 4, hipMemcpyDeviceToHost));
      HIP_CHECK(hipMemcpy(hr.data(), m->runs.get(), hr.size() * sizeof(SellRun), hipMemcpyDeviceToHost));
      for (int64_t c = 0; c < m->n_chunks; ++c)
        for (int i = 0; i < kSellC; ++i) {
          const int64_t p = c * kSellC + i;
          uint32_t q = hrp[p];
          for (uint32_t j = 0; j < m->h_len[p]; ++j) {
            while (q + 1 < hrp[p + 1] && static_cast<int64_t>(j) >= hr[q].end) ++q;
            const size_t dst = (static_cast<size_t>(m->h_chunks[c].slice0) + j / kSellLaneEntries) * kSellSliceEntries +
                               static_cast<size_t>(i) * kSellLaneEntries + j % kSellLaneEntries;
            hc[dst] = static_cast<int32_t>(j) + hr[q].delta;
          }
        }
    } else if (m->idx_bytes == 4) {
      // the two halves of each slice (sell_slot) back into a row's 8 entries together
      std::vector<int32_t> raw(n_ent);
      HIP_CHECK(hipMemcpy(raw.data(), m->col.get(), n_ent * 4, hipMemcpyDeviceToHost));
      for (size_t sl = 0; sl < n_ent / kSellSliceEntries; ++sl)
        for (int i = 0; i < kSellC; ++i)
          for (int e = 0; e < kSellLaneEntries; ++e)
            hc[sl * kSellSliceEntries + static_cast<size_t>(i) * kSellLaneEntries + e] =
                raw[sl * kSellSliceEntries + sell_slot(4, i, e)];
    } else {
      std::vector<uint16_t> h16(n_ent);
      HIP_CHECK(hipMemcpy(h16.data(), m->col.get(), n_ent * 2, hipMemcpyDeviceToHost));
      for (size_t k = 0; k < n_ent; ++k) hc[k] = h16[k];
    }
    // Kreutzer's layout: entry j of the row at chunk position i at
    // off_c + j * 64 + i; slots past the row's end hold 0 and column -1
    int64_t off = 0;
    for (int64_t c = 0; c < m->n_chunks; ++c) {
      const SellChunk& ch = m->h_chunks[c];
      for (int64_t j = 0; j < m->h_width[c]; ++j)
        for (int i = 0; i < kSellC; ++i) {
          const int64_t slot = off + j * kSellC + i;
          const uint32_t L = m->h_len[c * kSellC + i];
          const size_t src = (static_cast<size_t>(ch.slice0) + static_cast<size_t>(j / kSellLaneEntries)) *
                                 kSellSliceEntries + static_cast<size_t>(i) * kSellLaneEntries +
                             static_cast<size_t>(j % kSellLaneEntries);
          val[slot] = j < L ? hv[src] : 0.0f;
          col[slot] = j < L ? hc[src] : -1;
        }
      off += kSellC * m->h_width[c];
    }
  });
}

dose_status dose_sell_runs(dose_sell m, int64_t* run_ptr, int32_t* start, int32_t* length) {
  return guarded([&] {
    if (!m || !run_ptr) fail(DOSE_ERR_INVALID_ARGUMENT, "null argument");
    if (m->idx_bytes != 0) fail(DOSE_ERR_INVALID_ARGUMENT, "the matrix has no run-length indices");
    if (m->n_runs > 0 && (!start || !length)) fail(DOSE_ERR_INVALID_ARGUMENT, "null start or length");
    DeviceGuard g(m->device);
    std::vector<uint32_t> hrp(static_cast<size_t>(m->n_groups) * kSellGroupRows + 1);
    std::vector<SellRun> hr(static_cast<size_t>(std::max<int64_t>(m->n_runs, 1)));
    HIP_CHECK(hipMemcpy(hrp.data(), m->run_ptr.get(), hrp.size() * 4, hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(hr.data(), m->runs.get(), hr.size() * sizeof(SellRun), hipMemcpyDeviceToHost));
    // by row: position p holds row h_perm[p]
    std::vector<int64_t> pos_of(static_cast<size_t>(m->n_rows));
    for (int64_t p = 0; p < m->n_rows; ++p) pos_of[m->h_perm[p]] = p;
    run_ptr[0] = 0;
    for (int64_t r = 0; r < m->n_rows; ++r) {
      const int64_t p = pos_of[r];
      int64_t o = run_ptr[r];
      int32_t begin = 0;
      for (uint32_t q = hrp[p]; q < hrp[p + 1]; ++q) {
        start[o] = begin + hr[q].delta;
        length[o] = hr[q].end - begin;
        begin = hr[q].end;
        ++o;
      }
      run_ptr[r + 1] = o;
    }
  });
}

dose_status dose_sell_spmv(dose_sell m, const float* x, float* y, void* hip_stream) {
  return guarded([&] {
    check_sell_product(m, 1, x, y);
    DeviceGuard g(m->device);
    HIP_CHECK(launch_sell_spmv(m->vf, m->vf == kFp8 ? kScaleRow : kScaleNone, 1, sell_args(m, 1, x, y),
                               as_stream(hip_stream)));
  });
}

dose_status dose_sell_spmv_f64(dose_sell m, const double* x, double* y, void* hip_stream) {
  return guarded([&] {
    if (!m) fail(DOSE_ERR_INVALID_ARGUMENT, "matrix is null");
    if ((m->n_cols > 0 && !x) || (m->n_rows > 0 && !y)) fail(DOSE_ERR_INVALID_ARGUMENT, "null x or y");
    if (overlaps(x, m->n_cols * 8, y, m->n_rows * 8)) fail(DOSE_ERR_INVALID_ARGUMENT, "x and y overlap");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 8 != 0)
      fail(DOSE_ERR_INVALID_ARGUMENT, "x and y must be 8-byte aligned");
    if (m->n_cols > INT32_MAX / 2) fail(DOSE_ERR_UNSUPPORTED, "n_cols must stay below 2^30");
    DeviceGuard g(m->device);
    HIP_CHECK(launch_sell_spmv_f64(m->vf, m->vf == kFp8 ? kScaleRow : kScaleNone, sell_args(m, 2, x, y),
                                   as_stream(hip_stream)));
  });
}

dose_status dose_sell_spmv_multi(dose_sell m, int32_t n_rhs, const float* x, float* y, void* hip_stream) {
  return guarded([&] {
    check_sell_product(m, n_rhs, x, y);
    DeviceGuard g(m->device);
    HIP_CHECK(launch_sell_spmv(m->vf, m->vf == kFp8 ? kScaleRow : kScaleNone, n_rhs, sell_args(m, n_rhs, x, y),
                               as_stream(hip_stream)));
  });
}

dose_status dose_sell_batch_plan_create(const dose_sell_batch_item* items, int32_t n_items, uint32_t flags,
                                        void* hip_stream, dose_batch_plan* out) {
  return guarded([&] {
    if (!out) fail(DOSE_ERR_INVALID_ARGUMENT, "out is null");
    *out = nullptr;
    if (flags != 0) fail(DOSE_ERR_INVALID_ARGUMENT, "unknown flags");
    check_sell_items(items, n_items);
    DeviceGuard g(items[0].S->device);
    std::unique_ptr<dose_batch_plan_s> p(build_sell_plan(items, n_items, as_stream(hip_stream)));
    capture_plan(p.get());
    *out = p.release();
  });
}

dose_status dose_sell_destroy(dose_sell m) {
  return guarded([&] {
    if (!m) return;
    {
      DeviceGuard g(m->device);
      (void)hipDeviceSynchronize();
    }
    delete m;
  });
}

}  // extern "C"
