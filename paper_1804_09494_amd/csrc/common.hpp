// Shared host-side definitions of the tucker_hip library: the context, device
// buffers, error plumbing and launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tucker_hip.h"

namespace tk {

// Error carried out of internal functions and turned into a tk_status at the ABI.
struct Error {
  tk_status status;
  std::string msg;
};

[[noreturn]] inline void fail(tk_status s, const std::string& msg) { throw Error{s, msg}; }

#define TK_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      ::tk::fail(TK_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define TK_CHECK_LAUNCH() TK_HIP(hipGetLastError())

#define TK_REQUIRE(cond, status, msg) \
  do {                                \
    if (!(cond)) ::tk::fail(status, msg); \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// HOOI failure flags (int32, device): [0] the current mode's bits (1 = a
// Cholesky pivot failed, 2 = a column below the rank floor), [1] 1 + the first
// failed mode of a deferred invocation, [FLAG_BITS + n] mode n's bits, and
// [FLAG_KVALID + n] mode n's number of columns above the floor.
constexpr int FLAG_BITS = 2;
constexpr int FLAG_KVALID = FLAG_BITS + 8;
constexpr int FLAG_INTS = FLAG_KVALID + 8;
constexpr int FIX_CHUNK = 128;  // partial rows summed per fixup block (one tree level for up to 16K)

struct Ctx;

// Device allocation owned by a Buf; freed on destruction.  Allocation goes
// through the context so mem_limit_bytes is enforced.
class Buf {
 public:
  Buf() = default;
  Buf(Ctx* c, size_t bytes) { alloc(c, bytes); }
  ~Buf() { release(); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : ctx_(o.ctx_), p_(o.p_), bytes_(o.bytes_) { o.p_ = nullptr; o.bytes_ = 0; }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) { release(); ctx_ = o.ctx_; p_ = o.p_; bytes_ = o.bytes_; o.p_ = nullptr; o.bytes_ = 0; }
    return *this;
  }
  void alloc(Ctx* c, size_t bytes);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return bytes_; }
  explicit operator bool() const { return p_ != nullptr; }

 private:
  Ctx* ctx_ = nullptr;
  void* p_ = nullptr;
  size_t bytes_ = 0;
};

// Per-mode plan: the Lite partition, the mode-sorted copy of the tensor and
// the fixup table of slices shared by several bins.
struct ModePlan {
  int64_t L = 0;          // mode length
  int64_t L_nz = 0;       // nonempty slices = rows of compact Y
  int64_t P = 0, limit = 0, n_stage1 = 0, M2 = 0;
  int64_t S = 0;          // segments (= R_sum)
  int64_t n_bad = 0, n_slots = 0, E_max = 0, R_max = 0;
  int64_t khat = 0;
  int rows_cap = 0;       // LDS rows per bin the TTM kernel was sized for
  bool whole_slices = false;  // CoarseG: bins of whole slices, of any size (vector-ALU kernel only)
  Buf row_slice;          // int32[L_nz]  slice id of each compact row (ascending)
  Buf row_of;             // int32[L]     compact row of each slice id (valid for nonempty slices)
  Buf label;              // int32[L]     storage row of each index in the working factor copies:
                          //              descending slice size (hot rows packed first)
  Buf bin_ptr;            // int64[P+1]
  Buf seg_ptr;            // int32[P+1]
  Buf seg_row;            // int32[S]     compact row of each segment
  Buf seg_begin;          // int64[S+1]
  Buf seg_slot;           // int32[S]     -1 = good, else partial-row slot
  // The TTM-chain streams a padded copy of the layout: every segment is padded
  // to a multiple of 4 elements with zero-valued elements (coordinate 0), so an
  // MFMA step over 4 consecutive elements never straddles two slices.
  int64_t m_pad = 0;      // padded layout length
  int64_t E_pad_max = 0;  // largest padded bin
  Buf bin_pptr;           // int64[P+1]   padded bin offsets
  Buf seg_pbegin;         // int64[S+1]   padded segment offsets
  Buf order_pad;          // uint32[m_pad] element index at each padded position (0xffffffff = padding)
  Buf bad_row;            // int32[n_bad]
  Buf bad_slot;           // int32[n_bad+1] slots of bad slice k: [bad_slot[k], bad_slot[k+1])
  // Fixup tree over the rows of the partial buffer (rows [0, n_slots) are the
  // slots; each level appends the sums of runs of at most FIX_CHUNK rows of
  // one slice, until every slice has at most FIX_CHUNK rows left).
  std::vector<int64_t> fix_n;   // rows added by each level
  Buf fix_lohi;                 // int32 per level: [lo | hi] row ranges summed by that level's rows
  Buf fix_fin;                  // int32[2 n_bad]: [lo | hi] rows summed into Y for bad slice k
  int64_t fix_rows = 0;         // n_slots + all level rows
  Buf lay_idx[7];         // int32[m_pad] other modes' coordinates in padded layout order (modes ascending)
  Buf lay_val;            // float[m_pad]
  Buf elem_order;         // uint32[m] canonical element index per layout position (optional)
};

// Element-sized work buffers of the slice sort (keys and positions before
// and after, and the radix sort's temporary storage).  The modes of one
// partition build reuse them instead of allocating and freeing them per mode:
// at 2e9 elements a fresh allocation of this size costs the runtime 0.3-0.5 s.
struct SortScratch {
  Buf key, skey, perm, sperm, tmp;
};

struct Timings {
  std::vector<std::string> names;
  std::vector<double> ms;
  void clear() { names.clear(); ms.clear(); }
  void add(const std::string& n, double v) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) { ms[i] += v; return; }
    names.push_back(n);
    ms.push_back(v);
  }
};

// Event counts of the adaptive parts of the path (tk_get_counters).
struct Counters {
  int64_t eig_krylov_solves = 0;     // block-Krylov eigensolves
  int64_t eig_krylov_cycles = 0;     // their restart cycles
  int64_t eig_dense_fallbacks = 0;   // Krylov results replaced by the dense solver (not accepted)
  int64_t rank_completions = 0;      // factors completed after a rank-deficient penultimate matrix
};

// A streamed load in progress (tk_load_coo_begin .. tk_load_coo_end): the raw
// element list, filled append by append.
struct LoadState {
  bool active = false;
  int N = 0;
  int64_t dims[8] = {0};
  int64_t nnz = 0, filled = 0;
  unsigned flags = 0;
  Buf raw[8];             // int32[nnz] per mode, input order
  Buf rawv;               // float[nnz]
  Buf flag;               // int32: 1 = coordinate out of range, 2 = NaN/Inf value
};

struct ObsSet {
  int N = 0;
  int64_t n_obs = 0;
  int64_t dims[8] = {0};
  int32_t K[8] = {0};
  Buf idx[8];  // int32[n_obs], input order
  ModePlan plan[8];  // Lite partition of the observations along each mode (adjoint TTM-chain)
  Buf F32[8];        // padded FP32 copies of the caller's factors
  int kp[8] = {0};
  Buf gl;            // float[n_obs] upstream gradient in one mode's layout order
  Buf Yg;            // float[max R_n x Khat_n]
  Buf G32;           // float[prod K] core copy
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  tk_options opt{};
  std::string last_error;
  int64_t bytes_in_use = 0;
  tk_allocator allocator{};   // all-null: hipMalloc / hipFree
  int cu_count = 256;
  size_t lds_per_block = 65536;

  // tensor
  int N = 0;
  int64_t dims[8] = {0};
  int64_t m = 0;
  double norm_sq = 0.0;
  Buf idx_c[8];           // int32[m] canonical order
  Buf val_c;              // float[m]
  bool have_tensor = false;
  LoadState load;
  Buf slice_order[8];     // int32[L_n] caller-given random slice order (CoarseG)

  // ranks / plans / factors
  int32_t K[8] = {0};
  bool have_ranks = false;
  ModePlan plan[8];
  Buf F64[8];             // double[L_n x K_n]
  Buf F32[8];             // float [L_n x Kp_n], Kp_n = padded row stride
  int kp32[8] = {0};      // FP32 row stride

  // work buffers (grown on demand)
  Buf Y;                  // float [max R_n x Khat_n]
  Buf Ybf16;              // bf16 copy of Y (precision form)
  Buf partial;            // float [slots x Khat]
  Buf work;               // general scratch
  Buf gram_part;          // float/double partial Grams
  Buf gram64;             // double[Khat x Khat]
  Buf ybf;                // BF16 copy of Y in MFMA operand order (wide BF16 Gram)
  Buf eig_val;            // double[Khat]
  Buf U64;                // double[R_n x K_n]
  Buf small64;            // double scratch for K x K matrices, reductions
  Buf kr_work;            // block-Krylov eigensolver workspace (large Khat)
  Buf mf_work;            // matrix-free eigensolve: Y X and the row-range partials of Y^T (Y X)
  Buf diag64;             // diag(Y^T Y) on the matrix-free route
  Buf eig_warm[8];        // last eigenvectors of each mode's Gram (Krylov warm start)
  int eig_warm_k[8] = {0};
  bool fac_dirty[8] = {true, true, true, true, true, true, true, true};   // rows of empty slices may be nonzero
  Buf unit_rows[8];       // int32: rows of empty slices a completion set to unit vectors (device)
  int n_unit_rows[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // how many; the next factor step zeroes them
  Buf core64;             // double[prod K]
  Buf flag;               // int32 flags

  Timings timings;
  Counters counters;
  bool completed_once = false;   // a factor of this tensor was completed (rank deficiency) at least once
  hipEvent_t ev_ttm[2] = {nullptr, nullptr};  // when set, bracket the TTM-chain kernel launch
  ObsSet obs;
  bool have_obs = false;

  void* alloc_raw(size_t bytes);
  void free_raw(void* p, size_t bytes);
  void sync() { TK_HIP(hipStreamSynchronize(stream)); }
  // Krylov acceptance: a positive eig_tol bounds the estimated subspace error;
  // 0 accepts a residual at the FP32 input's rounding level (4 u)
  bool krylov_accepts(double res, double err) const {
    return opt.eig_tol > 0.0 ? err <= opt.eig_tol : res <= 4.0 / 16777216.0;
  }
};

inline void Buf::alloc(Ctx* c, size_t bytes) {
  release();
  ctx_ = c;
  bytes_ = bytes;
  p_ = bytes ? c->alloc_raw(bytes) : nullptr;
}

inline void Buf::release() {
  if (p_ && ctx_) ctx_->free_raw(p_, bytes_);
  p_ = nullptr;
  bytes_ = 0;
}

// Grow-only reuse of a work buffer.
inline void ensure(Ctx* c, Buf& b, size_t bytes) {
  if (b.bytes() < bytes) b.alloc(c, bytes);
}

template <class T>
inline void h2d(Ctx* c, T* dst, const T* src, size_t n) {
  if (n) TK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
}
template <class T>
inline void d2h(Ctx* c, T* dst, const T* src, size_t n) {
  if (n) TK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
}
template <class T>
inline void d2d(Ctx* c, T* dst, const T* src, size_t n) {
  if (n) TK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
}
template <class T>
inline void copy_out(Ctx* c, T* dst, const T* src, size_t n, tk_mem mem) {
  if (!n) return;
  TK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T),
                        mem == TK_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
}
template <class T>
inline void copy_in(Ctx* c, T* dst, const T* src, size_t n, tk_mem mem) {
  if (!n) return;
  TK_HIP(hipMemcpyAsync(dst, src, n * sizeof(T),
                        mem == TK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c->stream));
}

// Launch-size helper for grid-stride kernels.
// Buffer-resource loads: a byte offset at or beyond the resource's size returns
// zero without touching memory, so edge tiles load with a computed offset and no
// branch (a predicated global load becomes a branch and a full wait).
constexpr uint32_t BUF_OOB = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

inline unsigned grid_for(int64_t n, int block, int64_t cap = 65536) {
  int64_t g = ceil_div(n > 0 ? n : 1, block);
  return (unsigned)(g < cap ? g : cap);
}

// ---- primitives (prim.hip, rocPRIM) ----
// tmp: grow-only temporary storage kept by the caller (nullptr: allocated per call)
void sort_pairs_u32(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout,
                    int64_t n, int end_bit, Buf* tmp = nullptr);
void sort_pairs_u64_u32(Ctx* c, const uint64_t* kin, uint64_t* kout, const uint32_t* vin, uint32_t* vout,
                        int64_t n, int end_bit);
void sort_pairs_u32_key(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, int64_t n,
                        int end_bit);
void sort_pairs_u32_key(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint64_t* vin, uint64_t* vout, int64_t n,
                        int end_bit);
void exclusive_scan_pos(Ctx* c, const uint32_t* in, uint32_t* out, int64_t n);
void exclusive_scan_pos(Ctx* c, const uint64_t* in, uint64_t* out, int64_t n);
void exclusive_scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n);
void inclusive_scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n);
void exclusive_scan_i32(Ctx* c, const int32_t* in, int32_t* out, int64_t n);
void reduce_max_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n);
void reduce_min_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n);

// ---- stages ----
void load_begin(Ctx* c, int N, const int64_t* dims, int64_t nnz, unsigned flags);
void load_append(Ctx* c, int64_t count, const int32_t* const* idx, const float* vals, tk_mem mem);
void load_end(Ctx* c);
// ss: the sort's work buffers, shared by the modes of one build; last: the
// build's final mode, which releases them as soon as it no longer needs them
void build_plan(Ctx* c, ModePlan& pl, int N, int n, const int64_t* dims, int64_t m, Buf* idx, const float* vals,
                int64_t khat, int tile_w, int64_t wg_default, bool keep_order, SortScratch& ss, bool last,
                const int32_t* coarse_order = nullptr);
void relabel_layout(Ctx* c, ModePlan& pl, int N, int n, const ModePlan* plans, int64_t m);
void export_partition(Ctx* c, ModePlan& pl, int64_t m, int64_t* bin_ptr, int64_t* elem_order, int32_t* seg_bin,
                      int32_t* seg_slice, int64_t* seg_begin, uint8_t* seg_bad, tk_mem mem);
int ttm_rows_cap(Ctx* c, int64_t tile_w);
int ttm_tile_width(int N, const int32_t* K, int n);
int64_t ttm_default_bin_nnz(int N, const int32_t* K, int n, int kernel);
bool ttm_uses_mfma(int N, const int32_t* K, int n, const int* kp);
bool ttm_uses_mfma4(int N, const int32_t* K, int n, const int* kp);
bool ttm_takes_mfma3(const Ctx* c, const ModePlan& pl, int N, int n, const int32_t* K, const int* kp);
void refresh_factor_copies(Ctx* c, int n);
// val_order non-null: lay_val is indexed through it (layout position p takes
// lay_val[val_order[p]], 0xffffffff giving zero); only where the three-mode
// matrix-core kernel runs (ttm_uses_mfma).
void ttm_run(Ctx* c, const ModePlan& pl, int N, int n, const int32_t* K, const float* const* F32, const int* kp,
             const float* lay_val, int64_t m, float* Y, bool bf16 = false, float* partial = nullptr,
             const uint32_t* val_order = nullptr);
void ttm_chain(Ctx* c, int n, float* Y, bool bf16, float* partial = nullptr);
void noalloc_scratch_init(int device);
void ttm_chain_noalloc(Ctx* c, int n, float* Y);
void hooi_iterate(Ctx* c, int iters, double* fits);
void core_and_fit(Ctx* c, double* core_dev, double* fit);

}  // namespace tk
