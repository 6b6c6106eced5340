// The C ABI (include/tucker_hip.h) and the HOOI driver.
//
// HOOI invocation (Section 2.2 and its figure), one mode at a time:
//   Y_(n) = TTM-chain of T with the other factors (eq. 1)      -> ttm.hip
//   G     = Y^T Y on the matrix cores                           -> gram.hip
//   leading K_n eigenpairs of G in FP64 (tridiagonal + bisection) -> eig.hip
//   F_n   = orthonormalised Y V_K S_K^-1 (CholeskyQR2, FP64)    -> factor.hip
// After the last mode the core G_(N) = F_N^T Y_(N) and the fit  -> core.hip
// Gauss-Seidel by default: mode n uses factors already refined in this
// invocation; the Jacobi option uses the invocation's input factors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.hpp"

namespace tk {

void gram(Ctx* c, const float* Y, int64_t R, int khat, double* G, bool bf16);
void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK, int mode);
void eig_topk_matfree(Ctx* c, const float* Y, int64_t R, int khat, int K, double* lam_k, double* VK, int mode,
                      double* diag);
bool form_factor(Ctx* c, int n, const float* Y, int64_t R, int khat, const double* gdiag, int64_t dstride,
                 const double* lam_k,
                 const double* VK, int* flag_dev, bool deferred);
void complete_factor(Ctx* c, int n, int g);
int computed_columns(Ctx* c, const int* flag_dev, int n);
void core_from_last(Ctx* c, const float* Y, double* core, double* out2);
void obs_eval(Ctx* c, const float* core, const float* const* F, float* model, tk_mem mem);
void obs_adjoint(Ctx* c, const float* g, const float* core, const float* const* F, float* dcore, float* const* dF,
                 tk_mem mem);
void load_obs(Ctx* c, int N, const int64_t* dims, const int32_t* ranks, int64_t n_obs, const int32_t* const* idx,
              tk_mem mem);

void* Ctx::alloc_raw(size_t bytes) {
  if (opt.mem_limit_bytes > 0 && bytes_in_use + (int64_t)bytes > opt.mem_limit_bytes)
    fail(TK_ERR_OOM, "allocation of " + std::to_string(bytes) + " bytes exceeds mem_limit_bytes");
  void* p = nullptr;
  if (allocator.alloc) {
    p = allocator.alloc(bytes, allocator.user);
    if (!p) fail(TK_ERR_OOM, "the allocator hook returned no memory for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(TK_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  bytes_in_use += (int64_t)bytes;
  return p;
}

void Ctx::free_raw(void* p, size_t bytes) {
  if (p) {
    if (allocator.free)
      allocator.free(p, bytes, allocator.user);
    else
      (void)hipFree(p);
    bytes_in_use -= (int64_t)bytes;
  }
}

static int64_t khat_of(const Ctx* c, int n) {
  int64_t k = 1;
  for (int j = 0; j < c->N; ++j)
    if (j != n) k *= c->K[j];
  return k;
}

// ---- events for per-step timings --------------------------------------------------------------

struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e;
      // timing only: no system-scope fence (its cache write-back costs ~5 us of GPU time per event)
      TK_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      ev.push_back(e);
    }
    return ev[used++];
  }
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

struct StepMarks {
  std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> marks;
};

void hooi_iterate(Ctx* c, int iters, double* fits) {
  const int N = c->N;
  c->timings.clear();
  EventPool pool;
  StepMarks sm;
  auto mark = [&](const std::string& name, hipEvent_t a) {
    hipEvent_t b = pool.next();
    TK_HIP(hipEventRecord(b, c->stream));
    sm.marks.push_back({name, {a, b}});
    return b;
  };
  // the SVD step's route per mode: the Gram formed, or matrix-free on Y
  auto matfree = [&](int n) {
    const int64_t kh = c->plan[n].khat;
    if (kh < 192 || c->K[n] > 31) return false;
    if (c->opt.eig_method == TK_EIG_MATFREE) return true;
    if (c->opt.eig_method == TK_EIG_GRAM) return false;
    return kh >= TK_MATFREE_MIN_KHAT;
  };
  int64_t maxY = 0, maxKh = 0, maxKhG = 0;
  for (int n = 0; n < N; ++n) {
    maxY = std::max(maxY, c->plan[n].L_nz * c->plan[n].khat);
    maxKh = std::max(maxKh, c->plan[n].khat);
    if (!matfree(n)) maxKhG = std::max(maxKhG, c->plan[n].khat);
  }
  ensure(c, c->Y, sizeof(float) * (size_t)std::max<int64_t>(maxY, 1));
  ensure(c, c->gram64, sizeof(double) * (size_t)std::max<int64_t>(maxKhG * maxKhG, 1));
  if (maxKhG < maxKh) ensure(c, c->diag64, sizeof(double) * (size_t)maxKh);
  ensure(c, c->eig_val, sizeof(double) * 64 + sizeof(double) * (size_t)maxKh * 64);
  ensure(c, c->flag, sizeof(int) * FLAG_INTS);
  int64_t core_n = 1;
  for (int j = 0; j < N; ++j) core_n *= c->K[j];
  ensure(c, c->core64, sizeof(double) * (size_t)core_n + 2 * sizeof(double));
  // Jacobi sweep: TTM reads the invocation's input factors (FP32 copies kept aside)
  std::vector<Buf> F32_in(c->opt.sweep == TK_SWEEP_JACOBI ? N : 0);
  for (int it = 0; it < iters; ++it) {
    if (c->opt.sweep == TK_SWEEP_JACOBI) {
      for (int n = 0; n < N; ++n) {
        F32_in[n].alloc(c, c->F32[n].bytes());
        d2d(c, F32_in[n].as<char>(), c->F32[n].as<char>(), c->F32[n].bytes());
      }
    }
    float* Y = c->Y.as<float>();
    // precision form: BF16 Kronecker tiles and Gram operands, except in the refining last invocation
    const bool low = c->opt.prec == TK_BF16 && !(c->opt.refine && it == iters - 1);
    // Gauss-Seidel sweeps check for a failed (rank-deficient) factor once, at
    // the end of the invocation, instead of stopping the stream after every
    // mode; a failure skips the later modes' factor writes and those modes are
    // run again below, after the failed factor is completed.  Once a factor
    // of this tensor has needed completion, later invocations check after
    // every mode instead (one host wait per mode, no reruns).
    const bool defer = c->opt.sweep == TK_SWEEP_GAUSS_SEIDEL && !c->completed_once;
    if (defer) TK_HIP(hipMemsetAsync(c->flag.as<int>() + 1, 0, sizeof(int), c->stream));
    auto run_mode = [&](int n, bool deferred) {
      ModePlan& pl = c->plan[n];
      const int khat = (int)pl.khat;
      const int K = c->K[n];
      TK_REQUIRE(K <= 32, TK_ERR_UNSUPPORTED, "HOOI supports ranks up to 32");
      hipEvent_t t0 = pool.next();
      TK_HIP(hipEventRecord(t0, c->stream));
      hipEvent_t k0 = pool.next(), k1 = pool.next();
      c->ev_ttm[0] = k0;
      c->ev_ttm[1] = k1;
      sm.marks.push_back({"ttm_kernel[" + std::to_string(n) + "]", {k0, k1}});
      // the precision form's invocations (all but a refining last one) form
      // the Kronecker tiles in BF16 on the matrix cores
      if (c->opt.sweep == TK_SWEEP_JACOBI) {
        // swap in the input copies for the other modes
        for (int j = 0; j < N; ++j)
          if (j != n) std::swap(c->F32[j], F32_in[j]);
        ttm_chain(c, n, Y, low);
        for (int j = 0; j < N; ++j)
          if (j != n) std::swap(c->F32[j], F32_in[j]);
      } else {
        ttm_chain(c, n, Y, low);
      }
      c->ev_ttm[0] = c->ev_ttm[1] = nullptr;
      if (c->m == 0) {  // no launch: give the bracket a zero-length interval
        TK_HIP(hipEventRecord(k0, c->stream));
        TK_HIP(hipEventRecord(k1, c->stream));
      }
      hipEvent_t t1 = mark("ttm[" + std::to_string(n) + "]", t0);
      double* lam_k = c->eig_val.as<double>();
      double* VK = lam_k + 64;
      if (matfree(n)) {
        // block Krylov on Y (the diagonal of Y^T Y, for the rank floor, on the way)
        hipEvent_t t2 = mark("gram", t1);
        eig_topk_matfree(c, Y, pl.L_nz, khat, K, lam_k, VK, n, c->diag64.as<double>());
        hipEvent_t t3 = mark("eig", t2);
        form_factor(c, n, Y, pl.L_nz, khat, c->diag64.as<double>(), 1, lam_k, VK, c->flag.as<int>(), deferred);
        mark("factor", t3);
      } else {
        gram(c, Y, pl.L_nz, khat, c->gram64.as<double>(), low);
        hipEvent_t t2 = mark("gram", t1);
        eig_topk(c, c->gram64.as<double>(), khat, K, lam_k, VK, n);
        hipEvent_t t3 = mark("eig", t2);
        form_factor(c, n, Y, pl.L_nz, khat, c->gram64.as<double>(), (int64_t)khat + 1, lam_k, VK, c->flag.as<int>(),
                    deferred);
        mark("factor", t3);
      }
    };
    for (int n = 0; n < N; ++n) run_mode(n, defer);
    if (defer) {
      int failed = 0;
      d2h(c, &failed, c->flag.as<int>() + 1, 1);
      c->sync();
      if (failed > 0) {
        const int n0 = failed - 1;
        if (!c->opt.complete_rank_deficient) fail(TK_ERR_NUMERIC, "rank-deficient penultimate matrix");
        int bits = 0;
        d2h(c, &bits, c->flag.as<int>() + FLAG_BITS + n0, 1);
        c->sync();
        complete_factor(c, n0, bits == 2 ? computed_columns(c, c->flag.as<int>(), n0) : -1);
        TK_HIP(hipMemsetAsync(c->flag.as<int>() + 1, 0, sizeof(int), c->stream));
        // the skipped modes' factor copies were not cleared on the device (the
        // clear was conditional on no earlier failure) although their host-side
        // flags say so: mark them again so the rerun zeroes rows of empty slices
        for (int n = n0 + 1; n < N; ++n) c->fac_dirty[n] = true;
        for (int n = n0 + 1; n < N; ++n) run_mode(n, false);
      }
    }
    // core and fit from the last mode (valid for Gauss-Seidel: Y_(N) used the final factors)
    hipEvent_t t4 = pool.next();
    TK_HIP(hipEventRecord(t4, c->stream));
    if (c->opt.sweep == TK_SWEEP_JACOBI) ttm_chain(c, N - 1, Y, low);
    double* core = c->core64.as<double>();
    core_from_last(c, Y, core, core + core_n);
    mark("core", t4);
    double out2[2] = {0, 0};
    d2h(c, out2, core + core_n, 2);
    c->sync();
    if (fits) fits[it] = out2[1];
  }
  c->ev_ttm[0] = c->ev_ttm[1] = nullptr;
  c->sync();
  for (auto& m : sm.marks) {
    float ms = 0;
    TK_HIP(hipEventElapsedTime(&ms, m.second.first, m.second.second));
    c->timings.add(m.first, ms);
  }
}

}  // namespace tk

using namespace tk;

struct tk_ctx : public Ctx {};

static thread_local std::string g_err;

template <class F>
static tk_status guard(tk_ctx* c, F&& f) {
  try {
    f();
    if (c) c->last_error.clear();
    return TK_OK;
  } catch (const Error& e) {
    if (c) c->last_error = e.msg;
    g_err = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    return TK_ERR_OOM;
  } catch (...) {
    if (c) c->last_error = "unexpected exception";
    return TK_ERR_DEVICE;
  }
}

extern "C" {

const char* tk_status_string(tk_status s) {
  switch (s) {
    case TK_OK: return "ok";
    case TK_ERR_INVALID_ARG: return "invalid argument";
    case TK_ERR_STATE: return "call out of order";
    case TK_ERR_OOM: return "out of memory";
    case TK_ERR_DEVICE: return "device error";
    case TK_ERR_NUMERIC: return "numerical failure";
    case TK_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

tk_status tk_default_options(tk_options* o) {
  if (!o) return TK_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->prec = TK_FP32;
  o->sweep = TK_SWEEP_GAUSS_SEIDEL;
  o->wg_nnz_target = 0;
  o->lds_rows_cap = 0;
  o->refine = 1;
  o->mem_limit_bytes = 0;
  o->complete_rank_deficient = 1;
  o->keep_elem_order = 1;
  o->eig_tol = 0.0;
  o->partition = TK_PART_LITE;
  o->ttm_kernel = TK_TTM_AUTO;
  o->eig_method = TK_EIG_AUTO;
  return TK_OK;
}

tk_status tk_create(int device, void* hip_stream, const tk_allocator* allocator, tk_ctx** out) {
  if (!out) return TK_ERR_INVALID_ARG;
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) {
    g_err = "tk_create: the allocator needs both alloc and free";
    return TK_ERR_INVALID_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    g_err = "no HIP device";
    return TK_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return TK_ERR_INVALID_ARG;
  tk_ctx* c = new (std::nothrow) tk_ctx();
  if (!c) return TK_ERR_OOM;
  tk_status s = guard(c, [&] {
    TK_HIP(hipSetDevice(device));
    c->device = device;
    if (allocator) c->allocator = *allocator;
    noalloc_scratch_init(device);
    c->stream = (hipStream_t)hip_stream;
    tk_default_options(&c->opt);
    int v = 0;
    TK_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
    c->cu_count = v;
    TK_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    c->lds_per_block = (size_t)v;
  });
  if (s != TK_OK) {
    delete c;
    return s;
  }
  *out = c;
  return TK_OK;
}

void tk_destroy(tk_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* tk_last_error(const tk_ctx* c) { return c ? c->last_error.c_str() : g_err.c_str(); }

tk_status tk_set_options(tk_ctx* c, const tk_options* o) {
  if (!c || !o) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(o->prec == TK_FP32 || o->prec == TK_BF16, TK_ERR_INVALID_ARG, "prec");
    TK_REQUIRE(o->sweep == TK_SWEEP_GAUSS_SEIDEL || o->sweep == TK_SWEEP_JACOBI, TK_ERR_INVALID_ARG, "sweep");
    TK_REQUIRE(o->wg_nnz_target >= 0 && o->mem_limit_bytes >= 0, TK_ERR_INVALID_ARG, "negative size");
    TK_REQUIRE(o->eig_tol >= 0.0, TK_ERR_INVALID_ARG, "negative eig_tol");
    TK_REQUIRE(o->partition == TK_PART_LITE || o->partition == TK_PART_COARSE, TK_ERR_INVALID_ARG, "partition");
    TK_REQUIRE(o->ttm_kernel >= TK_TTM_AUTO && o->ttm_kernel <= TK_TTM_FIBER, TK_ERR_INVALID_ARG, "ttm_kernel");
    TK_REQUIRE(o->eig_method >= TK_EIG_AUTO && o->eig_method <= TK_EIG_MATFREE, TK_ERR_INVALID_ARG, "eig_method");
    c->opt = *o;
  });
}

tk_status tk_set_stream(tk_ctx* c, void* s) {
  if (!c) return TK_ERR_INVALID_ARG;
  c->stream = (hipStream_t)s;
  return TK_OK;
}

static void drop_tensor(Ctx* c) {
  c->have_tensor = false;
  c->have_ranks = false;
  for (int j = 0; j < 8; ++j) {
    c->plan[j] = ModePlan();
    c->F64[j].release();
    c->F32[j].release();
    c->eig_warm[j].release();
    c->eig_warm_k[j] = 0;
  }
  for (int j = 0; j < 8; ++j) {
    c->idx_c[j].release();
    c->slice_order[j].release();
  }
  c->val_c.release();
  c->m = 0;
  c->completed_once = false;
}

tk_status tk_load_coo_begin(tk_ctx* c, int N, const int64_t* dims, int64_t nnz, unsigned flags) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(N >= 2 && N <= 8, TK_ERR_INVALID_ARG, "N must be in [2, 8]");
    TK_REQUIRE(dims != nullptr, TK_ERR_INVALID_ARG, "dims is NULL");
    for (int j = 0; j < N; ++j)
      TK_REQUIRE(dims[j] >= 1 && dims[j] <= 2147483647LL, TK_ERR_INVALID_ARG, "dims out of range");
    TK_REQUIRE(nnz >= 0 && nnz <= (1LL << 40), TK_ERR_INVALID_ARG, "nnz must be in [0, 2^40]");
    TK_REQUIRE((flags & ~TK_ASSUME_UNIQUE) == 0, TK_ERR_INVALID_ARG, "unknown flags");
    TK_HIP(hipSetDevice(c->device));
    // drop the previous tensor and plan (and any load in progress)
    c->load = LoadState();
    drop_tensor(c);
    try {
      load_begin(c, N, dims, nnz, flags);
    } catch (...) {
      c->load = LoadState();
      throw;
    }
  });
}

tk_status tk_load_coo_append(tk_ctx* c, int64_t count, const int32_t* const* idx, const float* vals, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->load.active, TK_ERR_STATE, "tk_load_coo_begin first");
    TK_REQUIRE(mem == TK_MEM_HOST || mem == TK_MEM_DEVICE, TK_ERR_INVALID_ARG, "mem");
    TK_REQUIRE(count >= 0 && count <= c->load.nnz - c->load.filled, TK_ERR_INVALID_ARG,
               "append beyond the announced element count");
    if (count == 0) return;
    TK_REQUIRE(idx != nullptr && vals != nullptr, TK_ERR_INVALID_ARG, "idx or vals is NULL");
    for (int j = 0; j < c->load.N; ++j) TK_REQUIRE(idx[j] != nullptr, TK_ERR_INVALID_ARG, "idx[n] is NULL");
    TK_HIP(hipSetDevice(c->device));
    load_append(c, count, idx, vals, mem);
  });
}

tk_status tk_load_coo_end(tk_ctx* c) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->load.active, TK_ERR_STATE, "tk_load_coo_begin first");
    TK_HIP(hipSetDevice(c->device));
    try {
      load_end(c);
    } catch (...) {
      c->load = LoadState();   // nothing is kept
      drop_tensor(c);
      throw;
    }
  });
}

tk_status tk_load_coo(tk_ctx* c, int N, const int64_t* dims, int64_t nnz, const int32_t* const* idx,
                      const float* vals, tk_mem mem, unsigned flags) {
  if (!c) return TK_ERR_INVALID_ARG;
  tk_status s = tk_load_coo_begin(c, N, dims, nnz, flags);
  if (s != TK_OK) return s;
  s = tk_load_coo_append(c, nnz, idx, vals, mem);
  if (s != TK_OK) {
    c->load = LoadState();
    return s;
  }
  return tk_load_coo_end(c);
}

tk_status tk_get_tensor_info(const tk_ctx* c, int64_t* nnz_c, double* norm_sq) {
  if (!c) return TK_ERR_INVALID_ARG;
  if (!c->have_tensor) return TK_ERR_STATE;
  if (nnz_c) *nnz_c = c->m;
  if (norm_sq) *norm_sq = c->norm_sq;
  return TK_OK;
}

tk_status tk_get_coo(tk_ctx* c, int32_t* const* idx, float* vals, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_tensor, TK_ERR_STATE, "no tensor loaded");
    for (int j = 0; j < c->N; ++j)
      if (idx && idx[j]) copy_out(c, idx[j], c->idx_c[j].as<int32_t>(), (size_t)c->m, mem);
    if (vals) copy_out(c, vals, c->val_c.as<float>(), (size_t)c->m, mem);
    c->sync();
  });
}

// F (L x K, row-major) = the first K columns of the identity: the factors'
// placeholder until the caller sets them.
__global__ void k_leading_identity(double* __restrict__ F, int64_t L, int K) {
  const int64_t total = L * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    F[i] = (i / K == i % K) ? 1.0 : 0.0;
}

tk_status tk_set_ranks(tk_ctx* c, const int32_t* K) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_tensor, TK_ERR_STATE, "load a tensor first");
    TK_REQUIRE(K != nullptr, TK_ERR_INVALID_ARG, "K is NULL");
    const int N = c->N;
    for (int j = 0; j < N; ++j) {
      TK_REQUIRE(K[j] >= 1 && (int64_t)K[j] <= c->dims[j], TK_ERR_INVALID_ARG, "K[n] must be in [1, dims[n]]");
      TK_REQUIRE(K[j] <= 64, TK_ERR_UNSUPPORTED, "ranks above 64");
    }
    TK_HIP(hipSetDevice(c->device));
    c->have_ranks = false;
    for (int j = 0; j < N; ++j) c->K[j] = K[j];
    // memory plan check before allocating (mem_limit_bytes)
    if (c->opt.mem_limit_bytes > 0) {
      int64_t need = 0;
      for (int n = 0; n < N; ++n) need += c->m * (4 * (int64_t)N + (c->opt.keep_elem_order ? 4 : 0));
      need += c->m * 24;  // sort buffers during construction
      for (int n = 0; n < N; ++n) need += c->dims[n] * (int64_t)K[n] * (8 + 4) + c->dims[n] * 32;
      TK_REQUIRE(c->bytes_in_use + need <= c->opt.mem_limit_bytes, TK_ERR_OOM,
                 "the plan needs about " + std::to_string(need) + " bytes, above mem_limit_bytes");
    }
    const bool coarse = c->opt.partition == TK_PART_COARSE;
    if (coarse)
      for (int n = 0; n < N; ++n)
        TK_REQUIRE(c->slice_order[n].bytes() == sizeof(int32_t) * (size_t)c->dims[n], TK_ERR_STATE,
                   "the CoarseG partition needs tk_set_slice_order for every mode");
    {
      SortScratch ss;
      for (int n = 0; n < N; ++n) {
        const int tw = ttm_tile_width(N, K, n);
        build_plan(c, c->plan[n], N, n, c->dims, c->m, c->idx_c, c->val_c.as<float>(), khat_of(c, n), tw,
                   ttm_default_bin_nnz(N, K, n, c->opt.ttm_kernel), c->opt.keep_elem_order != 0, ss, n == N - 1,
                   coarse ? c->slice_order[n].as<int32_t>() : nullptr);
      }
    }
    for (int n = 0; n < N; ++n) relabel_layout(c, c->plan[n], N, n, c->plan, c->m);
    for (int n = 0; n < N; ++n) {
      c->kp32[n] = K[n] <= 16 ? 16 : (K[n] + 3) & ~3;  // 64-byte rows: one 16-lane MFMA operand load
      c->F64[n].alloc(c, sizeof(double) * (size_t)c->dims[n] * K[n]);
      c->F32[n].alloc(c, sizeof(float) * (size_t)c->dims[n] * c->kp32[n]);
      const int64_t LK = c->dims[n] * K[n];
      hipLaunchKernelGGL(k_leading_identity, dim3(grid_for(LK, 256)), dim3(256), 0, c->stream,
                         c->F64[n].as<double>(), c->dims[n], K[n]);
      TK_CHECK_LAUNCH();
      refresh_factor_copies(c, n);
      c->fac_dirty[n] = true;
      c->eig_warm_k[n] = 0;
      c->sync();
    }
    c->have_ranks = true;
  });
}

__global__ void k_count_ids(const int32_t* __restrict__ p, int64_t L, int32_t* __restrict__ seen,
                            int32_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = p[i];
    if (v < 0 || (int64_t)v >= L) {
      atomicOr(flag, 1);
    } else if (atomicAdd(seen + v, 1) != 0) {
      atomicOr(flag, 1);
    }
  }
}

tk_status tk_set_slice_order(tk_ctx* c, int n, const int32_t* perm, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_tensor, TK_ERR_STATE, "load a tensor first");
    TK_REQUIRE(n >= 0 && n < c->N && perm, TK_ERR_INVALID_ARG, "mode out of range or perm is NULL");
    TK_REQUIRE(mem == TK_MEM_HOST || mem == TK_MEM_DEVICE, TK_ERR_INVALID_ARG, "mem");
    TK_HIP(hipSetDevice(c->device));
    const int64_t L = c->dims[n];
    Buf p(c, sizeof(int32_t) * (size_t)L), seen(c, sizeof(int32_t) * (size_t)(L + 1));
    copy_in(c, p.as<int32_t>(), perm, (size_t)L, mem);
    TK_HIP(hipMemsetAsync(seen.get(), 0, sizeof(int32_t) * (size_t)(L + 1), c->stream));
    hipLaunchKernelGGL(k_count_ids, dim3(grid_for(L, 256, 4096)), dim3(256), 0, c->stream, p.as<int32_t>(), L,
                       seen.as<int32_t>(), seen.as<int32_t>() + L);
    TK_CHECK_LAUNCH();
    int32_t bad = 0;
    d2h(c, &bad, seen.as<int32_t>() + L, 1);
    c->sync();
    TK_REQUIRE(bad == 0, TK_ERR_INVALID_ARG, "tk_set_slice_order: not a permutation of [0, L_n)");
    c->slice_order[n] = std::move(p);
  });
}

tk_status tk_get_partition_stats(tk_ctx* c, int n, tk_part_stats* out) {
  if (!c || !out) return TK_ERR_INVALID_ARG;
  if (!c->have_ranks) return TK_ERR_STATE;
  if (n < 0 || n >= c->N) return TK_ERR_INVALID_ARG;
  const ModePlan& p = c->plan[n];
  out->P = p.P;
  out->limit = p.limit;
  out->m = c->m;
  out->L_nonempty = p.L_nz;
  out->n_stage1 = p.n_stage1;
  out->E_max = p.E_max;
  out->R_sum = p.S;
  out->R_max = p.R_max;
  out->n_bad = p.n_bad;
  return TK_OK;
}

tk_status tk_get_partition(tk_ctx* c, int n, int64_t* bin_ptr, int64_t* elem_order, int32_t* seg_bin,
                           int32_t* seg_slice, int64_t* seg_begin, uint8_t* seg_bad, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(n >= 0 && n < c->N, TK_ERR_INVALID_ARG, "mode out of range");
    export_partition(c, c->plan[n], c->m, bin_ptr, elem_order, seg_bin, seg_slice, seg_begin, seg_bad, mem);
  });
}

tk_status tk_set_factor(tk_ctx* c, int n, const double* F, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(n >= 0 && n < c->N && F, TK_ERR_INVALID_ARG, "mode out of range or F is NULL");
    copy_in(c, c->F64[n].as<double>(), F, (size_t)c->dims[n] * c->K[n], mem);
    refresh_factor_copies(c, n);
    c->fac_dirty[n] = true;
    c->sync();
  });
}

tk_status tk_get_factor(tk_ctx* c, int n, double* F, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(n >= 0 && n < c->N && F, TK_ERR_INVALID_ARG, "mode out of range or F is NULL");
    copy_out(c, F, c->F64[n].as<double>(), (size_t)c->dims[n] * c->K[n], mem);
    c->sync();
  });
}

tk_status tk_ttm_shape(tk_ctx* c, int n, int64_t* R_n, int64_t* Khat_n) {
  if (!c) return TK_ERR_INVALID_ARG;
  if (!c->have_ranks) return TK_ERR_STATE;
  if (n < 0 || n >= c->N) return TK_ERR_INVALID_ARG;
  if (R_n) *R_n = c->plan[n].L_nz;
  if (Khat_n) *Khat_n = c->plan[n].khat;
  return TK_OK;
}

tk_status tk_ttm_chain(tk_ctx* c, int n, float* Y, int32_t* row_slice, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(n >= 0 && n < c->N, TK_ERR_INVALID_ARG, "mode out of range");
    const ModePlan& pl = c->plan[n];
    const size_t ny = (size_t)pl.L_nz * (size_t)pl.khat;
    if (Y) {
      // the kernels store rows 16 bytes at a time: a device Y that is not
      // 16-byte aligned is filled through the library's buffer
      if (mem == TK_MEM_DEVICE && (reinterpret_cast<uintptr_t>(Y) & 15) == 0) {
        ttm_chain(c, n, Y, c->opt.prec == TK_BF16);
      } else {
        ensure(c, c->Y, sizeof(float) * std::max<size_t>(ny, 1));
        ttm_chain(c, n, c->Y.as<float>(), c->opt.prec == TK_BF16);
        copy_out(c, Y, c->Y.as<float>(), ny, mem);
        if (mem == TK_MEM_HOST) c->sync();
      }
    }
    if (row_slice) {
      copy_out(c, row_slice, pl.row_slice.as<int32_t>(), (size_t)pl.L_nz, mem);
      if (mem == TK_MEM_HOST) c->sync();
    }
  });
}

static bool is_device_ptr(const void* p, int device) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice && at.device == device;
}

tk_status tk_ttm_chain_noalloc(tk_ctx* c, int n, float* Y, int32_t* row_slice) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(n >= 0 && n < c->N, TK_ERR_INVALID_ARG, "mode out of range");
    const ModePlan& pl = c->plan[n];
    if (pl.L_nz > 0) {
      TK_REQUIRE(Y && is_device_ptr(Y, c->device), TK_ERR_INVALID_ARG, "Y must be device memory of the context's GPU");
      TK_REQUIRE((reinterpret_cast<uintptr_t>(Y) & 15) == 0, TK_ERR_INVALID_ARG,
                 "Y must be 16-byte aligned (rows are stored 16 bytes at a time)");
      TK_REQUIRE(!row_slice || is_device_ptr(row_slice, c->device), TK_ERR_INVALID_ARG,
                 "row_slice must be device memory of the context's GPU");
    }
    TK_HIP(hipSetDevice(c->device));
    ttm_chain_noalloc(c, n, Y);
    if (row_slice && pl.L_nz > 0) copy_out(c, row_slice, pl.row_slice.as<int32_t>(), (size_t)pl.L_nz, TK_MEM_DEVICE);
  });
}

tk_status tk_hooi_iterate(tk_ctx* c, int iters, double* fits) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(iters >= 0, TK_ERR_INVALID_ARG, "iters < 0");
    TK_HIP(hipSetDevice(c->device));
    hooi_iterate(c, iters, fits);
  });
}

tk_status tk_init_hosvd(tk_ctx* c, const double* const* sketch, tk_mem mem, double* fit) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    TK_REQUIRE(sketch != nullptr, TK_ERR_INVALID_ARG, "sketch is NULL");
    for (int j = 0; j < c->N; ++j) TK_REQUIRE(sketch[j] != nullptr, TK_ERR_INVALID_ARG, "a sketch matrix is NULL");
    TK_HIP(hipSetDevice(c->device));
    // the sketches go where the factors are read from: the TTM-chain then
    // forms T_(n) times their Kronecker product
    for (int j = 0; j < c->N; ++j) {
      copy_in(c, c->F64[j].as<double>(), sketch[j], (size_t)c->dims[j] * c->K[j], mem);
      refresh_factor_copies(c, j);
      c->fac_dirty[j] = true;
    }
    struct Restore {
      Ctx* c;
      tk_options o;
      ~Restore() { c->opt = o; }
    } restore{c, c->opt};
    c->opt.sweep = TK_SWEEP_JACOBI;
    c->opt.prec = TK_FP32;
    double f = 0.0;
    hooi_iterate(c, 1, &f);
    if (fit) *fit = f;
  });
}

tk_status tk_core(tk_ctx* c, double* core, double* fit, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_ranks, TK_ERR_STATE, "set ranks first");
    const int N = c->N;
    int64_t core_n = 1;
    for (int j = 0; j < N; ++j) core_n *= c->K[j];
    int64_t ny = c->plan[N - 1].L_nz * c->plan[N - 1].khat;
    ensure(c, c->Y, sizeof(float) * (size_t)std::max<int64_t>(ny, 1));
    ensure(c, c->core64, sizeof(double) * (size_t)core_n + 2 * sizeof(double));
    ttm_chain(c, N - 1, c->Y.as<float>(), false);
    double* d = c->core64.as<double>();
    core_from_last(c, c->Y.as<float>(), d, d + core_n);
    if (core) copy_out(c, core, d, (size_t)core_n, mem);
    double out2[2];
    d2h(c, out2, d + core_n, 2);
    c->sync();
    if (fit) *fit = out2[1];
  });
}

tk_status tk_get_timings(tk_ctx* c, double* ms, const char** names, int* count) {
  if (!c || !count) return TK_ERR_INVALID_ARG;
  int n = (int)c->timings.names.size();
  int cap = *count;
  int w = std::min(n, cap);
  for (int i = 0; i < w; ++i) {
    if (ms) ms[i] = c->timings.ms[i];
    if (names) names[i] = c->timings.names[i].c_str();
  }
  *count = w;
  return TK_OK;
}

tk_status tk_get_counters(tk_ctx* c, int64_t* values, const char** names, int* count) {
  if (!c || !count) return TK_ERR_INVALID_ARG;
  static const char* const kNames[] = {"eig_krylov_solves", "eig_krylov_cycles", "eig_dense_fallbacks",
                                       "rank_completions"};
  const int64_t v[] = {c->counters.eig_krylov_solves, c->counters.eig_krylov_cycles,
                       c->counters.eig_dense_fallbacks, c->counters.rank_completions};
  const int w = std::min(*count, 4);
  for (int i = 0; i < w; ++i) {
    if (values) values[i] = v[i];
    if (names) names[i] = kNames[i];
  }
  *count = w;
  return TK_OK;
}

tk_status tk_load_obs(tk_ctx* c, int N, const int64_t* dims, const int32_t* ranks, int64_t n_obs,
                      const int32_t* const* idx, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(N >= 2 && N <= 8 && dims && ranks, TK_ERR_INVALID_ARG, "N, dims or ranks");
    TK_REQUIRE(n_obs >= 0 && n_obs < (1LL << 31), TK_ERR_INVALID_ARG, "n_obs out of range");
    for (int j = 0; j < N; ++j) {
      TK_REQUIRE(dims[j] >= 1 && dims[j] <= 2147483647LL, TK_ERR_INVALID_ARG, "dims out of range");
      TK_REQUIRE(ranks[j] >= 1 && ranks[j] <= 64, TK_ERR_INVALID_ARG, "ranks out of range");
    }
    if (n_obs > 0) {
      TK_REQUIRE(idx != nullptr, TK_ERR_INVALID_ARG, "idx is NULL");
      for (int j = 0; j < N; ++j) TK_REQUIRE(idx[j] != nullptr, TK_ERR_INVALID_ARG, "idx[n] is NULL");
    }
    TK_HIP(hipSetDevice(c->device));
    load_obs(c, N, dims, ranks, n_obs, idx, mem);
  });
}

tk_status tk_tucker_eval(tk_ctx* c, const float* core, const float* const* F, float* model, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_obs, TK_ERR_STATE, "load observations first");
    TK_REQUIRE(core && F && model, TK_ERR_INVALID_ARG, "NULL argument");
    for (int j = 0; j < c->obs.N; ++j) TK_REQUIRE(F[j], TK_ERR_INVALID_ARG, "F[n] is NULL");
    obs_eval(c, core, F, model, mem);
  });
}

tk_status tk_tucker_adjoint(tk_ctx* c, const float* g, const float* core, const float* const* F, float* dcore,
                            float* const* dF, tk_mem mem) {
  if (!c) return TK_ERR_INVALID_ARG;
  return guard(c, [&] {
    TK_REQUIRE(c->have_obs, TK_ERR_STATE, "load observations first");
    TK_REQUIRE(g && core && F && dcore && dF, TK_ERR_INVALID_ARG, "NULL argument");
    for (int j = 0; j < c->obs.N; ++j) TK_REQUIRE(F[j] && dF[j], TK_ERR_INVALID_ARG, "F[n] or dF[n] is NULL");
    obs_adjoint(c, g, core, F, dcore, dF, mem);
  });
}

}  // extern "C"
