/*
 * tucker_hip.h -- C ABI of a one-GPU (MI355X, gfx950) library for the hot path
 * of sparse Tucker decomposition by HOOI, following Chakaravarthy et al., "On
 * Optimizing Distributed Tucker Decomposition for Sparse Tensors" (arXiv
 * 1804.09494).
 *
 * What it computes (paper references are to sections, equations and figures):
 *   - the sparse tensor T is a list of elements, each a coordinate vector and a
 *     value (Section 3);
 *   - for each mode n, the penultimate matrix Y_(n) = (T x_{j!=n} F_j^T)_(n)
 *     through the Kronecker reformulation (eq. 1, Appendix A): every element
 *     adds val * (Kronecker product of its factor rows, first remaining mode
 *     fastest) into row l_n of Y_(n);
 *   - the leading K_n left singular vectors of Y_(n) as the new factor
 *     (Section 2.2, HOOI figure), here through the Gram matrix Y^T Y, an FP64
 *     eigensolve (Householder tridiagonalisation, bisection, inverse
 *     iteration), U = Y V S^-1 and FP64 CholeskyQR2;
 *   - the core G = T x_1 F_1^T ... x_N F_N^T once after the invocations
 *     (Section 2.2);
 *   - the elements of each mode are split over GPU workgroups ("bins") by the
 *     Lite scheme (Section 6, Lite figure, Theorem 6.1), which bounds the
 *     elements (limit = ceil(m/P)) and distinct slices (ceil(L/P) + 2) of every
 *     bin so that each bin reduces its rows of Y_(n) in LDS.
 *
 * Conventions
 *   - Every call returns tk_status (TK_OK = 0); nothing throws, exits or aborts.
 *     After a failure, tk_last_error(ctx) holds a message.
 *   - Coordinates are 0-based int32 (the paper's are 1-based).
 *   - "mem" arguments say whether a pointer is host memory (TK_MEM_HOST) or
 *     device memory of the context's GPU (TK_MEM_DEVICE).
 *   - Ownership: inputs are copied before the call returns; outputs are written
 *     into caller-owned buffers; the context owns all of its device memory and
 *     frees it in tk_destroy.
 *   - Streams: all device work is ordered on the stream given to tk_create
 *     (NULL = the null stream).  Calls that return host values synchronise
 *     that stream.  A context is not thread-safe; distinct contexts are
 *     independent.
 *   - Canonical element order: lexicographic on (l_1, ..., l_N), l_1 most
 *     significant.
 *   - Unfolding / Kronecker column order: the first remaining mode varies
 *     fastest (Section 2.1, Appendix A).  The core is stored first index
 *     fastest.
 */
#ifndef TUCKER_HIP_H
#define TUCKER_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tk_ctx tk_ctx;

typedef enum {
  TK_OK = 0,
  TK_ERR_INVALID_ARG = 1,  /* bad pointer, size, coordinate, rank or non-finite value */
  TK_ERR_STATE = 2,        /* call out of order (e.g. iterate before tk_set_ranks) */
  TK_ERR_OOM = 3,          /* device allocation failed or the plan exceeds mem_limit_bytes */
  TK_ERR_DEVICE = 4,       /* a HIP runtime call failed */
  TK_ERR_NUMERIC = 5,      /* rank-deficient Y_(n) with completion disabled */
  TK_ERR_UNSUPPORTED = 6   /* a size outside what this build handles (e.g. ranks above 64) */
} tk_status;

typedef enum { TK_MEM_HOST = 0, TK_MEM_DEVICE = 1 } tk_mem;
typedef enum { TK_FP32 = 0, TK_BF16 = 1 } tk_prec;
typedef enum { TK_SWEEP_GAUSS_SEIDEL = 0, TK_SWEEP_JACOBI = 1 } tk_sweep;
/* How each mode's elements are split over the workgroups ("bins"). */
typedef enum {
  TK_PART_LITE = 0,    /* Lite (Section 6): the default */
  TK_PART_COARSE = 1   /* CoarseG (Section 5, coarse grained schemes): the mode's slices in a caller-given
                          random order (tk_set_slice_order), cut into contiguous blocks of whole slices, the
                          block of slice t holding the slices whose element prefix starts in
                          [p m / P, (p+1) m / P); an ablation baseline */
} tk_partition;
/* Which TTM-chain kernel runs. */
typedef enum {
  TK_TTM_AUTO = 0,     /* matrix-core kernels where they apply, else the vector-ALU one */
  TK_TTM_VECTOR = 1,   /* the vector-ALU kernel for every shape (and whatever the bin sizes) */
  TK_TTM_ATOMIC = 2,   /* no partition: the merged element list in canonical order, each wave's
                          running row sums added to Y with FP32 atomics when the mode-n index changes
                          (not deterministic); an ablation baseline */
  TK_TTM_FIBER = 3     /* fiber-factored (three or four modes, other ranks <= 16; other shapes as AUTO):
                          the elements of a slice sharing all remaining coordinates but the last are
                          summed first, t = sum val F_c[l_c], then F_a (x) F_b (x) t is added once per
                          fiber (eq. 1 grouped by fibers); Lite bins of 512 elements by default */
} tk_ttm_kernel;
/* How the SVD step of HOOI reaches the eigenpairs of Y^T Y (Section 3, "SVD Component"). */
typedef enum {
  TK_EIG_AUTO = 0,     /* the Gram route below Khat = TK_MATFREE_MIN_KHAT, matrix-free from there (K <= 31) */
  TK_EIG_GRAM = 1,     /* form G = Y^T Y (Khat x Khat, matrix cores), then the dense solver (Khat up to
                          about 100) or block Krylov on G */
  TK_EIG_MATFREE = 2   /* block Krylov on Y itself, never squared: each block product is Y^T (Y X), two
                          passes over Y; Khat >= 192 and K <= 31 (smaller Khat takes the Gram route) */
} tk_eig_method;
#define TK_MATFREE_MIN_KHAT 8192

typedef struct {
  int32_t prec;                   /* tk_prec (default TK_FP32).  TK_BF16 (the precision form): the
                                     Kronecker tiles of the TTM-chain (three- and four-mode tensors with
                                     other ranks <= 16) and the Gram operands are rounded to BF16 on the
                                     matrix cores, FP32 accumulation, in tk_ttm_chain and in HOOI
                                     invocations (but a refining last one, see refine).  The eigensolve,
                                     CholeskyQR2, core and fit stay FP64 */
  int32_t sweep;                  /* tk_sweep (default Gauss-Seidel: mode n uses factors refined earlier in the invocation) */
  int64_t wg_nnz_target;          /* target elements per bin; 0 (default) = per kernel: 448 for the
                                     three-mode matrix-core TTM-chain, 1024 for the four-mode one and
                                     for the completion adjoint, 4096 otherwise */
  int32_t lds_rows_cap;           /* max slices per bin; 0 = from the LDS budget */
  int32_t refine;                 /* BF16 only: 1 = the last invocation runs in FP32 (default 1) */
  int64_t mem_limit_bytes;        /* 0 = no limit; plans above it fail with TK_ERR_OOM before allocating */
  int32_t complete_rank_deficient;/* 1 (default) = complete U with unit vectors; 0 = TK_ERR_NUMERIC */
  int32_t keep_elem_order;        /* 1 (default) = keep each mode's element order for tk_get_partition */
  double eig_tol;                 /* block-Krylov eigensolve (Khat >= 192): when its result is accepted.
                                     0 (default): once the relative residual ||A v - theta v|| / theta_1
                                     is at the rounding level of the FP32 data the operator is formed
                                     from (4 u, u = 2^-24); below it the dense solver on the same data
                                     would not fix the subspace any better.  > 0: only when the estimated
                                     subspace error sqrt(2) * residual * theta_1 / (theta_K - theta_{K+1})
                                     (sin-theta theorem) is at most eig_tol.  A rejected result reruns the
                                     mode's eigensolve with the dense solver (the matrix-free route first
                                     forms G and takes the Gram route) */
  int32_t partition;              /* tk_partition (default TK_PART_LITE); read by tk_set_ranks */
  int32_t ttm_kernel;             /* tk_ttm_kernel (default TK_TTM_AUTO) */
  int32_t eig_method;             /* tk_eig_method (default TK_EIG_AUTO) */
} tk_options;

/* Lite statistics of one mode (Section 4 metrics 1-3; Theorem 6.1). */
typedef struct {
  int64_t P;            /* number of bins */
  int64_t limit;        /* ceil(m / P) */
  int64_t m;            /* elements (after coalescing) */
  int64_t L_nonempty;   /* nonempty mode-n slices = rows of the compact Y_(n) */
  int64_t n_stage1;     /* slices placed whole by stage 1 (the paper's t-hat minus one) */
  int64_t E_max;        /* metric 1: max elements in a bin (<= limit) */
  int64_t R_sum;        /* metric 2: sum over bins of slices shared (= number of segments) */
  int64_t R_max;        /* metric 3: max slices in a bin (<= ceil(L_nonempty/P) + 2) */
  int64_t n_bad;        /* slices shared by more than one bin (<= P) */
} tk_part_stats;

/* Device-memory hooks: alloc returns `bytes` of device memory of the
 * context's GPU (NULL on failure, which the library reports as TK_ERR_OOM);
 * free returns such a block.  Both are called on the thread that calls the
 * library; blocks are in use on the context's stream until the call that
 * freed them returns. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, size_t bytes, void* user);
  void* user;
} tk_allocator;

/* ---- context ------------------------------------------------------------------------------- */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t or
 * NULL; `allocator` (copied; may be NULL = hipMalloc / hipFree) backs every
 * device allocation the context makes. */
tk_status tk_create(int device, void* hip_stream, const tk_allocator* allocator, tk_ctx** out);
void tk_destroy(tk_ctx* ctx);
const char* tk_status_string(tk_status s);
/* Message of the last failure on this context ("" if none).  Valid until the next call. */
const char* tk_last_error(const tk_ctx* ctx);
tk_status tk_default_options(tk_options* out);
tk_status tk_set_options(tk_ctx* ctx, const tk_options* opt);
/* Change the stream later calls are ordered on. */
tk_status tk_set_stream(tk_ctx* ctx, void* hip_stream);

/* ---- tensor (Section 3: the element list E) --------------------------------------------------- */

/* Flags of tk_load_coo / tk_load_coo_begin. */
#define TK_ASSUME_UNIQUE 1u   /* the caller guarantees distinct coordinates: the merge of repeated
                                 coordinates is skipped (any left are kept as separate elements) */

/* Load a sparse tensor in COO form.  N in [2, 8]; dims[n] in [1, 2^31 - 1];
 * nnz in [0, 2^40]; idx[n] points to nnz int32 coordinates of mode n (0-based,
 * < dims[n]); vals to nnz finite floats.  `mem` applies to idx[n] and vals
 * (the arrays of pointers themselves are host memory).
 * Repeated coordinates are merged by summing their values in FP64 (input
 * order), rounded once to FP32; the merged list is kept in canonical order.
 * ||T||^2 is accumulated in FP64.  Replaces any previous tensor and plan.
 * Device memory: about 16 + 4N bytes per element while the list is sorted
 * and merged, then (4N + 4) bytes per merged element.
 * Errors: TK_ERR_INVALID_ARG for a coordinate out of range or a NaN/Inf value
 * (checked on the device), nothing is kept; TK_ERR_OOM when the device memory
 * (or mem_limit_bytes) does not hold the list; TK_ERR_UNSUPPORTED for 2^32 or
 * more distinct coordinates. */
tk_status tk_load_coo(tk_ctx* ctx, int N, const int64_t* dims, int64_t nnz, const int32_t* const* idx,
                      const float* vals, tk_mem mem, unsigned flags);
/* The same load streamed in pieces, for lists the caller does not hold at
 * once: begin announces N, dims and the total nnz (same limits) and drops the
 * previous tensor; each append copies `count` more elements (host or device
 * memory, reusable when the call returns); end checks that nnz elements
 * arrived, then merges and sorts as tk_load_coo.  Errors of an append's
 * elements are reported by end. */
tk_status tk_load_coo_begin(tk_ctx* ctx, int N, const int64_t* dims, int64_t nnz, unsigned flags);
tk_status tk_load_coo_append(tk_ctx* ctx, int64_t count, const int32_t* const* idx, const float* vals, tk_mem mem);
tk_status tk_load_coo_end(tk_ctx* ctx);
/* m' (elements after merging) and ||T||^2 (FP64). */
tk_status tk_get_tensor_info(const tk_ctx* ctx, int64_t* nnz_coalesced, double* norm_sq);
/* Copy the merged element list out: idx[n] gets m' int32, vals m' floats. */
tk_status tk_get_coo(tk_ctx* ctx, int32_t* const* idx, float* vals, tk_mem mem);

/* ---- ranks and the Lite partition (Section 6) ------------------------------------------------- */

/* Set the Tucker ranks K[0..N-1] (1 <= K[n] <= dims[n]) and build, for every
 * mode, the Lite partition of the elements over bins and the mode-sorted copy
 * of the tensor the TTM-chain streams.  Factors are reset to the first K_n
 * columns of the identity; set them with tk_set_factor. */
tk_status tk_set_ranks(tk_ctx* ctx, const int32_t* K);
tk_status tk_get_partition_stats(tk_ctx* ctx, int n, tk_part_stats* out);
/* The random order of mode n's slice ids used by partition = TK_PART_COARSE:
 * perm holds L_n distinct ids in [0, L_n) (checked on the device; copied).
 * Needed for every mode before tk_set_ranks with that partition. */
tk_status tk_set_slice_order(tk_ctx* ctx, int n, const int32_t* perm, tk_mem mem);
/* Export mode n's partition (sizes from tk_get_partition_stats, S = R_sum):
 *   bin_ptr[P+1]   layout offset of each bin (int64)
 *   elem_order[m]  canonical element index at each layout position (int64; NULL to skip;
 *                  needs keep_elem_order)
 *   seg_bin[S]     bin of each segment (one slice piece), layout order
 *   seg_slice[S]   slice id (mode-n coordinate) of each segment
 *   seg_begin[S+1] layout offset of each segment, seg_begin[S] = m
 *   seg_bad[S]     1 when the segment's slice is shared by more than one bin
 * Any output may be NULL. */
tk_status tk_get_partition(tk_ctx* ctx, int n, int64_t* bin_ptr, int64_t* elem_order, int32_t* seg_bin,
                           int32_t* seg_slice, int64_t* seg_begin, uint8_t* seg_bad, tk_mem mem);

/* ---- factors --------------------------------------------------------------------------------- */

/* F: L_n x K_n row-major FP64.  The library keeps the FP64 master and derives
 * its FP32/BF16 working copies. */
tk_status tk_set_factor(tk_ctx* ctx, int n, const double* F, tk_mem mem);
tk_status tk_get_factor(tk_ctx* ctx, int n, double* F, tk_mem mem);

/* ---- the hot path ---------------------------------------------------------------------------- */

/* Shape of mode n's compact penultimate matrix: R_n nonempty slices x Khat_n. */
tk_status tk_ttm_shape(tk_ctx* ctx, int n, int64_t* R_n, int64_t* Khat_n);
/* TTM-chain along mode n with the current factors (eq. 1): Y gets the rows of
 * the nonempty slices in ascending slice id (R_n x Khat_n, row-major FP32);
 * row_slice (may be NULL) gets their slice ids (int32).  With prec = TK_BF16
 * the Kronecker tiles are BF16 on the matrix cores (where such a kernel runs).
 * A 16-byte aligned device Y is written in place; any other Y is filled
 * through the library's own buffer and copied. */
tk_status tk_ttm_chain(tk_ctx* ctx, int n, float* Y, int32_t* row_slice, tk_mem mem);
/* Size of the library's static scratch array per GPU (bytes), used by
 * tk_ttm_chain_noalloc. */
#define TK_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * TTM-chain as tk_ttm_chain (same kernels, same results bit for bit), with no
 * allocation of any kind (no hipMalloc, hipFree or allocating library call,
 * and no memset node).  Y (R_n x Khat_n FP32, 16-byte aligned) and row_slice
 * (R_n int32, may be NULL) must be device memory of the context's GPU
 * (TK_ERR_INVALID_ARG otherwise).  The partial rows of
 * slices split across bins live in a static array of
 * TK_NOALLOC_SCRATCH_BYTES per GPU (set up by tk_create, held until the
 * process ends): a mode whose split slices need more (Khat_n * 4 bytes per
 * partial row) gives TK_ERR_UNSUPPORTED and nothing is launched.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (other streams,
 * other contexts, other threads) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero (every partial row is written
 * before it is read). */
tk_status tk_ttm_chain_noalloc(tk_ctx* ctx, int n, float* Y, int32_t* row_slice);

/* Run `iters` HOOI invocations (Section 2.2): for each mode in turn, TTM-chain,
 * Gram, FP64 eigensolve, U = Y V S^-1, CholeskyQR2, new factor.  The
 * eigensolve is dense for Khat up to about 100 and a block Krylov method
 * (warm-started from the mode's previous eigenvectors) for Khat >= 192.
 * With prec = TK_BF16 and refine = 1 the last invocation runs in FP32.
 * fit_per_iter (host, may be NULL) gets 1 - sqrt(max(0, ||T||^2 - ||G||^2))/||T||
 * after each invocation. */
tk_status tk_hooi_iterate(tk_ctx* ctx, int iters, double* fit_per_iter);

/* Initial factors from a higher-order SVD of T (Section 2.2: HOOI starts from
 * HOSVD factors or from random ones).  F_n becomes the leading K_n left
 * singular vectors of T_(n) Omega_n, where Omega_n is the Kronecker product of
 * the sketch matrices Omega_j, j != n: a randomized range finder for T_(n)
 * whose test matrix is applied through the TTM-chain (eq. 1), so
 * T_(n) Omega_n = Y_(n) with the sketches in place of the factors.  sketch[j]
 * is L_j x K_j row-major FP64 (host or device per mem), drawn by the caller
 * (e.g. independent standard normal entries); it is read, not kept.  For a
 * tensor of multilinear rank at most (K_1..K_N) and sketches in general
 * position the result spans exactly the column space of every T_(n), i.e. it
 * is the truncated HOSVD.  All modes use the sketches (a Jacobi sweep) in FP32
 * whatever the options say; rank-deficient modes are completed as in
 * tk_hooi_iterate.  fit (host, may be NULL) gets the fit of the initial
 * decomposition.  Errors as tk_hooi_iterate; TK_ERR_STATE before tk_set_ranks. */
tk_status tk_init_hosvd(tk_ctx* ctx, const double* const* sketch, tk_mem mem, double* fit);
/* Core G = T x_1 F_1^T ... x_N F_N^T with the current factors (FP64, prod K
 * entries, first index fastest) and the fit; either output may be NULL. */
tk_status tk_core(tk_ctx* ctx, double* core, double* fit, tk_mem mem);
/* Milliseconds of the last tk_hooi_iterate per step; names[i] is a static string.
 * *count is in/out: capacity in, entries written out. */
tk_status tk_get_timings(tk_ctx* ctx, double* ms, const char** names, int* count);

/* Event counts since the context was created (names[i] static strings):
 *   eig_krylov_solves, eig_krylov_cycles, eig_dense_fallbacks, rank_completions (factors
 *   completed after a rank-deficient penultimate matrix).
 * *count is in/out: capacity in, entries written out. */
tk_status tk_get_counters(tk_ctx* ctx, int64_t* values, const char** names, int* count);

/* ---- differentiation form (Tucker completion; not in the paper) -------------------------------- */

/* Load an observation list (never merged: repeated coordinates stay separate
 * terms of the loss).  Same limits as tk_load_coo. */
tk_status tk_load_obs(tk_ctx* ctx, int N, const int64_t* dims, const int32_t* ranks, int64_t n_obs,
                      const int32_t* const* idx, tk_mem mem);
/* model[e] = sum_c G[c] prod_n F_n[l_n(e), c_n]; core (prod K, first index
 * fastest) and F[n] (dims[n] x ranks[n], row-major) are FP32 in `mem`. */
tk_status tk_tucker_eval(tk_ctx* ctx, const float* core, const float* const* F, float* model, tk_mem mem);
/* Given g[e] = dL/dmodel[e]: dcore = sum_e g_e (x)_n F_n[l_n(e)] and
 * dF[n] = Y^g_(n) G_(n)^T, where Y^g_(n) is the TTM-chain (eq. 1) of the
 * observations with values g.  Outputs are overwritten (FP32). */
tk_status tk_tucker_adjoint(tk_ctx* ctx, const float* g, const float* core, const float* const* F,
                            float* dcore, float* const* dF, tk_mem mem);

#ifdef __cplusplus
}
#endif
#endif /* TUCKER_HIP_H */
