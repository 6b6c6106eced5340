// Loading and coalescing the element list E (Section 3 keeps the tensor as a
// set of elements, each a coordinate vector and a value).
//
// The elements arrive in one or more appends (tk_load_coo_begin / _append /
// _end; tk_load_coo is one append).  Steps, all on the device:
//   1. validate coordinates (0 <= l_n < L_n) and values (finite) of each
//      append -> one flag, read at the end;
//   2. LSD radix sort of element positions by the coordinates, least
//      significant mode first, so the result is lexicographic with l_1 most
//      significant; the sort is stable, so repeated coordinates keep input order;
//   3. mark the first element of every run of equal coordinates, scan the
//      marks into run ids;
//   4. one thread per run sums its values sequentially in FP64 (input order)
//      and rounds once to FP32;
//   5. ||T||^2 in FP64 by a two-level fixed-order reduction.
#include "common.hpp"

namespace tk {

__global__ void k_validate(const int32_t* __restrict__ idx, int64_t m, int64_t L, int32_t* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = idx[i];
    bad |= (v < 0 || (int64_t)v >= L);
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_validate_vals(const float* __restrict__ vals, int64_t m, int32_t* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(vals[i]);
  if (bad) atomicOr(flag, 2);
}

// The element-position type PT is uint32_t below 2^32 elements, else uint64_t.
template <class PT>
__global__ void k_iota(PT* __restrict__ out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (PT)i;
}

template <class PT>
__global__ void k_gather_key(const int32_t* __restrict__ idx, const PT* __restrict__ perm, uint32_t* __restrict__ key,
                             int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = (uint32_t)idx[perm[i]];
}

// run_start[s] = 1 when sorted element s starts a new coordinate.
struct IdxPtrs {
  const int32_t* p[8];
};

// Each lane gathers its own element's coordinates once; the previous sorted
// element's come from the lane before it (consecutive positions share a
// wave), and only lane 0 gathers them itself.  A lane that runs an iteration
// has its left neighbour running it too, since positions increase with the
// lane.
template <class PT>
__global__ void k_mark_runs(IdxPtrs idx, int N, const PT* __restrict__ perm, int64_t m, PT* __restrict__ mark) {
  const int lane = threadIdx.x & 63;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    const PT a = perm[s];
    const PT b = (lane == 0 && s > 0) ? perm[s - 1] : a;
    int d = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < N) {
        const int32_t cur = idx.p[j][a];
        int32_t prev = __shfl_up(cur, 1, 64);
        if (lane == 0) prev = idx.p[j][b];
        d |= (cur != prev);
      }
    }
    mark[s] = s == 0 ? (PT)1 : (PT)d;
  }
}

// Run r starts at sorted position s where mark[s] == 1 and runid[s] = r.
template <class PT>
__global__ void k_run_starts(const PT* __restrict__ mark, const PT* __restrict__ runid, int64_t m,
                             PT* __restrict__ start) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x)
    if (mark[s]) start[runid[s]] = (PT)s;
}

struct OutPtrs {
  int32_t* p[8];
};

// One thread per run: its values summed in FP64 in input order (the stable
// sort keeps that order inside a run), rounded once.  Loads of 16 elements are
// issued before their adds, which stay in order.
template <class PT>
__global__ void k_merge_runs(IdxPtrs idx, int N, const float* __restrict__ vals, const PT* __restrict__ perm,
                             const PT* __restrict__ start, int64_t runs, int64_t m, OutPtrs out_idx,
                             float* __restrict__ out_val) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < runs; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = (int64_t)start[r];
    const int64_t b = (r + 1 < runs) ? (int64_t)start[r + 1] : m;
    const PT e0 = perm[a];
    double s = 0.0;
    int64_t k = a;
    for (; k + 16 <= b; k += 16) {
      float v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = vals[perm[k + i]];
#pragma unroll
      for (int i = 0; i < 16; ++i) s += (double)v[i];
    }
    for (; k < b; ++k) s += (double)vals[perm[k]];
    out_val[r] = (float)s;
    for (int j = 0; j < N; ++j) out_idx.p[j][r] = idx.p[j][e0];
  }
}

// Elements known to be distinct: the sorted list itself.
template <class PT>
__global__ void k_gather_sorted(IdxPtrs idx, int N, const float* __restrict__ vals, const PT* __restrict__ perm,
                                int64_t m, OutPtrs out_idx, float* __restrict__ out_val) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    const PT e = perm[s];
    out_val[s] = vals[e];
    for (int j = 0; j < N; ++j) out_idx.p[j][s] = idx.p[j][e];
  }
}

// Sum of squares in FP64: fixed per-block order, then a single block over partials.
__global__ void k_sumsq_blocks(const float* __restrict__ v, int64_t m, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    double x = v[i];
    s += x * x;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

static int bits_for(int64_t L) {
  int b = 0;
  while (b < 32 && ((int64_t)1 << b) < L) ++b;
  return b < 1 ? 1 : b;
}

// ---- streamed load: begin, appends, end ---------------------------------------------------------

void load_begin(Ctx* c, int N, const int64_t* dims, int64_t nnz, unsigned flags) {
  LoadState& ls = c->load;
  ls = LoadState();
  for (int j = 0; j < N; ++j) ls.raw[j].alloc(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
  ls.rawv.alloc(c, sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
  ls.flag.alloc(c, sizeof(int32_t));
  TK_HIP(hipMemsetAsync(ls.flag.get(), 0, sizeof(int32_t), c->stream));
  ls.N = N;
  for (int j = 0; j < 8; ++j) ls.dims[j] = j < N ? dims[j] : 0;
  ls.nnz = nnz;
  ls.filled = 0;
  ls.flags = flags;
  ls.active = true;
}

void load_append(Ctx* c, int64_t count, const int32_t* const* idx, const float* vals, tk_mem mem) {
  LoadState& ls = c->load;
  const int B = 256;
  const int64_t off = ls.filled;
  for (int j = 0; j < ls.N; ++j) {
    int32_t* dst = ls.raw[j].as<int32_t>() + off;
    copy_in(c, dst, idx[j], (size_t)count, mem);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(count, B, 4096)), dim3(B), 0, c->stream, dst, count, ls.dims[j],
                       ls.flag.as<int32_t>());
    TK_CHECK_LAUNCH();
  }
  float* dv = ls.rawv.as<float>() + off;
  copy_in(c, dv, vals, (size_t)count, mem);
  hipLaunchKernelGGL(k_validate_vals, dim3(grid_for(count, B, 4096)), dim3(B), 0, c->stream, dv, count,
                     ls.flag.as<int32_t>());
  TK_CHECK_LAUNCH();
  // the caller may reuse its buffers once the call returns
  c->sync();
  ls.filled += count;
}

template <class PT>
static void coalesce(Ctx* c, int N, const int64_t* dims, int64_t nnz, Buf* raw, Buf& rawv, bool assume_unique) {
  const int B = 256;
  // LSD sort by coordinates, least significant mode (N-1) first; stable, so
  // repeated coordinates keep input order
  const size_t n1 = (size_t)std::max<int64_t>(nnz, 1);
  Buf perm(c, sizeof(PT) * n1), perm2(c, sizeof(PT) * n1);
  Buf key(c, sizeof(uint32_t) * n1), key2(c, sizeof(uint32_t) * n1);
  hipLaunchKernelGGL(k_iota<PT>, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, perm.as<PT>(), nnz);
  TK_CHECK_LAUNCH();
  for (int j = N - 1; j >= 0; --j) {
    hipLaunchKernelGGL(k_gather_key<PT>, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, raw[j].as<int32_t>(),
                       perm.as<PT>(), key.as<uint32_t>(), nnz);
    TK_CHECK_LAUNCH();
    sort_pairs_u32_key(c, key.as<uint32_t>(), key2.as<uint32_t>(), perm.as<PT>(), perm2.as<PT>(), nnz,
                       bits_for(dims[j]));
    std::swap(perm, perm2);
  }
  perm2.release();
  key.release();
  key2.release();

  IdxPtrs ip{};
  for (int j = 0; j < N; ++j) ip.p[j] = raw[j].as<int32_t>();
  int64_t runs = nnz;
  Buf mark, runid;
  if (!assume_unique && nnz > 0) {
    mark.alloc(c, sizeof(PT) * n1);
    runid.alloc(c, sizeof(PT) * n1);
    hipLaunchKernelGGL(k_mark_runs<PT>, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, ip, N, perm.as<PT>(), nnz,
                       mark.as<PT>());
    TK_CHECK_LAUNCH();
    exclusive_scan_pos(c, mark.as<PT>(), runid.as<PT>(), nnz);
    PT last_id = 0, last_mark = 0;
    d2h(c, &last_id, runid.as<PT>() + nnz - 1, 1);
    d2h(c, &last_mark, mark.as<PT>() + nnz - 1, 1);
    c->sync();
    runs = (int64_t)last_id + (int64_t)last_mark;
  }
  TK_REQUIRE(runs < ((int64_t)1 << 32), TK_ERR_UNSUPPORTED,
             "this build handles fewer than 2^32 distinct coordinates");
  for (int j = 0; j < 8; ++j) c->idx_c[j].release();
  c->val_c.release();
  OutPtrs op{};
  const size_t r1 = (size_t)std::max<int64_t>(runs, 1);
  for (int j = 0; j < N; ++j) {
    c->idx_c[j].alloc(c, sizeof(int32_t) * r1);
    op.p[j] = c->idx_c[j].as<int32_t>();
  }
  c->val_c.alloc(c, sizeof(float) * r1);
  if (runs > 0 && assume_unique) {
    hipLaunchKernelGGL(k_gather_sorted<PT>, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, ip, N, rawv.as<float>(),
                       perm.as<PT>(), nnz, op, c->val_c.as<float>());
    TK_CHECK_LAUNCH();
  } else if (runs > 0) {
    Buf start(c, sizeof(PT) * r1);
    hipLaunchKernelGGL(k_run_starts<PT>, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, mark.as<PT>(),
                       runid.as<PT>(), nnz, start.as<PT>());
    TK_CHECK_LAUNCH();
    mark.release();
    runid.release();
    hipLaunchKernelGGL(k_merge_runs<PT>, dim3(grid_for(runs, B)), dim3(B), 0, c->stream, ip, N, rawv.as<float>(),
                       perm.as<PT>(), start.as<PT>(), runs, nnz, op, c->val_c.as<float>());
    TK_CHECK_LAUNCH();
    c->sync();
  }
  c->m = runs;
}

void load_end(Ctx* c) {
  LoadState& ls = c->load;
  TK_REQUIRE(ls.filled == ls.nnz, TK_ERR_INVALID_ARG,
             "tk_load_coo_end: " + std::to_string(ls.filled) + " of " + std::to_string(ls.nnz) +
                 " announced elements were appended");
  int32_t hflag = 0;
  d2h(c, &hflag, ls.flag.as<int32_t>(), 1);
  c->sync();
  if (hflag & 1) fail(TK_ERR_INVALID_ARG, "tk_load_coo: a coordinate is out of range");
  if (hflag & 2) fail(TK_ERR_INVALID_ARG, "tk_load_coo: a value is NaN or Inf");
  const int N = ls.N;
  const bool unique = (ls.flags & TK_ASSUME_UNIQUE) != 0;
  if (ls.nnz < ((int64_t)1 << 32))
    coalesce<uint32_t>(c, N, ls.dims, ls.nnz, ls.raw, ls.rawv, unique);
  else
    coalesce<uint64_t>(c, N, ls.dims, ls.nnz, ls.raw, ls.rawv, unique);
  for (int j = 0; j < 8; ++j) ls.raw[j].release();
  ls.rawv.release();
  ls.active = false;

  // ||T||^2
  const int nb = 1024;
  Buf part(c, sizeof(double) * (nb + 1));
  hipLaunchKernelGGL(k_sumsq_blocks, dim3(nb), dim3(256), 0, c->stream, c->val_c.as<float>(), c->m,
                     part.as<double>());
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, c->stream, part.as<double>(), nb, part.as<double>() + nb);
  TK_CHECK_LAUNCH();
  double nsq = 0;
  d2h(c, &nsq, part.as<double>() + nb, 1);
  c->sync();

  c->N = N;
  for (int j = 0; j < 8; ++j) c->dims[j] = j < N ? ls.dims[j] : 0;
  c->norm_sq = nsq;
  c->have_tensor = true;
}

}  // namespace tk
