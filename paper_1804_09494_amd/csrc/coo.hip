// Loading and coalescing the element list E (Section 3 keeps the tensor as a
// set of elements, each a coordinate vector and a value).
//
// Steps, all on the device:
//   1. validate coordinates (0 <= l_n < L_n) and values (finite) -> one flag;
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

__global__ void k_iota_u32(uint32_t* __restrict__ out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)i;
}

__global__ void k_gather_key(const int32_t* __restrict__ idx, const uint32_t* __restrict__ perm,
                             uint32_t* __restrict__ key, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = (uint32_t)idx[perm[i]];
}

// run_start[s] = 1 when sorted element s starts a new coordinate.
struct IdxPtrs {
  const int32_t* p[8];
};

__global__ void k_mark_runs(IdxPtrs idx, int N, const uint32_t* __restrict__ perm, int64_t m,
                            int32_t* __restrict__ mark) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    int32_t f = 1;
    if (s > 0) {
      uint32_t a = perm[s], b = perm[s - 1];
      f = 0;
      for (int j = 0; j < N; ++j) f |= (idx.p[j][a] != idx.p[j][b]);
    }
    mark[s] = f;
  }
}

// Run r starts at sorted position s where mark[s] == 1 and runid[s] = r.
__global__ void k_run_starts(const int32_t* __restrict__ mark, const int32_t* __restrict__ runid, int64_t m,
                             uint32_t* __restrict__ start) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x)
    if (mark[s]) start[runid[s]] = (uint32_t)s;
}

struct OutPtrs {
  int32_t* p[8];
};

__global__ void k_merge_runs(IdxPtrs idx, int N, const float* __restrict__ vals, const uint32_t* __restrict__ perm,
                             const uint32_t* __restrict__ start, int64_t runs, int64_t m, OutPtrs out_idx,
                             float* __restrict__ out_val) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < runs; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = start[r];
    int64_t b = (r + 1 < runs) ? (int64_t)start[r + 1] : m;
    uint32_t e0 = perm[a];
    double s = 0.0;
    for (int64_t k = a; k < b; ++k) s += (double)vals[perm[k]];
    out_val[r] = (float)s;
    for (int j = 0; j < N; ++j) out_idx.p[j][r] = idx.p[j][e0];
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

void load_coo(Ctx* c, int N, const int64_t* dims, int64_t nnz, const int32_t* const* idx, const float* vals,
              tk_mem mem) {
  const int B = 256;
  // raw copies
  Buf raw[8];
  Buf rawv(c, sizeof(float) * (size_t)nnz);
  for (int j = 0; j < N; ++j) {
    raw[j].alloc(c, sizeof(int32_t) * (size_t)nnz);
    copy_in(c, raw[j].as<int32_t>(), idx[j], (size_t)nnz, mem);
  }
  copy_in(c, rawv.as<float>(), vals, (size_t)nnz, mem);

  Buf flag(c, sizeof(int32_t));
  TK_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int32_t), c->stream));
  for (int j = 0; j < N; ++j) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(nnz, B, 4096)), dim3(B), 0, c->stream, raw[j].as<int32_t>(), nnz,
                       dims[j], flag.as<int32_t>());
    TK_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_validate_vals, dim3(grid_for(nnz, B, 4096)), dim3(B), 0, c->stream, rawv.as<float>(), nnz,
                     flag.as<int32_t>());
  TK_CHECK_LAUNCH();
  int32_t hflag = 0;
  d2h(c, &hflag, flag.as<int32_t>(), 1);
  c->sync();
  if (hflag & 1) fail(TK_ERR_INVALID_ARG, "tk_load_coo: a coordinate is out of range");
  if (hflag & 2) fail(TK_ERR_INVALID_ARG, "tk_load_coo: a value is NaN or Inf");

  // LSD sort by coordinates, least significant mode (N-1) first.
  Buf perm(c, sizeof(uint32_t) * (size_t)nnz), perm2(c, sizeof(uint32_t) * (size_t)nnz);
  Buf key(c, sizeof(uint32_t) * (size_t)nnz), key2(c, sizeof(uint32_t) * (size_t)nnz);
  hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, perm.as<uint32_t>(), nnz);
  TK_CHECK_LAUNCH();
  for (int j = N - 1; j >= 0; --j) {
    hipLaunchKernelGGL(k_gather_key, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, raw[j].as<int32_t>(),
                       perm.as<uint32_t>(), key.as<uint32_t>(), nnz);
    TK_CHECK_LAUNCH();
    sort_pairs_u32(c, key.as<uint32_t>(), key2.as<uint32_t>(), perm.as<uint32_t>(), perm2.as<uint32_t>(), nnz,
                   bits_for(dims[j]));
    std::swap(perm, perm2);
  }
  key2.release();

  IdxPtrs ip{};
  for (int j = 0; j < N; ++j) ip.p[j] = raw[j].as<int32_t>();
  Buf mark(c, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)), runid(c, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t runs = 0;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_mark_runs, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, ip, N, perm.as<uint32_t>(), nnz,
                       mark.as<int32_t>());
    TK_CHECK_LAUNCH();
    exclusive_scan_i32(c, mark.as<int32_t>(), runid.as<int32_t>(), nnz);
    int32_t last_id = 0, last_mark = 0;
    d2h(c, &last_id, runid.as<int32_t>() + nnz - 1, 1);
    d2h(c, &last_mark, mark.as<int32_t>() + nnz - 1, 1);
    c->sync();
    runs = (int64_t)last_id + last_mark;
  }
  Buf start(c, sizeof(uint32_t) * (size_t)(runs > 0 ? runs : 1));
  for (int j = 0; j < 8; ++j) c->idx_c[j].release();
  c->val_c.release();
  OutPtrs op{};
  for (int j = 0; j < N; ++j) {
    c->idx_c[j].alloc(c, sizeof(int32_t) * (size_t)(runs > 0 ? runs : 1));
    op.p[j] = c->idx_c[j].as<int32_t>();
  }
  c->val_c.alloc(c, sizeof(float) * (size_t)(runs > 0 ? runs : 1));
  if (runs > 0) {
    hipLaunchKernelGGL(k_run_starts, dim3(grid_for(nnz, B)), dim3(B), 0, c->stream, mark.as<int32_t>(),
                       runid.as<int32_t>(), nnz, start.as<uint32_t>());
    TK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_merge_runs, dim3(grid_for(runs, B)), dim3(B), 0, c->stream, ip, N, rawv.as<float>(),
                       perm.as<uint32_t>(), start.as<uint32_t>(), runs, nnz, op, c->val_c.as<float>());
    TK_CHECK_LAUNCH();
  }
  // ||T||^2
  const int nb = 1024;
  Buf part(c, sizeof(double) * (nb + 1));
  hipLaunchKernelGGL(k_sumsq_blocks, dim3(nb), dim3(256), 0, c->stream, c->val_c.as<float>(), runs,
                     part.as<double>());
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, c->stream, part.as<double>(), nb, part.as<double>() + nb);
  TK_CHECK_LAUNCH();
  double nsq = 0;
  d2h(c, &nsq, part.as<double>() + nb, 1);
  c->sync();

  c->N = N;
  for (int j = 0; j < 8; ++j) c->dims[j] = j < N ? dims[j] : 0;
  c->m = runs;
  c->norm_sq = nsq;
  c->have_tensor = true;
}

}  // namespace tk
