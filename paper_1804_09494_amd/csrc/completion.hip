// Differentiation form: Tucker completion over a list of observed coordinates.
//
//   model:    m_e = sum_c G[c] prod_n F_n[l_n(e), c_n]
//   adjoint:  given g_e = dL/dm_e,
//             Y^g_(n) = TTM-chain of the observations with values g (eq. 1),
//             dF_n    = Y^g_(n) G_(n)^T   (row i only from slice i),
//             dG      = F_1^T Y^g_(1) folded back (first index fastest).
// The adjoint reuses the TTM-chain kernel on a Lite partition of the
// observations along each mode; Kronecker rows are recomputed from the factors,
// never stored.  Observations are a list: repeated coordinates stay separate.
#include <cmath>

#include "common.hpp"

namespace tk {

__global__ void k_obs_validate(const int32_t* __restrict__ idx, int64_t m, int64_t L, int32_t* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = idx[i];
    bad |= (v < 0 || (int64_t)v >= L);
  }
  if (bad) atomicOr(flag, 1);
}

void load_obs(Ctx* c, int N, const int64_t* dims, const int32_t* ranks, int64_t n_obs, const int32_t* const* idx,
              tk_mem mem) {
  ObsSet& o = c->obs;
  c->have_obs = false;
  for (int j = 0; j < 8; ++j) {
    o.idx[j].release();
    o.plan[j] = ModePlan();
    o.F32[j].release();
  }
  o.N = N;
  o.n_obs = n_obs;
  for (int j = 0; j < 8; ++j) {
    o.dims[j] = j < N ? dims[j] : 0;
    o.K[j] = j < N ? ranks[j] : 0;
  }
  Buf flag(c, sizeof(int32_t));
  TK_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int32_t), c->stream));
  for (int j = 0; j < N; ++j) {
    o.idx[j].alloc(c, sizeof(int32_t) * (size_t)std::max<int64_t>(n_obs, 1));
    copy_in(c, o.idx[j].as<int32_t>(), idx ? idx[j] : nullptr, (size_t)n_obs, mem);
    hipLaunchKernelGGL(k_obs_validate, dim3(grid_for(n_obs, 256, 4096)), dim3(256), 0, c->stream,
                       o.idx[j].as<int32_t>(), n_obs, dims[j], flag.as<int32_t>());
    TK_CHECK_LAUNCH();
  }
  int32_t h = 0;
  d2h(c, &h, flag.as<int32_t>(), 1);
  c->sync();
  TK_REQUIRE(h == 0, TK_ERR_INVALID_ARG, "tk_load_obs: a coordinate is out of range");
  int64_t maxY = 1;
  for (int n = 0; n < N; ++n) {
    int64_t khat = 1;
    for (int j = 0; j < N; ++j)
      if (j != n) khat *= ranks[j];
    build_plan(c, o.plan[n], N, n, dims, n_obs, o.idx, nullptr, khat, ttm_tile_width(N, ranks, n), 1024, true);
    maxY = std::max(maxY, o.plan[n].L_nz * khat);
  }
  for (int j = 0; j < N; ++j) {
    o.kp[j] = ranks[j] <= 16 ? 16 : (ranks[j] + 3) & ~3;
    o.F32[j].alloc(c, sizeof(float) * (size_t)dims[j] * o.kp[j]);
  }
  o.gl.alloc(c, sizeof(float) * (size_t)std::max<int64_t>(n_obs, 1));
  o.Yg.alloc(c, sizeof(float) * (size_t)maxY);
  int64_t pk = 1;
  for (int j = 0; j < N; ++j) pk *= ranks[j];
  o.G32.alloc(c, sizeof(float) * (size_t)pk);
  c->have_obs = true;
}

// ---- model values ---------------------------------------------------------------------------------

struct FPtrs {
  const float* p[8];
};
struct IPtrs {
  const int32_t* p[8];
};

// One thread per observation: contract the core with the first mode's row
// (kept in registers, K0 <= K0MAX), then fold the remaining modes' rows in
// with a carry chain over the remaining digits.
template <int K0MAX>
__global__ __launch_bounds__(256) void k_eval(FPtrs F, IPtrs ip, int N, int32_t K0, const int32_t* __restrict__ Kd,
                                              const float* __restrict__ Gin, int64_t n_obs, int64_t pK, int use_lds,
                                              float* __restrict__ out) {
  extern __shared__ float gsh[];
  const float* G = Gin;
  if (use_lds) {
    for (int64_t i = threadIdx.x; i < pK; i += blockDim.x) gsh[i] = Gin[i];
    __syncthreads();
    G = gsh;
  }
  int32_t Kl[8];
  for (int j = 0; j < N; ++j) Kl[j] = Kd[j];
  const int64_t rest = pK / K0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_obs; e += (int64_t)gridDim.x * blockDim.x) {
    float a[K0MAX];
    const float* ar = F.p[0] + (int64_t)ip.p[0][e] * K0;
#pragma unroll
    for (int d = 0; d < K0MAX; ++d) a[d] = (d < K0) ? ar[d] : 0.f;
    const float* rows[8];
    for (int j = 1; j < N; ++j) rows[j] = F.p[j] + (int64_t)ip.p[j][e] * Kl[j];
    float lvl[8];
    for (int j = 0; j < 8; ++j) lvl[j] = 0.f;
    int dig[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t r = 0; r < rest; ++r) {
      const float* g = G + r * K0;
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < K0MAX; ++d)
        if (d < K0) s = fmaf(a[d], g[d], s);
      // carry chain over the remaining modes (mode 1 fastest)
      float v = s;
      int j = 1;
      for (; j < N; ++j) {
        lvl[j] = fmaf(rows[j][dig[j]], v, lvl[j]);
        if (++dig[j] < Kl[j]) break;
        dig[j] = 0;
        v = lvl[j];
        lvl[j] = 0.f;
      }
      if (j == N) lvl[0] += v;  // every digit wrapped: v is a completed full contraction
    }
    out[e] = lvl[0];
  }
}

static const float* dev_copy_f32(Ctx* c, Buf& tmp, const float* src, size_t n, tk_mem mem) {
  if (mem == TK_MEM_DEVICE) return src;
  tmp.alloc(c, sizeof(float) * std::max<size_t>(n, 1));
  h2d(c, tmp.as<float>(), src, n);
  return tmp.as<float>();
}

void obs_eval(Ctx* c, const float* core, const float* const* F, float* model, tk_mem mem) {
  ObsSet& o = c->obs;
  const int N = o.N;
  int64_t pK = 1;
  for (int j = 0; j < N; ++j) pK *= o.K[j];
  Buf tF[8], tG, tOut, tK(c, sizeof(int32_t) * 8);
  FPtrs fp{};
  IPtrs ip{};
  for (int j = 0; j < N; ++j) {
    fp.p[j] = dev_copy_f32(c, tF[j], F[j], (size_t)o.dims[j] * o.K[j], mem);
    ip.p[j] = o.idx[j].as<int32_t>();
  }
  const float* G = dev_copy_f32(c, tG, core, (size_t)pK, mem);
  h2d(c, tK.as<int32_t>(), o.K, 8);
  float* out = model;
  if (mem == TK_MEM_HOST) {
    tOut.alloc(c, sizeof(float) * (size_t)std::max<int64_t>(o.n_obs, 1));
    out = tOut.as<float>();
  }
  if (o.n_obs > 0) {
    const int use_lds = (size_t)pK * 4 <= std::min<size_t>(c->lds_per_block, 65536) ? 1 : 0;
    const size_t lds = use_lds ? (size_t)pK * 4 : 0;
    if (o.K[0] <= 16)
      hipLaunchKernelGGL(k_eval<16>, dim3(grid_for(o.n_obs, 256, 8192)), dim3(256), lds, c->stream, fp, ip, N, o.K[0],
                         tK.as<int32_t>(), G, o.n_obs, pK, use_lds, out);
    else
      hipLaunchKernelGGL(k_eval<64>, dim3(grid_for(o.n_obs, 256, 8192)), dim3(256), lds, c->stream, fp, ip, N, o.K[0],
                         tK.as<int32_t>(), G, o.n_obs, pK, use_lds, out);
    TK_CHECK_LAUNCH();
  }
  if (mem == TK_MEM_HOST) d2h(c, model, out, (size_t)o.n_obs);
  c->sync();
}

// ---- adjoint ----------------------------------------------------------------------------------

__global__ void k_pad_copy(const float* __restrict__ src, int64_t L, int K, float* __restrict__ dst, int kp) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L * kp; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / kp;
    const int k = (int)(i - l * kp);
    dst[i] = k < K ? src[l * K + k] : 0.f;
  }
}

__global__ void k_gather_layout(const float* __restrict__ g, const uint32_t* __restrict__ order, int64_t m,
                                float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t e = order[i];
    out[i] = e == 0xffffffffu ? 0.f : g[e];   // padding positions carry zero
  }
}

// Linear core index of (c_n = k, other modes from col with the first remaining mode fastest).
__device__ __forceinline__ int64_t core_lin(int N, const int32_t* K, int n, int k, int64_t col) {
  int64_t lin = 0, stride = 1;
  for (int j = 0; j < N; ++j) {
    int d;
    if (j == n) {
      d = k;
    } else {
      d = (int)(col % K[j]);
      col /= K[j];
    }
    lin += d * stride;
    stride *= K[j];
  }
  return lin;
}

// dF[row_slice[r]][k] = sum_col Yg[r][col] * G_(n)[k][col]; G_(n) staged in LDS.
__global__ __launch_bounds__(256) void k_dF(const float* __restrict__ Yg, int64_t R, int khat,
                                            const float* __restrict__ G, int N, const int32_t* __restrict__ Kd, int n,
                                            const int32_t* __restrict__ row_slice, float* __restrict__ dF) {
  extern __shared__ float gn[];  // K_n x khat
  int32_t K[8];
  for (int j = 0; j < N; ++j) K[j] = Kd[j];
  const int Kn = K[n];
  for (int i = threadIdx.x; i < Kn * khat; i += blockDim.x) {
    const int k = i / khat;
    const int64_t col = i - (int64_t)k * khat;
    gn[i] = G[core_lin(N, K, n, k, col)];
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R * Kn; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / Kn;
    const int k = (int)(i - r * Kn);
    const float* y = Yg + r * khat;
    const float* w = gn + k * khat;
    double s = 0.0;
    for (int col = 0; col < khat; ++col) s += (double)y[col] * (double)w[col];
    dF[(int64_t)row_slice[r] * Kn + k] = (float)s;
  }
}

// dcore[c0 + K0 * col] = sum_r F0[slice(r)][c0] * Yg[r][col]  (FP64 accumulation, fixed order per entry)
__global__ __launch_bounds__(256) void k_dcore(const float* __restrict__ Yg, int64_t R, int khat,
                                               const float* __restrict__ F0, int K0, int kp0,
                                               const int32_t* __restrict__ row_slice, float* __restrict__ dcore) {
  const int64_t nent = (int64_t)K0 * khat;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nent; i += (int64_t)gridDim.x * blockDim.x) {
    const int c0 = (int)(i % K0);
    const int64_t col = i / K0;
    double s = 0.0;
    for (int64_t r = 0; r < R; ++r) s += (double)F0[(int64_t)row_slice[r] * kp0 + c0] * (double)Yg[r * khat + col];
    dcore[i] = (float)s;
  }
}

void obs_adjoint(Ctx* c, const float* g, const float* core, const float* const* F, float* dcore, float* const* dF,
                 tk_mem mem) {
  ObsSet& o = c->obs;
  const int N = o.N;
  int64_t pK = 1;
  for (int j = 0; j < N; ++j) pK *= o.K[j];
  Buf tF[8], tG, tg, tK(c, sizeof(int32_t) * 8);
  h2d(c, tK.as<int32_t>(), o.K, 8);
  for (int j = 0; j < N; ++j) {
    const float* src = dev_copy_f32(c, tF[j], F[j], (size_t)o.dims[j] * o.K[j], mem);
    hipLaunchKernelGGL(k_pad_copy, dim3(grid_for(o.dims[j] * o.kp[j], 256)), dim3(256), 0, c->stream, src, o.dims[j],
                       o.K[j], o.F32[j].as<float>(), o.kp[j]);
    TK_CHECK_LAUNCH();
  }
  const float* G = dev_copy_f32(c, tG, core, (size_t)pK, mem);
  const float* gd = dev_copy_f32(c, tg, g, (size_t)o.n_obs, mem);
  const float* Fp[8];
  for (int j = 0; j < N; ++j) Fp[j] = o.F32[j].as<float>();
  for (int n = 0; n < N; ++n) {
    ModePlan& pl = o.plan[n];
    const int khat = (int)pl.khat;
    ensure(c, o.gl, sizeof(float) * (size_t)std::max<int64_t>(pl.m_pad, 1));
    hipLaunchKernelGGL(k_gather_layout, dim3(grid_for(pl.m_pad, 256)), dim3(256), 0, c->stream, gd,
                       pl.order_pad.as<uint32_t>(), pl.m_pad, o.gl.as<float>());
    TK_CHECK_LAUNCH();
    float* Yg = o.Yg.as<float>();
    ttm_run(c, pl, N, n, o.K, Fp, o.kp, o.gl.as<float>(), o.n_obs, Yg);
    Buf tdF;
    float* dFn = dF[n];
    if (mem == TK_MEM_HOST) {
      tdF.alloc(c, sizeof(float) * (size_t)o.dims[n] * o.K[n]);
      dFn = tdF.as<float>();
    }
    TK_HIP(hipMemsetAsync(dFn, 0, sizeof(float) * (size_t)o.dims[n] * o.K[n], c->stream));
    if (pl.L_nz > 0) {
      const size_t lds = sizeof(float) * (size_t)o.K[n] * khat;
      TK_REQUIRE(lds <= c->lds_per_block, TK_ERR_UNSUPPORTED, "adjoint: K_n x Khat too large for LDS");
      hipLaunchKernelGGL(k_dF, dim3(grid_for(pl.L_nz * o.K[n], 256, 16384)), dim3(256), lds, c->stream, Yg, pl.L_nz,
                         khat, G, N, tK.as<int32_t>(), n, pl.row_slice.as<int32_t>(), dFn);
      TK_CHECK_LAUNCH();
    }
    if (mem == TK_MEM_HOST) d2h(c, dF[n], dFn, (size_t)o.dims[n] * o.K[n]);
    if (n == 0) {
      Buf tdc;
      float* dc = dcore;
      if (mem == TK_MEM_HOST) {
        tdc.alloc(c, sizeof(float) * (size_t)pK);
        dc = tdc.as<float>();
      }
      if (pl.L_nz > 0) {
        hipLaunchKernelGGL(k_dcore, dim3(grid_for(pK, 256)), dim3(256), 0, c->stream, Yg, pl.L_nz, khat,
                           o.F32[0].as<float>(), o.K[0], o.kp[0], pl.row_slice.as<int32_t>(), dc);
        TK_CHECK_LAUNCH();
      } else {
        TK_HIP(hipMemsetAsync(dc, 0, sizeof(float) * (size_t)pK, c->stream));
      }
      if (mem == TK_MEM_HOST) d2h(c, dcore, dc, (size_t)pK);
      c->sync();
    }
    c->sync();
  }
}

}  // namespace tk
