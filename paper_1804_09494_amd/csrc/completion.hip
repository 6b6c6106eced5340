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

int uw_product(Ctx* c, const float* Y, int64_t R, int khat, const double* W, int K, double* U, double* part);
int uw_product_parts(int64_t R);

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
  {
    SortScratch ss;
    for (int n = 0; n < N; ++n) {
      int64_t khat = 1;
      for (int j = 0; j < N; ++j)
        if (j != n) khat *= ranks[j];
      build_plan(c, o.plan[n], N, n, dims, n_obs, o.idx, nullptr, khat, ttm_tile_width(N, ranks, n), 1024, true, ss,
                 n == N - 1);
      maxY = std::max(maxY, o.plan[n].L_nz * khat);
    }
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

typedef float floatx4_e __attribute__((ext_vector_type(4)));

// dst (L x kp) = src (L x K) with zero columns past K
__global__ void k_pad_copy(const float* __restrict__ src, int64_t L, int K, float* __restrict__ dst, int kp) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L * kp; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / kp;
    const int k = (int)(i - l * kp);
    dst[i] = k < K ? src[l * K + k] : 0.f;
  }
}

// Three modes, every rank <= 16, on the matrix cores, grouped by the slices
// of one mode c (the one with the fewest nonempty slices, so each slice holds
// many observations).  For an observation of slice l_c,
//   m = F_a[l_a]^T M F_b[l_b],  M[a][b] = sum_c G[a, b, c] F_c[l_c][c]
// (a < b the other two modes, G indexed with the first mode fastest).  The
// observations are walked in the layout of mode c's plan (bins of Lite
// segments, padded to multiples of four, a segment being one slice's run in
// one bin).  Per segment the wave forms M once, in the B-operand layout of
// v_mfma_f32_16x16x4_f32 (lane (q, j) holds M[4q + s][j], s = 0..3, the
// contraction index of step s being 4q + s); per block of 16 observations
// four MFMA steps give D = F_a-rows x M with A[i][4q + s] = F_a[l_a(i)][4q + s]
// (one 16-byte load per lane), and m_i = sum_j D[i][j] F_b[l_b(i)][j] is a sum
// over the 16 lanes of a row group.  Factors are the 16-float padded copies.
// Each observation's value goes to its own index (order_pad); padding
// positions are skipped.
__global__ __launch_bounds__(256) void k_eval3_slab(const int64_t* __restrict__ bin_pptr,
                                                    const int32_t* __restrict__ seg_ptr,
                                                    const int64_t* __restrict__ seg_pbegin,
                                                    const int32_t* __restrict__ seg_row,
                                                    const int32_t* __restrict__ row_slice,
                                                    const int32_t* __restrict__ lay_a, const int32_t* __restrict__ lay_b,
                                                    const uint32_t* __restrict__ order, const float* __restrict__ Fa,
                                                    const float* __restrict__ Fb, const float* __restrict__ Fc,
                                                    const float* __restrict__ G, int Ka, int Kb, int Kc, int sa,
                                                    int sb, int sc, int64_t P, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int j = lane & 15, q = lane >> 4;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); bin < P; bin += nw) {
    const int s0 = seg_ptr[bin], s1 = seg_ptr[bin + 1];
    for (int sg = s0; sg < s1; ++sg) {
      const int64_t pb = seg_pbegin[sg], pe = seg_pbegin[sg + 1];
      const int64_t lc = row_slice[seg_row[sg]];
      // M in the B-operand layout: Mr[s] = M[4q + s][j]
      float fc[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) fc[c] = Fc[lc * 16 + c];
      float Mr[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int a = 4 * q + s;
        float t = 0.f;
        if (a < Ka && j < Kb)
          for (int c = 0; c < Kc; ++c) t = fmaf(G[a * sa + j * sb + c * sc], fc[c], t);
        Mr[s] = t;
      }
      for (int64_t p0 = pb; p0 < pe; p0 += 16) {
        const int64_t pi = p0 + j;   // this lane's observation for the A operand
        const bool ok = pi < pe;
        const int la = ok ? lay_a[pi] : 0;
        const floatx4_e xa = ok ? *reinterpret_cast<const floatx4_e*>(Fa + (int64_t)la * 16 + 4 * q)
                                : floatx4_e{0.f, 0.f, 0.f, 0.f};
        floatx4_e D = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) D = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[s], Mr[s], D, 0, 0, 0);
        // D[4q + r][j] in register r: times F_b[l_b(obs 4q + r)][j], summed over the row group
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t pr = p0 + 4 * q + r;
          const bool okr = pr < pe;
          const float v = okr ? D[r] * Fb[(int64_t)lay_b[pr] * 16 + j] : 0.f;
          float w = v;
#pragma unroll
          for (int x = 8; x >= 1; x >>= 1) w += __shfl_xor(w, x, 16);
          if (j == 0 && okr) {
            const uint32_t e = order[pr];
            if (e != 0xffffffffu) out[e] = w;
          }
        }
      }
    }
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
  if (o.n_obs > 0 && N == 3 && o.K[0] <= 16 && o.K[1] <= 16 && o.K[2] <= 16) {
    // group by the mode with the fewest nonempty slices; factors as 16-float rows
    int mc = 0;
    for (int jn = 1; jn < 3; ++jn)
      if (o.plan[jn].L_nz < o.plan[mc].L_nz) mc = jn;
    const int ma = mc == 0 ? 1 : 0, mb = mc == 2 ? 1 : 2;
    for (int jn = 0; jn < 3; ++jn) {
      hipLaunchKernelGGL(k_pad_copy, dim3(grid_for(o.dims[jn] * 16, 256)), dim3(256), 0, c->stream, fp.p[jn],
                         o.dims[jn], o.K[jn], o.F32[jn].as<float>(), 16);
      TK_CHECK_LAUNCH();
    }
    const int st[3] = {1, o.K[0], o.K[0] * o.K[1]};
    const ModePlan& pl = o.plan[mc];
    hipLaunchKernelGGL(k_eval3_slab, dim3(grid_for(pl.P, 4, 16384)), dim3(256), 0, c->stream,
                       pl.bin_pptr.as<int64_t>(), pl.seg_ptr.as<int32_t>(), pl.seg_pbegin.as<int64_t>(),
                       pl.seg_row.as<int32_t>(), pl.row_slice.as<int32_t>(), pl.lay_idx[0].as<int32_t>(),
                       pl.lay_idx[1].as<int32_t>(), pl.order_pad.as<uint32_t>(), o.F32[ma].as<float>(),
                       o.F32[mb].as<float>(), o.F32[mc].as<float>(), G, o.K[ma], o.K[mb], o.K[mc], st[ma], st[mb],
                       st[mc], pl.P, out);
    TK_CHECK_LAUNCH();
  } else if (o.n_obs > 0) {
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

__global__ void k_fill_zero_f(float* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
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
// The general path (K_n above 16); FP64 accumulation.
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

// W = G_(n)^T as a Khat x K_n FP64 matrix (the right operand of dF_n = Y^g_(n) G_(n)^T).
__global__ void k_core_unfold_t(const float* __restrict__ G, int N, const int32_t* __restrict__ Kd, int n, int khat,
                                double* __restrict__ W) {
  int32_t K[8];
  for (int j = 0; j < N; ++j) K[j] = Kd[j];
  const int Kn = K[n];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)khat * Kn;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = i / Kn;
    const int k = (int)(i - col * Kn);
    W[i] = (double)G[core_lin(N, K, n, k, col)];
  }
}

// dF rows from U = Y^g W (R x K, FP64): dF[row_slice[r]] = U[r], FP32.
__global__ void k_scatter_rows(const double* __restrict__ U, int64_t R, int K, const int32_t* __restrict__ row_slice,
                               float* __restrict__ dF) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R * K; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / K;
    const int k = (int)(i - r * K);
    dF[(int64_t)row_slice[r] * K + k] = (float)U[i];
  }
}

// dcore[c0 + K0 * col] = sum_r F0[slice(r)][c0] * Yg[r][col] (the general path, K_0 above 16).
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

typedef float floatx4_c __attribute__((ext_vector_type(4)));

// dG as A^T Y on the matrix cores (K_0 <= 16): A[r] = F0[row_slice[r]] (16
// floats, zero past K_0), Y = Y^g_(1) (R x khat).  Workgroup w takes rows
// [w*rpw, (w+1)*rpw) and column tiles blockIdx.y*4 + wave (16 columns each):
// v_mfma_f32_16x16x4_f32 with lane l supplying A[r0 + 4s + l/16][l%16] as the
// left operand (i over K_0) and Y[r0 + 4s + l/16][16 t + l%16] as the right
// one (j over columns), so D[4(l/16)+q][l%16] = sum_r A[r][4(l/16)+q] Y[r][16t + l%16].
// Each workgroup writes its FP32 partial tile; k_dcore_sum adds the partials
// in workgroup order in FP64.
__global__ __launch_bounds__(256) void k_dcore_mfma(const float* __restrict__ Yg, int64_t R, int khat,
                                                    const float* __restrict__ F0, int kp0,
                                                    const int32_t* __restrict__ row_slice, int64_t rpw,
                                                    float* __restrict__ part) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int t = blockIdx.y * 4 + wave;           // column tile
  const int i16 = lane & 15, q = lane >> 4;
  const int col = 16 * t + i16;
  const int64_t r0 = (int64_t)blockIdx.x * rpw, r1 = min(r0 + rpw, R);
  floatx4_c acc = {0.f, 0.f, 0.f, 0.f};
  if (16 * t < khat) {
    // the loop is uniform over the wave; rows past r1 contribute zero
    for (int64_t r4 = r0; r4 < r1; r4 += 4) {
      const int64_t r = r4 + q;
      const bool ok = r < r1;
      const float a = ok ? F0[(int64_t)row_slice[r] * kp0 + i16] : 0.f;
      const float b = ok && col < khat ? Yg[r * khat + col] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  // partial tile of this workgroup: part[(wg * ntiles + t) * 256 + (row i)*16 + col j]
  const int ntiles = (khat + 15) >> 4;
  if (t < ntiles) {
    float* dst = part + ((int64_t)blockIdx.x * ntiles + t) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(4 * q + r) * 16 + i16] = acc[r];
  }
}

// dcore[c0 + K0 * col] = sum over workgroups (in order) of the partial tiles, FP64.
__global__ void k_dcore_sum(const float* __restrict__ part, int nwg, int khat, int K0, float* __restrict__ dcore) {
  const int ntiles = (khat + 15) >> 4;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)K0 * khat;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c0 = (int)(i % K0);
    const int col = (int)(i / K0);
    const int t = col >> 4, j = col & 15;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += (double)part[((int64_t)w * ntiles + t) * 256 + c0 * 16 + j];
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
    float* Yg = o.Yg.as<float>();
    if (ttm_takes_mfma3(c, pl, N, n, o.K, o.kp)) {
      // the kernel fetches each residual from observation order as it stages a bin
      ttm_run(c, pl, N, n, o.K, Fp, o.kp, gd, o.n_obs, Yg, false, nullptr, pl.order_pad.as<uint32_t>());
    } else {
      ensure(c, o.gl, sizeof(float) * (size_t)std::max<int64_t>(pl.m_pad, 1));
      hipLaunchKernelGGL(k_gather_layout, dim3(grid_for(pl.m_pad, 256)), dim3(256), 0, c->stream, gd,
                         pl.order_pad.as<uint32_t>(), pl.m_pad, o.gl.as<float>());
      TK_CHECK_LAUNCH();
      ttm_run(c, pl, N, n, o.K, Fp, o.kp, o.gl.as<float>(), o.n_obs, Yg);
    }
    Buf tdF;
    float* dFn = dF[n];
    if (mem == TK_MEM_HOST) {
      tdF.alloc(c, sizeof(float) * (size_t)o.dims[n] * o.K[n]);
      dFn = tdF.as<float>();
    }
    {
      const int64_t nd = o.dims[n] * (int64_t)o.K[n];
      hipLaunchKernelGGL(k_fill_zero_f, dim3(grid_for(nd, 256, 4096)), dim3(256), 0, c->stream, dFn, nd);
      TK_CHECK_LAUNCH();
    }
    if (pl.L_nz > 0 && o.K[n] <= 16) {
      // dF_n = Y^g_(n) G_(n)^T on the matrix cores, then scattered to the slices' rows
      const int Kn = o.K[n];
      ensure(c, c->small64, sizeof(double) * ((size_t)khat * Kn + (size_t)uw_product_parts(pl.L_nz) * Kn * Kn));
      ensure(c, c->U64, sizeof(double) * (size_t)pl.L_nz * Kn);
      double* W = c->small64.as<double>();
      hipLaunchKernelGGL(k_core_unfold_t, dim3(grid_for((int64_t)khat * Kn, 256, 256)), dim3(256), 0, c->stream, G, N,
                         tK.as<int32_t>(), n, khat, W);
      TK_CHECK_LAUNCH();
      uw_product(c, Yg, pl.L_nz, khat, W, Kn, c->U64.as<double>(), W + (size_t)khat * Kn);
      hipLaunchKernelGGL(k_scatter_rows, dim3(grid_for(pl.L_nz * Kn, 256)), dim3(256), 0, c->stream,
                         c->U64.as<double>(), pl.L_nz, Kn, pl.row_slice.as<int32_t>(), dFn);
      TK_CHECK_LAUNCH();
    } else if (pl.L_nz > 0) {
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
      if (pl.L_nz > 0 && o.K[0] <= 16 && o.kp[0] == 16) {
        // A^T Y on the matrix cores, partials summed in workgroup order in FP64
        const int ntiles = (khat + 15) >> 4;
        const int64_t rpw = std::max<int64_t>(256, ceil_div(ceil_div(pl.L_nz, 512), 4) * 4);
        const int nwg = (int)ceil_div(pl.L_nz, rpw);
        Buf part(c, sizeof(float) * (size_t)nwg * ntiles * 256);
        hipLaunchKernelGGL(k_dcore_mfma, dim3(nwg, (unsigned)ceil_div(ntiles, 4)), dim3(256), 0, c->stream, Yg,
                           pl.L_nz, khat, o.F32[0].as<float>(), o.kp[0], pl.row_slice.as<int32_t>(), rpw,
                           part.as<float>());
        TK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_dcore_sum, dim3(grid_for(pK, 256)), dim3(256), 0, c->stream, part.as<float>(), nwg,
                           khat, o.K[0], dc);
        TK_CHECK_LAUNCH();
        c->sync();
      } else if (pl.L_nz > 0) {
        hipLaunchKernelGGL(k_dcore, dim3(grid_for(pK, 256)), dim3(256), 0, c->stream, Yg, pl.L_nz, khat,
                           o.F32[0].as<float>(), o.K[0], o.kp[0], pl.row_slice.as<int32_t>(), dc);
        TK_CHECK_LAUNCH();
      } else {
        hipLaunchKernelGGL(k_fill_zero_f, dim3(grid_for(pK, 256)), dim3(256), 0, c->stream, dc, pK);
        TK_CHECK_LAUNCH();
      }
      if (mem == TK_MEM_HOST) d2h(c, dcore, dc, (size_t)pK);
      c->sync();
    }
    c->sync();
  }
}

}  // namespace tk
