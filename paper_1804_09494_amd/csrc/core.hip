// Core tensor and fit.  Section 2.2 computes the new core
// G = T x_1 F_1^T ... x_N F_N^T once, after the invocations.  With the
// mode-N penultimate matrix Y_(N) = (T x_{j<N} F_j^T)_(N) in hand this is one
// more (small) product: G_(N) = F_N^T Y_(N), here summed over the nonempty
// slices' rows in FP64:  G_(N)[k][col] = sum_r F_N[slice(r)][k] * Y[r][col].
// The core is stored first index fastest, so core[col + Khat_N * k] = G_(N)[k][col].
// fit = 1 - sqrt(max(0, ||T||^2 - ||G||^2)) / ||T||  (orthonormal factors).
#include <cmath>

#include "common.hpp"

namespace tk {

constexpr int CORE_TILE = 64;

__global__ __launch_bounds__(256) void k_core_part(const float* __restrict__ Y, int64_t R, int khat,
                                                   const double* __restrict__ F, int K,
                                                   const int32_t* __restrict__ row_slice, int rows_per_wg,
                                                   int tile, double* __restrict__ part) {
  extern __shared__ double shc[];
  double* ft = shc;                                      // tile x K
  float* yt = reinterpret_cast<float*>(ft + tile * K);   // tile x khat
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min<int64_t>(r0 + rows_per_wg, R);
  const int nent = K * khat;
  // each thread owns entries i = tid, tid + 256, ... (at most 8 here; larger sets loop)
  for (int base = 0; base < nent; base += 256 * 8) {
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int64_t t0 = r0; t0 < r1; t0 += tile) {
      const int nr = (int)min<int64_t>(tile, r1 - t0);
      __syncthreads();
      for (int i = threadIdx.x; i < nr * K; i += blockDim.x) {
        const int r = i / K, k = i - r * K;
        ft[i] = F[(int64_t)row_slice[t0 + r] * K + k];
      }
      for (int i = threadIdx.x; i < nr * khat; i += blockDim.x) yt[i] = Y[t0 * khat + i];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + u * 256 + threadIdx.x;
        if (i < nent) {
          const int k = i / khat, col = i - k * khat;
          double s = acc[u];
          for (int r = 0; r < nr; ++r) s += ft[r * K + k] * (double)yt[r * khat + col];
          acc[u] = s;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = base + u * 256 + threadIdx.x;
      if (i < nent) part[(int64_t)blockIdx.x * nent + i] = acc[u];
    }
  }
}

constexpr int CORE_GROUP = 32;   // workgroup partials summed per first-level thread

// Level 1: sums of CORE_GROUP consecutive workgroup partials (fixed order).
__global__ void k_core_group(const double* __restrict__ part, int nwg, int nent, double* __restrict__ gsum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nent) return;
  const int w0 = blockIdx.y * CORE_GROUP, w1 = min(w0 + CORE_GROUP, nwg);
  double s = 0.0;
  for (int w = w0; w < w1; ++w) s += part[(int64_t)w * nent + i];
  gsum[(int64_t)blockIdx.y * nent + i] = s;
}

// Level 2: sum the groups in order; write the core (first index fastest).
__global__ void k_core_reduce(const double* __restrict__ gsum, int ngroups, int K, int khat,
                              double* __restrict__ core) {
  const int nent = K * khat;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nent; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += gsum[(int64_t)g * nent + i];
    const int k = i / khat, col = i - k * khat;
    core[col + (int64_t)khat * k] = s;
  }
}

// ||G||^2 in fixed order and the fit.
__global__ void k_fit(const double* __restrict__ core, int64_t n, double norm_t_sq, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += core[i] * core[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double g = sh[0];
    out[0] = g;
    out[1] = norm_t_sq > 0 ? 1.0 - sqrt(fmax(0.0, norm_t_sq - g)) / sqrt(norm_t_sq) : 1.0;
  }
}

// core (device, prod K) from Y_(N) (R x khat) and the mode-N factor; out2[0] = ||G||^2, out2[1] = fit.
void core_from_last(Ctx* c, const float* Y, double* core, double* out2) {
  const int n = c->N - 1;
  const ModePlan& pl = c->plan[n];
  const int64_t R = pl.L_nz;
  const int khat = (int)pl.khat;
  const int K = c->K[n];
  int rows_per_wg = (int)std::max<int64_t>(CORE_TILE, ceil_div(ceil_div(std::max<int64_t>(R, 1), 1024), CORE_TILE) * CORE_TILE);
  const int nwg = (int)std::max<int64_t>(1, ceil_div(R, rows_per_wg));
  const int nent = K * khat;
  const int ngroups = (nwg + CORE_GROUP - 1) / CORE_GROUP;
  ensure(c, c->gram_part, sizeof(double) * ((size_t)nwg + ngroups) * nent);
  double* part = c->gram_part.as<double>();
  double* gsum = part + (size_t)nwg * nent;
  if (R > 0) {
    // rows staged per pass: CORE_TILE, fewer when Khat is wide
    const int64_t per_row = sizeof(double) * K + sizeof(float) * (int64_t)khat;
    const int tile = (int)std::min<int64_t>(CORE_TILE, ((int64_t)c->lds_per_block - 1024) / per_row);
    TK_REQUIRE(tile >= 1, TK_ERR_UNSUPPORTED, "core: Khat too large for LDS");
    const size_t lds = (size_t)per_row * tile;
    hipLaunchKernelGGL(k_core_part, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, c->F64[n].as<double>(), K,
                       pl.row_slice.as<int32_t>(), rows_per_wg, tile, part);
    TK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_core_group, dim3((unsigned)ceil_div(nent, 256), ngroups), dim3(256), 0, c->stream, part,
                       nwg, nent, gsum);
    TK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_core_reduce, dim3(grid_for((int64_t)nent, 256, 1024)), dim3(256), 0, c->stream, gsum,
                       ngroups, K, khat, core);
    TK_CHECK_LAUNCH();
  } else {
    TK_HIP(hipMemsetAsync(core, 0, sizeof(double) * (size_t)K * khat, c->stream));
  }
  hipLaunchKernelGGL(k_fit, dim3(1), dim3(256), 0, c->stream, core, (int64_t)K * khat, c->norm_sq, out2);
  TK_CHECK_LAUNCH();
}

}  // namespace tk
