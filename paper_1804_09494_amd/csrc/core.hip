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

constexpr int CORE_ROWS = 64;   // rows per workgroup: many short workgroups hide the load latency

// Workgroup partial of G_(N) over rows [r0, r1) (at most CORE_ROWS): thread t
// owns column blockIdx.y * 256 + t and entries k0 .. k0 + KM - 1 of it
// (k0 = blockIdx.z * KM), accumulated in row order.  The slices' factor rows
// are staged in LDS (read back as broadcasts); Y is read straight from HBM,
// coalesced along the row, sixteen rows' loads issued before their products.
template <int KM>
__global__ __launch_bounds__(256) void k_core_part(const float* __restrict__ Y, int64_t R, int khat,
                                                   const double* __restrict__ F, int K,
                                                   const int32_t* __restrict__ row_slice, int rows_per_wg,
                                                   double* __restrict__ part) {
  __shared__ double ft[CORE_ROWS * KM];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int nr = (int)min<int64_t>(rows_per_wg, R - r0);
  const int col = blockIdx.y * 256 + threadIdx.x;
  const bool ok = col < khat;
  const int cl = ok ? col : 0;
  const int k0 = blockIdx.z * KM, kn = min(KM, K - k0);
  for (int i = threadIdx.x; i < nr * KM; i += 256) {
    const int r = i / KM, k = i - r * KM;
    ft[i] = k < kn ? F[(int64_t)row_slice[r0 + r] * K + k0 + k] : 0.0;
  }
  __syncthreads();
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  const float* yb = Y + r0 * khat + cl;
  int r = 0;
  for (; r + 16 <= nr; r += 16) {
    float y[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) y[u] = yb[(int64_t)(r + u) * khat];
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < KM; ++k) acc[k] += ft[(r + u) * KM + k] * (double)y[u];
  }
  for (; r < nr; ++r) {
    const double y = (double)yb[(int64_t)r * khat];
#pragma unroll
    for (int k = 0; k < KM; ++k) acc[k] += ft[r * KM + k] * y;
  }
  if (ok) {
    const int64_t nent = (int64_t)K * khat;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < kn) part[(int64_t)blockIdx.x * nent + (int64_t)(k0 + k) * khat + col] = acc[k];
  }
}

// The same partial for Khat <= 128 over CORE_ROWS2 rows: thread t owns column
// t % 128 for one half of the rows (t / 128), the halves' sums are added in
// LDS (first half + second half), so a workgroup reads four times the rows of
// k_core_part with every thread busy and writes a quarter of the partials.
constexpr int CORE_ROWS2 = 256;
template <int KM>
__global__ __launch_bounds__(256) void k_core_part2(const float* __restrict__ Y, int64_t R, int khat,
                                                    const double* __restrict__ F, int K,
                                                    const int32_t* __restrict__ row_slice,
                                                    double* __restrict__ part) {
  __shared__ __align__(16) double ft[CORE_ROWS2 * KM];
  __shared__ double hsum[128 * KM];
  static_assert(KM % 2 == 0, "entries are read in pairs");
  const int64_t r0 = (int64_t)blockIdx.x * CORE_ROWS2;
  const int nr = (int)min<int64_t>(CORE_ROWS2, R - r0);
  const int t = threadIdx.x, col = t & 127, h = t >> 7;
  const bool ok = col < khat;
  const int cl = ok ? col : 0;
  const int k0 = blockIdx.z * KM, kn = min(KM, K - k0);
  for (int i = t; i < nr * KM; i += 256) {
    const int r = i / KM, k = i - r * KM;
    ft[i] = k < kn ? F[(int64_t)row_slice[r0 + r] * K + k0 + k] : 0.0;
  }
  __syncthreads();
  const int half = (nr + 1) >> 1;
  const int ra = h ? half : 0, rb = h ? nr : half;
  double acc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) acc[k] = 0.0;
  const float* yb = Y + r0 * khat + cl;
  int r = ra;
  for (; r + 16 <= rb; r += 16) {
    float y[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) y[u] = yb[(int64_t)(r + u) * khat];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double2* fr = reinterpret_cast<const double2*>(ft + (r + u) * KM);   // 16-byte broadcasts
#pragma unroll
      for (int k2 = 0; k2 < KM / 2; ++k2) {
        const double2 f = fr[k2];
        acc[2 * k2] += f.x * (double)y[u];
        acc[2 * k2 + 1] += f.y * (double)y[u];
      }
    }
  }
  for (; r < rb; ++r) {
    const double y = (double)yb[(int64_t)r * khat];
#pragma unroll
    for (int k = 0; k < KM; ++k) acc[k] += ft[r * KM + k] * y;
  }
  if (h) {
#pragma unroll
    for (int k = 0; k < KM; ++k) hsum[k * 128 + col] = acc[k];
  }
  __syncthreads();
  if (!h && ok) {
    const int64_t nent = (int64_t)K * khat;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < kn) part[(int64_t)blockIdx.x * nent + (int64_t)(k0 + k) * khat + col] = acc[k] + hsum[k * 128 + col];
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
  const bool narrow = khat <= 128;
  const int rows_per_wg = narrow ? CORE_ROWS2 : CORE_ROWS;
  const int nwg = (int)std::max<int64_t>(1, ceil_div(R, rows_per_wg));
  const int nent = K * khat;
  const int ngroups = (nwg + CORE_GROUP - 1) / CORE_GROUP;
  ensure(c, c->gram_part, sizeof(double) * ((size_t)nwg + ngroups) * nent);
  double* part = c->gram_part.as<double>();
  double* gsum = part + (size_t)nwg * nent;
  if (R > 0) {
    if (narrow) {
      // entries per pass: K rounded up to 4, at most 16
      const int km = K <= 4 ? 4 : K <= 8 ? 8 : K <= 12 ? 12 : 16;
      const dim3 g((unsigned)nwg, 1, (unsigned)ceil_div(K, km));
      const double* F64 = c->F64[n].as<double>();
      const int32_t* rs = pl.row_slice.as<int32_t>();
      switch (km) {
        case 4: hipLaunchKernelGGL(k_core_part2<4>, g, dim3(256), 0, c->stream, Y, R, khat, F64, K, rs, part); break;
        case 8: hipLaunchKernelGGL(k_core_part2<8>, g, dim3(256), 0, c->stream, Y, R, khat, F64, K, rs, part); break;
        case 12: hipLaunchKernelGGL(k_core_part2<12>, g, dim3(256), 0, c->stream, Y, R, khat, F64, K, rs, part); break;
        default: hipLaunchKernelGGL(k_core_part2<16>, g, dim3(256), 0, c->stream, Y, R, khat, F64, K, rs, part); break;
      }
    } else {
      const dim3 g((unsigned)nwg, (unsigned)ceil_div(khat, 256), (unsigned)ceil_div(K, 16));
      hipLaunchKernelGGL(k_core_part<16>, g, dim3(256), 0, c->stream, Y, R, khat, c->F64[n].as<double>(), K,
                         pl.row_slice.as<int32_t>(), rows_per_wg, part);
    }
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
