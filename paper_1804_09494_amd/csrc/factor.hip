// New factor from the leading eigenpairs of G = Y^T Y (Section 2.2: the new
// F_n holds the leading K_n left singular vectors of Y_(n)):
//   U  = Y W,  W = V_K diag(lam_k)^(-1/2)     (R_n x K_n; FP32 MFMA for K <= 16,
//                                              else FP64 accumulation)
//   CholeskyQR2 in FP64: A = U^T U, A = R^T R (Cholesky), U <- U R^-1, twice,
//   which restores orthonormality to working precision;
//   F_n = U on the nonempty slices' rows, zero elsewhere (FP64 master),
//   plus the padded FP32 working copy the TTM-chain gathers.
// Columns whose singular value is zero (rank deficiency) are completed on the
// host with unit vectors e_i (lowest i not yet spanned, Gram-Schmidt in FP64).
#include <cmath>

#include "common.hpp"

namespace tk {

void tall_times_small(Ctx* c, const float* Y, int64_t R, int khat, const double* W, int K, double* U);

constexpr int FT_ROWS = 64;  // rows of Y per workgroup

// U = Y W and per-workgroup partial of U^T U.  W (khat x K, FP64) is in LDS;
// Y rows are staged through LDS with a padded stride, FT_ROWS at a time, over
// `tiles` consecutive tiles per workgroup.
__global__ __launch_bounds__(256) void k_uw(const float* __restrict__ Y, int64_t R, int khat,
                                            const double* __restrict__ W, int K, int tiles, double* __restrict__ U,
                                            double* __restrict__ part) {
  extern __shared__ double shd[];
  double* w = shd;                                      // khat * K
  double* ut = w + (size_t)khat * K;                    // FT_ROWS * K
  float* yt = reinterpret_cast<float*>(ut + FT_ROWS * K);  // FT_ROWS * (khat + 1)
  const int ys = khat + 1;
  for (int i = threadIdx.x; i < khat * K; i += blockDim.x) w[i] = W[i];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // entries tid, tid+256, ... of U^T U (K <= 32)
  for (int tt = 0; tt < tiles; ++tt) {
    const int64_t r0 = ((int64_t)blockIdx.x * tiles + tt) * FT_ROWS;
    if (r0 >= R) break;
    const int nr = (int)min<int64_t>(FT_ROWS, R - r0);
    __syncthreads();
    for (int i = threadIdx.x; i < nr * khat; i += blockDim.x) {
      const int r = i / khat, cc = i - r * khat;
      yt[r * ys + cc] = Y[(r0 + r) * khat + cc];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr * K; i += blockDim.x) {
      const int r = i / K, k = i - r * K;
      double s = 0.0;
      for (int cc = 0; cc < khat; ++cc) s += (double)yt[r * ys + cc] * w[cc * K + k];
      ut[r * K + k] = s;
      U[(r0 + r) * K + k] = s;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i < K * K) {
        const int a = i / K, b = i - a * K;
        double s = acc[q];
        for (int r = 0; r < nr; ++r) s += ut[r * K + a] * ut[r * K + b];
        acc[q] = s;
      }
    }
  }
  for (int q = 0; q < 4; ++q) {
    const int i = threadIdx.x + 256 * q;
    if (i < K * K) part[(int64_t)blockIdx.x * K * K + i] = acc[q];
  }
}

typedef float floatx4_f __attribute__((ext_vector_type(4)));
typedef double doublex4_f __attribute__((ext_vector_type(4)));

// Combine the four waves' 16x16 Gram tiles in wave order and write the K x K
// block of this workgroup.  Register r of lane l holds G[row][l%16] with
// row = 4*(l/16) + r for the FP32 MFMA and row = l/16 + 4*r for the FP64 one.
template <bool F64LAYOUT, class T4>
__device__ __forceinline__ void write_gram_part(const T4& g, int K, double* red, double* __restrict__ part) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int w = 0; w < 4; ++w) {
    if (wave == w)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* dst = red + r * 64 + lane;
        *dst = (w == 0) ? (double)g[r] : *dst + (double)g[r];
      }
    __syncthreads();
  }
  if (threadIdx.x < 256) {
    const int r = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int a = F64LAYOUT ? (l >> 4) + 4 * r : 4 * (l >> 4) + r, b = l & 15;
    if (a < K && b < K) part[(int64_t)blockIdx.x * K * K + a * K + b] = red[threadIdx.x];
  }
}

// U = Y W on the matrix cores (K <= 16): v_mfma_f32_16x16x4_f32 over 16-row
// tiles, one tile per wave at a time.  Lane l reads four consecutive columns
// (s + 4*(l/16) .. +3) of row l%16 of the tile; MFMA u contracts column
// s + 4k + u of Y (k = l/16) with row s + 4k + u of W.  The result tile gives
// U (stored FP64) and, with the same registers as both operands, the
// workgroup's partial U^T U.  VEC: khat % 4 == 0 (16-byte loads).
template <bool VEC>
__global__ __launch_bounds__(256) void k_uw_mfma(const float* __restrict__ Y, int64_t R, int khat,
                                                 const double* __restrict__ W, int K, double* __restrict__ U,
                                                 double* __restrict__ part) {
  __shared__ double red[256];
  extern __shared__ float wl[];   // kpad x 16, FP32, zero beyond khat and K
  const int kpad = (khat + 15) & ~15;
  for (int i = threadIdx.x; i < kpad * 16; i += blockDim.x) {
    const int c = i >> 4, j = i & 15;
    wl[i] = (c < khat && j < K) ? (float)W[(int64_t)c * K + j] : 0.f;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  floatx4_f g = {0.f, 0.f, 0.f, 0.f};
  const int64_t ntile = (R + 15) >> 4;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntile; t += (int64_t)gridDim.x * 4) {
    const int64_t row = t * 16 + i16;
    const bool rok = row < R;
    const float* yr = Y + row * khat;
    floatx4_f c = {0.f, 0.f, 0.f, 0.f};
    // four 16-column steps per iteration, their loads issued before the first
    // MFMA (the MFMAs keep their order: same U as one step at a time)
    for (int s = 0; s < kpad; s += 64) {
      float y[4][4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int col = s + 16 * d + 4 * q;
        if (VEC) {
          const float4 v = (rok && col < khat) ? *reinterpret_cast<const float4*>(yr + col) : float4{0.f, 0.f, 0.f, 0.f};
          y[d][0] = v.x; y[d][1] = v.y; y[d][2] = v.z; y[d][3] = v.w;
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) y[d][u] = (rok && col + u < khat) ? yr[col + u] : 0.f;
        }
      }
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        if (s + 16 * d >= kpad) break;   // the same in every lane
        const int col = s + 16 * d + 4 * q;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(y[d][u], wl[(col + u) * 16 + i16], c, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = t * 16 + 4 * q + r;
      if (rr < R && i16 < K) U[rr * K + i16] = (double)c[r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) g = __builtin_amdgcn_mfma_f32_16x16x4f32(c[r], c[r], g, 0, 0, 0);
  }
  write_gram_part<false>(g, K, red, part);
}

// U <- U Rinv on the FP64 matrix cores (K <= 16), 16-row tiles: lane l supplies
// A[i = l%16][k = l/16] = U[row i][4s + k] and B[k][j = l%16] = Rinv[4s + k][j]
// for s = 0..3; v_mfma_f64_16x16x4_f64 returns D[l/16 + 4r][l%16] in register r.  Not FINAL: write U back and the partial U^T U of the result.
// FINAL: write the rows straight into the factor's FP64 master (slice order)
// and its FP32 working copy (storage labels).
template <bool FINAL>
__global__ __launch_bounds__(256) void k_rinv_mfma(double* __restrict__ U, int64_t R, int K,
                                                   const double* __restrict__ Rinv, double* __restrict__ part,
                                                   const int32_t* __restrict__ row_slice,
                                                   const int32_t* __restrict__ label, double* __restrict__ F64,
                                                   float* __restrict__ F32, int kp32, const int* __restrict__ abort) {
  // FINAL: an earlier mode of this invocation failed; keep this factor as it was
  if (FINAL && abort && *abort) return;
  __shared__ double red[256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  double rb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + q;
    rb[s] = (k < K && i16 < K) ? Rinv[k * K + i16] : 0.0;
  }
  doublex4_f g = {0.0, 0.0, 0.0, 0.0};
  const int64_t ntile = (R + 15) >> 4;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntile; t += (int64_t)gridDim.x * 4) {
    const int64_t row = t * 16 + i16;
    const bool rok = row < R;
    doublex4_f c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      const double a = (rok && k < K) ? U[row * K + k] : 0.0;
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rb[s], c, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = t * 16 + q + 4 * r;
      if (rr < R && i16 < K) {
        if (FINAL) {
          const int64_t l = row_slice[rr];
          const int64_t sl = label[l];
          F64[l * K + i16] = c[r];
          F32[sl * kp32 + i16] = (float)c[r];
        } else {
          U[rr * K + i16] = c[r];
        }
      }
    }
    if (!FINAL) {
      // every lane has read its U values above before any lane overwrote them:
      // a tile's rows are read and written by the same wave only
#pragma unroll
      for (int r = 0; r < 4; ++r) g = __builtin_amdgcn_mfma_f64_16x16x4f64(c[r], c[r], g, 0, 0, 0);
    }
  }
  if (!FINAL) write_gram_part<true>(g, K, red, part);
}

// U <- U Rinv (upper triangular, K x K) and partial U^T U of the result, over
// `tiles` consecutive 64-row tiles per workgroup.
__global__ __launch_bounds__(256) void k_apply_rinv(double* __restrict__ U, int64_t R, int K, int tiles,
                                                    const double* __restrict__ Rinv, double* __restrict__ part) {
  extern __shared__ double shd[];
  double* ri = shd;               // K * K
  double* ut = ri + K * K;        // FT_ROWS * K (old rows)
  double* un = ut + FT_ROWS * K;  // FT_ROWS * K (new rows)
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) ri[i] = Rinv[i];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int tt = 0; tt < tiles; ++tt) {
    const int64_t r0 = ((int64_t)blockIdx.x * tiles + tt) * FT_ROWS;
    if (r0 >= R) break;
    const int nr = (int)min<int64_t>(FT_ROWS, R - r0);
    __syncthreads();
    for (int i = threadIdx.x; i < nr * K; i += blockDim.x) ut[i] = U[r0 * K + i];
    __syncthreads();
    // new[r][k] = sum_{j <= k} old[r][j] * Rinv[j][k]
    for (int i = threadIdx.x; i < nr * K; i += blockDim.x) {
      const int r = i / K, k = i - r * K;
      double s = 0.0;
      for (int j = 0; j <= k; ++j) s += ut[r * K + j] * ri[j * K + k];
      un[i] = s;
      U[r0 * K + i] = s;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i < K * K) {
        const int a = i / K, b = i - a * K;
        double s = acc[q];
        for (int r = 0; r < nr; ++r) s += un[r * K + a] * un[r * K + b];
        acc[q] = s;
      }
    }
  }
  for (int q = 0; q < 4; ++q) {
    const int i = threadIdx.x + 256 * q;
    if (i < K * K) part[(int64_t)blockIdx.x * K * K + i] = acc[q];
  }
}

// Fixed-order sum of nparts rows of K*K doubles: one block per entry group.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nparts, int KK,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  for (int e = blockIdx.x; e < KK; e += gridDim.x) {
    double s = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += part[(int64_t)p * KK + e];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = sh[0];
    __syncthreads();
  }
}

// Row j of A beyond the diagonal is exactly zero.  A column of U zeroed below
// the rank floor (W = 0, so U's column is exactly 0.0) has an exactly zero row
// and column in A = U^T U, and every earlier step leaves them so: the Cholesky
// steps below take R[j][j] = 1 for it, so that U R^-1 keeps it zero and the
// other columns come out orthonormal; it is not a failure (the completion adds
// that direction).
__device__ __forceinline__ bool zero_row(const double* A, int K, int j) {
  for (int i = j + 1; i < K; ++i)
    if (A[j * K + i] != 0.0) return false;
  return true;
}

// Cholesky A = R^T R of the summed K x K matrix, Rinv = R^-1.
// flag bit 0 set when a pivot is not positive relative to the largest diagonal.
__global__ void k_chol_inv(const double* __restrict__ Asum, int K, double* __restrict__ Rinv, int* __restrict__ flag) {
  extern __shared__ double shd[];
  double* A = shd;          // K * K
  double* Rm = A + K * K;   // K * K
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) A[i] = Asum[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    double dmax = 0.0;
    for (int i = 0; i < K; ++i) dmax = fmax(dmax, A[i * K + i]);
    bool ok = dmax > 0.0;
    for (int i = 0; i < K * K; ++i) Rm[i] = 0.0;
    for (int j = 0; j < K && ok; ++j) {
      double d = A[j * K + j];
      for (int k = 0; k < j; ++k) d -= Rm[k * K + j] * Rm[k * K + j];
      if (A[j * K + j] == 0.0 && d == 0.0 && zero_row(A, K, j)) {   // a zeroed column stays zero (R[j][j] = 1)
        Rm[j * K + j] = 1.0;
        continue;
      }
      if (!(d > 1e-16 * dmax)) { ok = false; break; }
      const double rjj = sqrt(d);
      Rm[j * K + j] = rjj;
      for (int i = j + 1; i < K; ++i) {
        double s = A[j * K + i];
        for (int k = 0; k < j; ++k) s -= Rm[k * K + j] * Rm[k * K + i];
        Rm[j * K + i] = s / rjj;
      }
    }
    if (!ok) {
      flag[0] |= 1;
      for (int i = 0; i < K * K; ++i) Rinv[i] = (i / K == i % K) ? 1.0 : 0.0;
    } else {
      // inverse of upper triangular R, column by column
      for (int i = 0; i < K * K; ++i) Rinv[i] = 0.0;
      for (int j = 0; j < K; ++j) {
        Rinv[j * K + j] = 1.0 / Rm[j * K + j];
        for (int i = j - 1; i >= 0; --i) {
          double s = 0.0;
          for (int k = i + 1; k <= j; ++k) s += Rm[i * K + k] * Rinv[k * K + j];
          Rinv[i * K + j] = -s / Rm[i * K + i];
        }
      }
    }
  }
}

// The same for K <= 16 with one wavefront: right-looking Cholesky (lanes over
// the trailing block), then column c of R^-1 by back substitution in lane c.
__global__ __launch_bounds__(64) void k_chol_inv_wave(const double* __restrict__ Asum, int K,
                                                      double* __restrict__ Rinv, int* __restrict__ flag) {
  __shared__ double A[16 * 16];
  __shared__ double rdiag[16];
  __shared__ int okf;
  const int l = threadIdx.x;
  for (int i = l; i < K * K; i += 64) A[i] = Asum[i];
  if (l == 0) okf = 1;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < K; ++i) dmax = fmax(dmax, A[i * K + i]);
  if (!(dmax > 0.0) && l == 0) okf = 0;
  __syncthreads();
  // A = R^T R, R stored in the upper triangle of A (row j: R[j][j..K-1])
  for (int j = 0; j < K && okf; ++j) {
    const double d = A[j * K + j];
    const bool zr = Asum[j * K + j] == 0.0 && d == 0.0 && zero_row(A, K, j);   // the same in every lane
    __syncthreads();
    if (zr) {   // a zeroed column stays zero (R[j][j] = 1); its row of R is zero
      if (l == 0) { A[j * K + j] = 1.0; rdiag[j] = 1.0; }
      __syncthreads();
      continue;
    }
    if (!(d > 1e-16 * dmax)) {
      if (l == 0) okf = 0;
      __syncthreads();
      break;
    }
    const double r = sqrt(d);
    const double ri = 1.0 / r;
    // row j of R: R[j][i] = A[j][i] / r for i > j
    if (l > j && l < K) A[j * K + l] *= ri;
    if (l == 0) { A[j * K + j] = r; rdiag[j] = ri; }
    __syncthreads();
    // trailing update A[i][k] -= R[j][i] R[j][k], i, k > j (upper triangle)
    for (int q = l; q < K * K; q += 64) {
      const int i = q / K, k = q - i * K;
      if (i > j && k >= i) A[i * K + k] -= A[j * K + i] * A[j * K + k];
    }
    __syncthreads();
  }
  if (!okf) {
    if (l == 0) flag[0] |= 1;
    for (int i = l; i < K * K; i += 64) Rinv[i] = (i / K == i % K) ? 1.0 : 0.0;
    return;
  }
  // column c of R^-1 (upper triangular): X[c][c] = 1/R[c][c], X[i][c] = -(sum_{k=i+1..c} R[i][k] X[k][c]) / R[i][i]
  __shared__ double X[16 * 16];   // X[c][i] = R^-1[i][c] (LDS: a runtime-indexed register array would spill)
  if (l < K) {
    const int c = l;
    double* x = X + c * 16;
    for (int i = 0; i < K; ++i) x[i] = 0.0;
    x[c] = rdiag[c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= c; ++k) s += A[i * K + k] * x[k];
      x[i] = -s * rdiag[i];
    }
    for (int i = 0; i < K; ++i) Rinv[i * K + c] = x[i];
  }
}

// W = V_K diag(lam)^(-1/2); a column with a non-positive or negligible
// eigenvalue (relative to the largest) is zeroed and flagged (bit 1).
// W = V_K diag(lam)^(-1/2).  A column whose eigenvalue is at or below the
// Gram's rounding floor is not a direction of Y: an exactly zero singular
// value of Y shows up in the FP32 Gram as an eigenvalue of the size of the
// Gram's rounding error, below u ||Y||_F^2 (u = 2^-24), so eigenvalues up to
// RANK_FLOOR * trace(G) are taken as zero.  Such a column sets flag bit 2
// (rank deficiency) and gets W = 0.  Above the floor a small eigenvalue is
// kept: its vector is only as accurate as the Gram allows, but it lies in the
// range of Y.
constexpr double RANK_FLOOR = 4.0 / 16777216.0;   // 4 u

// diag[i * dstride], i < khat: the Gram's diagonal (dstride = khat + 1 in the
// Gram itself, 1 for a separate vector).
__global__ __launch_bounds__(256) void k_make_w(const double* __restrict__ VK, const double* __restrict__ lam,
                                                const double* __restrict__ diag, int64_t dstride, int khat, int K,
                                                double* __restrict__ W, int* __restrict__ flag,
                                                int* __restrict__ kvalid) {
  __shared__ double red[256];
  double t = 0.0;
  for (int i = threadIdx.x; i < khat; i += 256) t += diag[(int64_t)i * dstride];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double floor_ = RANK_FLOOR * red[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {   // eigenvalues come in descending order
    int kv = 0;
    while (kv < K && kv < khat && lam[kv] > floor_ && lam[kv] > 0.0) ++kv;
    *kvalid = kv;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < khat * K; i += gridDim.x * blockDim.x) {
    const int k = i % K;
    const bool ok = k < khat && lam[k] > floor_ && lam[k] > 0.0;  // only khat eigenpairs exist
    W[i] = ok ? VK[i] / sqrt(lam[k]) : 0.0;
    if (!ok && i < K) atomicOr(flag, 2);
  }
}

// F64[row_slice[r]] = U[r] (index order); the FP32 working copy of the same
// rows at their storage labels.
__global__ void k_scatter_factor(const double* __restrict__ U, int64_t R, int K, const int32_t* __restrict__ row_slice,
                                 const int32_t* __restrict__ label, double* __restrict__ F64, float* __restrict__ F32,
                                 int kp32, const int* __restrict__ abort) {
  if (abort && *abort) return;   // an earlier mode of this invocation failed
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R * K; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / K;
    const int k = (int)(i - r * K);
    const int64_t l = row_slice[r];
    const int64_t s = label[l];
    const double v = U[i];
    F64[l * K + k] = v;
    F32[s * kp32 + k] = (float)v;
  }
}

// The FP32 working copy of a whole FP64 factor at the storage labels (padding stays zero).
__global__ void k_factor_copies(const double* __restrict__ F64, int64_t L, int K, const int32_t* __restrict__ label,
                                float* __restrict__ F32, int kp32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L * K; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / K;
    const int k = (int)(i - l * K);
    const int64_t s = label[l];
    F32[s * kp32 + k] = (float)F64[i];
  }
}

void refresh_factor_copies(Ctx* c, int n) {
  const int64_t L = c->dims[n];
  const int K = c->K[n];
  TK_HIP(hipMemsetAsync(c->F32[n].get(), 0, c->F32[n].bytes(), c->stream));
  hipLaunchKernelGGL(k_factor_copies, dim3(grid_for(L * K, 256)), dim3(256), 0, c->stream, c->F64[n].as<double>(), L,
                     K, c->plan[n].label.as<int32_t>(), c->F32[n].as<float>(), c->kp32[n]);
  TK_CHECK_LAUNCH();
}

// ---- completion of a rank-deficient factor ----------------------------------------------------
//
// The factor's computed columns are orthonormalised, the ones that vanish are
// dropped, and the missing columns are unit vectors: at the lowest-index empty
// slices when the mode has enough of them (the computed columns are zero on
// those rows), else e_i (lowest i first) made orthogonal to everything before
// them.  The columns are not unique; only their span with the computed ones
// and their orthonormality are fixed.
//
// On the device: two passes of (Gram F^T F, FP64 over the L rows; Gram-Schmidt
// of the columns in coefficient space on the host, K x K; F <- F T in place).
// The unit-vector columns then need only the rows i of F that are tried: a new
// column is Q b + sum_r a_r e_{i_r}, with Q the orthonormal computed columns,
// so its coefficients follow from those rows, F <- F B adds the Q parts, and
// the few tried rows are written from the host.

constexpr int CG_ROWS = 64;   // rows per LDS tile

// part[b] = sum over block b's rows of F[i, :]^T F[i, :]  (K x K, row-major)
__global__ __launch_bounds__(256) void k_gram64_parts(const double* __restrict__ F, int64_t L, int K,
                                                      int64_t rows_per_block, double* __restrict__ part) {
  __shared__ double tile[CG_ROWS * 32];
  const int KK = K * K;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = std::min<int64_t>(L, r0 + rows_per_block);
  for (int64_t t0 = r0; t0 < r1; t0 += CG_ROWS) {
    const int nr = (int)std::min<int64_t>(CG_ROWS, r1 - t0);
    for (int i = threadIdx.x; i < nr * K; i += 256) tile[i] = F[t0 * K + i];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < KK) {
        const int a = e / K, b = e - a * K;
        double s = 0.0;
        for (int r = 0; r < nr; ++r) s += tile[r * K + a] * tile[r * K + b];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e < KK) part[(int64_t)blockIdx.x * KK + e] = acc[q];
  }
}

// F[i, :] <- F[i, :] T  (T: K x K row-major), in place
__global__ __launch_bounds__(256) void k_rows_times(double* __restrict__ F, int64_t L, int K,
                                                    const double* __restrict__ T) {
  __shared__ double Ts[32 * 32];
  __shared__ double in[CG_ROWS * 32];
  __shared__ double out[CG_ROWS * 32];
  for (int i = threadIdx.x; i < K * K; i += 256) Ts[i] = T[i];
  for (int64_t t0 = (int64_t)blockIdx.x * CG_ROWS; t0 < L; t0 += (int64_t)gridDim.x * CG_ROWS) {
    const int nr = (int)std::min<int64_t>(CG_ROWS, L - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < nr * K; i += 256) in[i] = F[t0 * K + i];
    __syncthreads();
    for (int o = threadIdx.x; o < nr * K; o += 256) {
      const int r = o / K, b = o - r * K;
      double s = 0.0;
      for (int a = 0; a < K; ++a) s += in[r * K + a] * Ts[a * K + b];
      out[o] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr * K; i += 256) F[t0 * K + i] = out[i];
  }
}

namespace {

// Gram of F64[n] (K x K, FP64) on the host.
std::vector<double> factor_gram(Ctx* c, int n, double* dev) {
  const int64_t L = c->dims[n];
  const int K = c->K[n];
  const int KK = K * K;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(L, 4096)));
  const int64_t rpb = ceil_div(L, nb);
  double* part = dev + 2 * KK;
  hipLaunchKernelGGL(k_gram64_parts, dim3(nb), dim3(256), 0, c->stream, c->F64[n].as<double>(), L, K, rpb, part);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_parts, dim3(std::min(KK, 1024)), dim3(256), 0, c->stream, part, nb, KK, dev);
  TK_CHECK_LAUNCH();
  std::vector<double> A((size_t)KK);
  d2h(c, A.data(), dev, A.size());
  c->sync();
  return A;
}

// Modified Gram-Schmidt, twice per column, of the columns of F in the inner
// product of their Gram A: T's columns 0..g-1 give F T orthonormal columns;
// a column whose remainder is at most 1e-6 of its norm is dropped.
int coeff_gram_schmidt(const std::vector<double>& A, int K, std::vector<double>& T) {
  auto dot = [&](const std::vector<double>& x, const std::vector<double>& y) {
    double s = 0.0;
    for (int a = 0; a < K; ++a) {
      if (x[a] == 0.0) continue;
      double t = 0.0;
      for (int b = 0; b < K; ++b) t += A[(size_t)a * K + b] * y[b];
      s += x[a] * t;
    }
    return s;
  };
  std::vector<std::vector<double>> acc;
  for (int k = 0; k < K; ++k) {
    const double n0 = std::sqrt(std::max(A[(size_t)k * K + k], 0.0));
    if (!(n0 > 0.0)) continue;
    std::vector<double> v((size_t)K, 0.0);
    v[k] = 1.0;
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& u : acc) {
        const double d = dot(u, v);
        for (int a = 0; a < K; ++a) v[a] -= d * u[a];
      }
    const double nv = std::sqrt(std::max(dot(v, v), 0.0));
    if (nv > 1e-6 * n0) {
      for (double& x : v) x /= nv;
      acc.push_back(std::move(v));
    }
  }
  T.assign((size_t)K * K, 0.0);
  for (size_t j = 0; j < acc.size(); ++j)
    for (int a = 0; a < K; ++a) T[(size_t)a * K + j] = acc[j][a];
  return (int)acc.size();
}

void apply_rows_times(Ctx* c, int n, const std::vector<double>& T, double* dev) {
  const int64_t L = c->dims[n];
  const int K = c->K[n];
  h2d(c, dev + K * K, T.data(), T.size());
  hipLaunchKernelGGL(k_rows_times, dim3(grid_for(ceil_div(L, CG_ROWS), 1, 4096)), dim3(256), 0, c->stream,
                     c->F64[n].as<double>(), L, K, dev + K * K);
  TK_CHECK_LAUNCH();
  c->sync();   // T's host copy may go
}

}  // namespace

// ids[t], t < M: the t-th empty slice (ascending) of a mode with nonempty
// slices row_slice[0..R) (ascending).  Before row_slice[r] lie row_slice[r] - r
// empty ids, so the t-th is t + r for the first r with row_slice[r] - r > t
// (r = R when the empty ids past the last nonempty slice are reached).
__global__ void k_find_empty(const int32_t* __restrict__ row_slice, int64_t R, int M, int32_t* __restrict__ ids) {
  const int t = threadIdx.x;
  if (t >= M) return;
  int64_t lo = 0, hi = R;   // first r in [0, R] with row_slice[r] - r > t
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)row_slice[mid] - mid > t) hi = mid; else lo = mid + 1;
  }
  ids[t] = (int32_t)(t + lo);
}

// Column g + t of factor n becomes e_{ids[t]} (its FP64 row and its FP32 copy at
// the row's storage label): the rows were zero, as rows of empty slices are.
__global__ void k_set_units(const int32_t* __restrict__ ids, int M, int g, int K, const int32_t* __restrict__ label,
                            double* __restrict__ F64, float* __restrict__ F32, int kp32) {
  const int t = threadIdx.x;
  if (t >= M) return;
  const int64_t i = ids[t];
  F64[i * K + g + t] = 1.0;
  F32[(int64_t)label[i] * kp32 + g + t] = 1.0f;
}

// Zero the rows ids[0..M) of factor n (FP64 and FP32 copy), unless an earlier
// mode of this invocation failed.
__global__ void k_zero_rows(const int32_t* __restrict__ ids, int M, int K, const int32_t* __restrict__ label,
                            double* __restrict__ F64, float* __restrict__ F32, int kp32, const int* __restrict__ abort) {
  if (abort && *abort) return;
  for (int q = threadIdx.x; q < M * K; q += blockDim.x) {
    const int t = q / K, k = q - t * K;
    const int64_t i = ids[t];
    F64[i * K + k] = 0.0;
    F32[(int64_t)label[i] * kp32 + k] = 0.0f;
  }
}

// Returns true when the missing columns are unit vectors at rows of empty slices.
static bool complete_on_device(Ctx* c, int n, int g_known) {
  const int64_t L = c->dims[n];
  const int K = c->K[n];
  const int KK = K * K;
  TK_REQUIRE(K <= 32, TK_ERR_UNSUPPORTED, "completion: rank above 32");
  ensure(c, c->small64, sizeof(double) * (size_t)KK * (2 + 1024));
  double* dev = c->small64.as<double>();
  // orthonormal computed columns: two passes, unless the factor step already
  // orthonormalised them (its only failure was the rank floor)
  int g = K;
  if (g_known >= 0) {
    g = g_known;
  } else {
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<double> A = factor_gram(c, n, dev);
      std::vector<double> T;
      g = coeff_gram_schmidt(A, K, T);
      apply_rows_times(c, n, T, dev);
    }
  }
  if (g == K) {
    refresh_factor_copies(c, n);
    c->sync();
    return false;
  }
  // a mode with enough empty slices: the computed columns vanish on those rows,
  // so unit vectors there are already orthogonal to them and to each other
  const ModePlan& pl = c->plan[n];
  const int M = K - g;
  if (L - pl.L_nz >= M) {
    ensure(c, c->unit_rows[n], sizeof(int32_t) * 32);
    int32_t* ids = c->unit_rows[n].as<int32_t>();
    hipLaunchKernelGGL(k_find_empty, dim3(1), dim3(32), 0, c->stream, pl.row_slice.as<int32_t>(), pl.L_nz, M, ids);
    TK_CHECK_LAUNCH();
    if (g_known < 0) refresh_factor_copies(c, n);   // the passes above rewrote F64
    hipLaunchKernelGGL(k_set_units, dim3(1), dim3(32), 0, c->stream, ids, M, g, K, pl.label.as<int32_t>(),
                       c->F64[n].as<double>(), c->F32[n].as<float>(), c->kp32[n]);
    TK_CHECK_LAUNCH();
    c->n_unit_rows[n] = M;
    c->sync();
    return true;
  }
  // unit vectors e_i, lowest i first.  A column is (b, a): Q b + sum_r a[r] e_{cand[r]}.
  struct Col {
    std::vector<double> b, a;
  };
  std::vector<int64_t> cand;            // tried rows, in order
  std::vector<std::vector<double>> qrow; // Q[cand[r], 0..g-1]
  std::vector<Col> added;
  auto inner = [&](const Col& x, const Col& y) {
    double s = 0.0;
    for (int j = 0; j < g; ++j) s += x.b[j] * y.b[j];
    for (size_t r = 0; r < cand.size(); ++r) {
      double qx = 0.0, qy = 0.0;
      for (int j = 0; j < g; ++j) {
        qx += qrow[r][j] * x.b[j];
        qy += qrow[r][j] * y.b[j];
      }
      s += y.a[r] * qx + x.a[r] * qy + x.a[r] * y.a[r];
    }
    return s;
  };
  std::vector<double> rows_h;
  int64_t rows_at = 0, rows_n = 0;
  for (int64_t i = 0; g + (int)added.size() < K; ++i) {
    TK_REQUIRE(i < L, TK_ERR_NUMERIC, "completion: unit vectors exhausted");
    if (i >= rows_at + rows_n) {   // read the next rows of Q
      rows_at = i;
      rows_n = std::min<int64_t>(256, L - i);
      rows_h.resize((size_t)rows_n * K);
      d2h(c, rows_h.data(), c->F64[n].as<double>() + i * K, rows_h.size());
      c->sync();
    }
    cand.push_back(i);
    qrow.emplace_back(rows_h.begin() + (i - rows_at) * K, rows_h.begin() + (i - rows_at) * K + g);
    for (auto& col : added) col.a.push_back(0.0);
    Col v{std::vector<double>((size_t)g), std::vector<double>(cand.size(), 0.0)};
    v.a.back() = 1.0;
    for (int pass = 0; pass < 2; ++pass) {
      // against Q's columns: <Q e_j, v> = v.b[j] + sum_r v.a[r] Q[cand[r], j]
      std::vector<double> d((size_t)g, 0.0);
      for (int j = 0; j < g; ++j) {
        double t = v.b[j];
        for (size_t r = 0; r < cand.size(); ++r) t += v.a[r] * qrow[r][j];
        d[j] = t;
      }
      for (int j = 0; j < g; ++j) v.b[j] -= d[j];
      for (const auto& u : added) {
        const double t = inner(u, v);
        for (int j = 0; j < g; ++j) v.b[j] -= t * u.b[j];
        for (size_t r = 0; r < cand.size(); ++r) v.a[r] -= t * u.a[r];
      }
    }
    const double nv = std::sqrt(std::max(inner(v, v), 0.0));
    if (nv > 0.5) {
      for (double& x : v.b) x /= nv;
      for (double& x : v.a) x /= nv;
      added.push_back(std::move(v));
    }
  }
  // F <- F B: column j < g stays, column g + t = Q b_t (columns g.. of F are zero)
  std::vector<double> B((size_t)KK, 0.0);
  for (int j = 0; j < g; ++j) B[(size_t)j * K + j] = 1.0;
  for (size_t t = 0; t < added.size(); ++t)
    for (int j = 0; j < g; ++j) B[(size_t)j * K + g + t] = added[t].b[j];
  apply_rows_times(c, n, B, dev);
  // the tried rows: Q[i] B + the unit-vector parts
  std::vector<double> patch(cand.size() * (size_t)K);
  for (size_t r = 0; r < cand.size(); ++r) {
    double* row = patch.data() + r * K;
    for (int j = 0; j < g; ++j) row[j] = qrow[r][j];
    for (size_t t = 0; t < added.size(); ++t) {
      double s = added[t].a[r];
      for (int j = 0; j < g; ++j) s += qrow[r][j] * added[t].b[j];
      row[g + t] = s;
    }
  }
  // the tried rows are 0 .. cand.size()-1, contiguous
  h2d(c, c->F64[n].as<double>(), patch.data(), patch.size());
  refresh_factor_copies(c, n);
  c->sync();
  return false;
}

void complete_factor(Ctx* c, int n, int g);
int computed_columns(Ctx* c, const int* flag_dev, int n);

// U = Y W (R x K, FP64 out) on the matrix cores for K <= 16, W khat x K in
// FP64 (rounded to FP32 for the MFMA operands); `part` receives nwg x K x K
// partial U^T U blocks (unused by callers that only want U).  Returns nwg.
int uw_product(Ctx* c, const float* Y, int64_t R, int khat, const double* W, int K, double* U, double* part) {
  TK_REQUIRE(K <= 16, TK_ERR_UNSUPPORTED, "Y W on the matrix cores: K above 16");
  const int64_t ntile = std::max<int64_t>(1, ceil_div(R, 16));
  const int nwg = (int)std::min<int64_t>(2048, ceil_div(ntile, 4));
  const int kpad = (khat + 15) & ~15;
  const size_t lds = sizeof(float) * (size_t)kpad * 16;
  TK_REQUIRE(lds + 2048 <= c->lds_per_block, TK_ERR_UNSUPPORTED, "Y W: Khat too large for LDS");
  if (khat % 4 == 0)
    hipLaunchKernelGGL(k_uw_mfma<true>, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, W, K, U, part);
  else
    hipLaunchKernelGGL(k_uw_mfma<false>, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, W, K, U, part);
  TK_CHECK_LAUNCH();
  return nwg;
}

int uw_product_parts(int64_t R) { return (int)std::min<int64_t>(2048, ceil_div(std::max<int64_t>(1, ceil_div(R, 16)), 4)); }

// zero a buffer (2-byte units) unless an earlier mode of this invocation failed
__global__ void k_clear_unless(uint16_t* __restrict__ p, int64_t n16, const int* __restrict__ abort) {
  if (*abort) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// flag[0]: this mode's failure flag; flag[1]: 1 + the first failed mode of the invocation
__global__ void k_flag_record(int* flag, int n) {
  flag[FLAG_BITS + n] = flag[0];
  if (flag[0] && !flag[1]) flag[1] = n + 1;
}

// New factor n from Y (R x khat) and the leading eigenpairs (lam_k, VK).
// Returns true when the completion path ran.
// deferred = false: the failure check reads flag_dev[0] on the host and
// completes the factor at once.
// deferred = true (a Gauss-Seidel invocation that checks once at its end):
// flag_dev[1] = 1 + the first failed mode of the invocation, or 0.  Once it is
// set, this call leaves factor n as it was (the caller runs the mode again
// after completing the failed factor); a failure of this mode sets it when
// R >= K, and is completed at once when R < K.
bool form_factor(Ctx* c, int n, const float* Y, int64_t R, int khat, const double* gdiag, int64_t dstride,
                 const double* lam_k, const double* VK, int* flag_dev, bool deferred) {
  const int* abort = deferred ? flag_dev + 1 : nullptr;
  const bool check_flag = !deferred || R < c->K[n];
  const int K = c->K[n];
  TK_REQUIRE(K <= 32, TK_ERR_UNSUPPORTED, "factor step: rank above 32");
  const bool mfma = K <= 16;
  const int64_t ntile = std::max<int64_t>(1, ceil_div(R, mfma ? 16 : FT_ROWS));
  const int tiles = (int)std::max<int64_t>(1, ceil_div(ntile, 1024));
  const int nwg = mfma ? (int)std::min<int64_t>(2048, ceil_div(ntile, 4)) : (int)ceil_div(ntile, tiles);
  ensure(c, c->U64, sizeof(double) * (size_t)std::max<int64_t>(R, 1) * K);
  ensure(c, c->small64, sizeof(double) * ((size_t)khat * K + 3 * (size_t)K * K + (size_t)nwg * K * K));
  double* W = c->small64.as<double>();
  double* Rinv = W + (size_t)khat * K;
  double* Asum = Rinv + (size_t)K * K;
  double* part = Asum + (size_t)K * K;
  double* U = c->U64.as<double>();
  const ModePlan& pl = c->plan[n];
  TK_HIP(hipMemsetAsync(flag_dev, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_make_w, dim3(grid_for((int64_t)khat * K, 256, 64)), dim3(256), 0, c->stream, VK, lam_k, gdiag,
                     dstride, khat, K, W, flag_dev, flag_dev + FLAG_KVALID + n);
  TK_CHECK_LAUNCH();
  // rows of empty slices (never written below) must be zero: clear the copies
  // only when something else may have written them (tk_set_factor, completion)
  auto clear_factor = [&]() {
    if (!c->fac_dirty[n] && c->n_unit_rows[n] > 0) {
      const int M = c->n_unit_rows[n];
      hipLaunchKernelGGL(k_zero_rows, dim3(1), dim3(256), 0, c->stream, c->unit_rows[n].as<int32_t>(), M, K,
                         pl.label.as<int32_t>(), c->F64[n].as<double>(), c->F32[n].as<float>(), c->kp32[n], abort);
      TK_CHECK_LAUNCH();
      c->n_unit_rows[n] = 0;
      return;
    }
    if (!c->fac_dirty[n]) return;
    c->n_unit_rows[n] = 0;
    if (abort) {
      // deferred check: a later pass may have to keep this factor as it was;
      // the clear then does not happen, and the driver marks the factor dirty
      // again before that pass
      for (Buf* b : {&c->F64[n], &c->F32[n]}) {
        const int64_t n16 = (int64_t)(b->bytes() / 2);
        hipLaunchKernelGGL(k_clear_unless, dim3(grid_for(n16, 256, 4096)), dim3(256), 0, c->stream,
                           b->as<uint16_t>(), n16, abort);
        TK_CHECK_LAUNCH();
      }
    } else {
      TK_HIP(hipMemsetAsync(c->F64[n].get(), 0, c->F64[n].bytes(), c->stream));
      TK_HIP(hipMemsetAsync(c->F32[n].get(), 0, c->F32[n].bytes(), c->stream));
    }
    c->fac_dirty[n] = false;
  };
  auto reduce_chol = [&]() {
    hipLaunchKernelGGL(k_sum_parts, dim3(std::min(K * K, 1024)), dim3(256), 0, c->stream, part, nwg, K * K, Asum);
    TK_CHECK_LAUNCH();
    if (K <= 16)
      hipLaunchKernelGGL(k_chol_inv_wave, dim3(1), dim3(64), 0, c->stream, Asum, K, Rinv, flag_dev);
    else
      hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), sizeof(double) * 2 * K * K, c->stream, Asum, K, Rinv,
                         flag_dev);
    TK_CHECK_LAUNCH();
  };
  if (R > 0 && mfma) {
    const int kpad = (khat + 15) & ~15;
    const size_t lds = sizeof(float) * (size_t)kpad * 16;
    if (lds + 2048 <= c->lds_per_block) {
      if (khat % 4 == 0)
        hipLaunchKernelGGL(k_uw_mfma<true>, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, W, K, U, part);
      else
        hipLaunchKernelGGL(k_uw_mfma<false>, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, W, K, U, part);
      TK_CHECK_LAUNCH();
    } else {
      // W too large for LDS: U = Y W as a tall-skinny FP64 product, then the
      // workgroups' row ranges of U^T U
      tall_times_small(c, Y, R, khat, W, K, U);
      hipLaunchKernelGGL(k_gram64_parts, dim3(nwg), dim3(256), 0, c->stream, U, R, K, ceil_div(R, nwg), part);
      TK_CHECK_LAUNCH();
    }
    reduce_chol();
    hipLaunchKernelGGL(k_rinv_mfma<false>, dim3(nwg), dim3(256), 0, c->stream, U, R, K, Rinv, part, nullptr, nullptr,
                       nullptr, nullptr, 0, nullptr);
    TK_CHECK_LAUNCH();
    reduce_chol();
    clear_factor();
    hipLaunchKernelGGL(k_rinv_mfma<true>, dim3(nwg), dim3(256), 0, c->stream, U, R, K, Rinv, part,
                       pl.row_slice.as<int32_t>(), pl.label.as<int32_t>(), c->F64[n].as<double>(),
                       c->F32[n].as<float>(), c->kp32[n], abort);
    TK_CHECK_LAUNCH();
  } else if (R > 0) {
    size_t lds = sizeof(double) * ((size_t)khat * K + FT_ROWS * K) + sizeof(float) * FT_ROWS * (size_t)(khat + 1);
    if (lds <= c->lds_per_block) {
      hipLaunchKernelGGL(k_uw, dim3(nwg), dim3(256), lds, c->stream, Y, R, khat, W, K, tiles, U, part);
      TK_CHECK_LAUNCH();
    } else {
      // W too large for LDS: U = Y W as a tall-skinny product, then the
      // workgroups' row ranges of U^T U
      tall_times_small(c, Y, R, khat, W, K, U);
      hipLaunchKernelGGL(k_gram64_parts, dim3(nwg), dim3(256), 0, c->stream, U, R, K, ceil_div(R, nwg), part);
      TK_CHECK_LAUNCH();
    }
    for (int pass = 0; pass < 2; ++pass) {
      reduce_chol();
      hipLaunchKernelGGL(k_apply_rinv, dim3(nwg), dim3(256), sizeof(double) * ((size_t)K * K + 2 * FT_ROWS * K),
                         c->stream, U, R, K, tiles, Rinv, part);
      TK_CHECK_LAUNCH();
    }
    clear_factor();
    hipLaunchKernelGGL(k_scatter_factor, dim3(grid_for(R * K, 256)), dim3(256), 0, c->stream, U, R, K,
                       pl.row_slice.as<int32_t>(), pl.label.as<int32_t>(), c->F64[n].as<double>(),
                       c->F32[n].as<float>(), c->kp32[n], abort);
    TK_CHECK_LAUNCH();
  } else {
    clear_factor();
  }
  if (!check_flag) {
    hipLaunchKernelGGL(k_flag_record, dim3(1), dim3(1), 0, c->stream, flag_dev, n);
    TK_CHECK_LAUNCH();
    return false;
  }
  int hflag[2] = {0, 0};
  d2h(c, hflag, flag_dev, deferred ? 2 : 1);
  c->sync();
  if (hflag[1]) return false;   // an earlier mode failed: this mode runs again later
  if (hflag[0] || R < K) {
    if (!c->opt.complete_rank_deficient) fail(TK_ERR_NUMERIC, "rank-deficient penultimate matrix");
    complete_factor(c, n, hflag[0] == 2 && R >= K ? computed_columns(c, flag_dev, n) : -1);
    return true;
  }
  return false;
}

// Columns of factor n above the rank floor, as its factor step recorded them.
int computed_columns(Ctx* c, const int* flag_dev, int n) {
  int kv = 0;
  d2h(c, &kv, flag_dev + FLAG_KVALID + n, 1);
  c->sync();
  return kv;
}

// Complete factor n (rank-deficient penultimate matrix) on the host.
// g >= 0: the factor step failed only on the rank floor, so columns 0..g-1
// are already orthonormal and the rest exactly zero.
void complete_factor(Ctx* c, int n, int g) {
  ++c->counters.rank_completions;
  c->completed_once = true;
  // the unit-vector rows of empty slices are zeroed by the next factor step
  // (only those rows after a completion by k_set_units, all of them otherwise)
  if (!complete_on_device(c, n, g)) c->fac_dirty[n] = true;
}

}  // namespace tk
