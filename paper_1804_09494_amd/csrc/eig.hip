// FP64 symmetric eigensolver for the Gram matrix G = Y^T Y (Khat x Khat):
// the leading K_n eigenpairs give the leading K_n left singular vectors of Y
// (Section 2.2: the SVD step of an HOOI invocation) as Y V_K S_K^-1.
//
// One workgroup of 512 threads, the matrix resident in LDS when it fits:
//   1. Householder tridiagonalisation G = Q T Q^T.  Reflector k is
//      I - tau_k v v^T on rows/columns k+1..n-1 with v_0 = 1; it is built from
//      row k (G stays symmetric), and row k is never touched again, so the
//      reflector is kept as that row plus the scale that turns it into v.
//      Per step: p = tau A22 v (four threads per row), then the symmetric
//      rank-2 update A22 -= v w^T + w v^T with w = p - (tau/2)(p.v) v; two
//      barriers per step.
//   2. The K largest eigenvalues of T by multisection: a group of 16-64 lanes
//      inside one wavefront per eigenvalue, two Sturm counts per lane (the
//      number of eigenvalues below x, from the signs of the LDL^T pivots), and
//      a ballot that picks the sub-interval holding the eigenvalue; no
//      barriers, as many rounds as FP64 resolution needs.
//   3. Eigenvectors of T by inverse iteration: one LU factorisation of
//      T - lambda I with partial pivoting per eigenvalue, then two solves from
//      a seeded start vector.
//   4. Back-transformation z <- H_0 ... H_{n-3} z, half a wavefront per vector,
//      then CholeskyQR2 of the K vectors (modified Gram-Schmidt when a pivot is
//      not safely positive).
#include <cmath>

#include "common.hpp"

namespace tk {

constexpr int EIG_THREADS = 512;
constexpr int EIG_WAVES = EIG_THREADS / 64;

// Offsets, in doubles, of the solver's arrays.  A (n x (n+1)) comes first; the
// rest follows it, in LDS or in the global workspace.
struct EigLayout {
  int64_t A, d, e, e2, tau, scl, p, red, Z, lu, lam, gm;
  int64_t a_size, total;
};

static EigLayout eig_layout(int n, int K) {
  EigLayout L{};
  int64_t o = 0;
  L.A = o; o += (int64_t)n * (n + 1);
  L.a_size = o;
  L.d = o; o += n;
  L.e = o; o += n;
  L.e2 = o; o += n;
  L.tau = o; o += n;
  L.scl = o; o += n;
  L.p = o; o += n;
  L.red = o; o += 64;
  L.Z = o; o += (int64_t)K * n;
  L.lu = o; o += (int64_t)K * 5 * n;   // per vector: 1/u0, u1, u2, multiplier, pivot flag
  L.lam = o; o += K;
  L.gm = o; o += 2 * (int64_t)K * K + 2;
  L.total = o;
  return L;
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ double half_sum(double x) {   // over each 32-lane half
  for (int off = 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Data-parallel-primitive move of a double (both 32-bit halves with the same control).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each row of 16 lanes, in every lane of the row: swap neighbours,
// swap pairs (quad permutes), then mirror within 8 and within 16 lanes.
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp_mov<0x141>(x);   // row_half_mirror
  x += dpp_mov<0x140>(x);   // row_mirror
  return x;
}

// row16_sum of several independent values, stage by stage (the DPP chains overlap)
template <int NV>
__device__ __forceinline__ void row16_sum_n(double (&x)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_mov<0xB1>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_mov<0x4E>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_mov<0x141>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_mov<0x140>(x[v]);
}

__device__ __forceinline__ double lane_val(double x, int l) {   // x of lane l (l wave-uniform)
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave sum as a wave-uniform value (same order in every wave).
__device__ __forceinline__ double wave_sum_u(double x) {
  x = row16_sum(x);
  return (lane_val(x, 0) + lane_val(x, 16)) + (lane_val(x, 32) + lane_val(x, 48));
}

// Sum over the workgroup: wave sums, then every thread adds the wave partials in order.
__device__ __forceinline__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < EIG_WAVES; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Eigenvalues of the symmetric tridiagonal (d, e) below x0 and below x1 (two
// independent recurrences interleaved).
__device__ __forceinline__ void sturm_count2(const double* d, const double* e2, int n, double x0, double x1,
                                             double pivmin, int& c0, int& c1) {
  double q0 = d[0] - x0, q1 = d[0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  c0 = q0 < 0.0;
  c1 = q1 < 0.0;
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
    q0 = di - x0 - ei / q0;
    q1 = di - x1 - ei / q1;
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    c0 += q0 < 0.0;
    c1 += q1 < 0.0;
  }
}

// Counter-based start vector entry (SplitMix64 mix of (j, i)) in [-1, 1).
__device__ __forceinline__ double start_entry(int j, int i) {
  unsigned long long z = 0x9E3779B97F4A7C15ULL * (unsigned long long)(j * 1315423911u + i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Modified Gram-Schmidt over the K rows of Z (each of length n), block-wide.
template <class P>
__device__ void mgs_rows(P Z, int K, int n, double* red) {
  for (int j = 0; j < K; ++j) {
    P zj = Z + (int64_t)j * n;
    for (int i = 0; i < j; ++i) {
      P zi = Z + (int64_t)i * n;
      double s = 0.0;
      for (int t = threadIdx.x; t < n; t += blockDim.x) s += zi[t] * zj[t];
      s = block_sum(s, red);
      for (int t = threadIdx.x; t < n; t += blockDim.x) zj[t] -= s * zi[t];
      __syncthreads();
    }
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) s += zj[t] * zj[t];
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) zj[t] *= inv;
    __syncthreads();
  }
}

// Orthonormalise the K rows of Z by CholeskyQR twice (Gram matrix of the rows,
// its Cholesky factor R, rows <- R^-T rows); falls back to modified
// Gram-Schmidt when a pivot is not safely positive.  gm: 2*K*K doubles + a flag,
// tmp: K*n.
template <class P>
__device__ void orth_rows(P Z, int K, int n, P gm, P tmp, double* red) {
  P R = gm + K * K;
  int* flag = reinterpret_cast<int*>(&gm[2 * K * K]);
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
      const int a = q / K, b = q - a * K;
      double s = 0.0;
      if (a <= b)
        for (int t = 0; t < n; ++t) s += Z[(int64_t)a * n + t] * Z[(int64_t)b * n + t];
      gm[q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int ok = 1;
      double dmax = 0.0;
      for (int i = 0; i < K; ++i) dmax = fmax(dmax, gm[i * K + i]);
      for (int i = 0; i < K * K; ++i) R[i] = 0.0;
      for (int j = 0; j < K && ok; ++j) {
        double dj = gm[j * K + j];
        for (int k = 0; k < j; ++k) dj -= R[k * K + j] * R[k * K + j];
        if (!(dj > 1e-20 * dmax)) { ok = 0; break; }
        const double rjj = sqrt(dj);
        R[j * K + j] = rjj;
        for (int i = j + 1; i < K; ++i) {
          double v = gm[j * K + i];
          for (int k = 0; k < j; ++k) v -= R[k * K + j] * R[k * K + i];
          R[j * K + i] = v / rjj;
        }
      }
      *flag = ok;
    }
    __syncthreads();
    if (!*flag) {  // (rare) nearly dependent vectors
      mgs_rows(Z, K, n, red);
      return;
    }
    // rows: q_j = (z_j - sum_{i<j} R[i][j] q_i) / R[j][j], solved column by column in parallel over t
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      for (int j = 0; j < K; ++j) {
        double v = Z[(int64_t)j * n + t];
        for (int i = 0; i < j; ++i) v -= R[i * K + j] * tmp[(int64_t)i * n + t];
        tmp[(int64_t)j * n + t] = v / R[j * K + j];
      }
      for (int j = 0; j < K; ++j) Z[(int64_t)j * n + t] = tmp[(int64_t)j * n + t];
    }
    __syncthreads();
  }
}

// MODE 2: everything in LDS.  MODE 1: A in the global workspace, the rest in
// LDS.  MODE 0: everything in the global workspace.
template <int MODE>
__global__ __launch_bounds__(EIG_THREADS) void k_syev_topk(const double* __restrict__ G, int n, int K, int Kout,
                                                           EigLayout L, double* __restrict__ gws,
                                                           double* __restrict__ lam_out, double* __restrict__ VK) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int stride = n + 1;
  double* A = MODE == 2 ? sh : gws;
  // the remaining arrays: in LDS (MODE 1 and 2, after A only in MODE 2) or after A in the workspace
  auto at = [&](int64_t off) -> double* { return MODE == 0 ? gws + off : sh + (off - (MODE == 1 ? L.a_size : 0)); };
  double* d = at(L.d);
  double* e = at(L.e);
  double* e2 = at(L.e2);
  double* tau = at(L.tau);
  double* scl = at(L.scl);
  double* p = at(L.p);
  double* red = at(L.red);
  double* Z = at(L.Z);
  double* lu = at(L.lu);
  double* lam = at(L.lam);
  double* gm = at(L.gm);

  for (int i = wave; i < n; i += EIG_WAVES)
    for (int j = lane; j < n; j += 64) A[(int64_t)i * stride + j] = G[(int64_t)i * n + j];
  __syncthreads();

  // 1. tridiagonalisation
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const double* rowk = A + (int64_t)k * stride + (k + 1);   // x_0..x_{m-1}, later the reflector
    double s = 0.0;
    for (int i = lane + 1; i < m; i += 64) s += rowk[i] * rowk[i];
    const double xn2 = wave_sum(s);     // every wave computes the same value
    const double alpha = rowk[0];
    if (xn2 == 0.0) {                   // the column is already reduced: identity reflector
      if (tid == 0) {
        d[k] = A[(int64_t)k * stride + k];
        e[k] = alpha;
        tau[k] = 0.0;
        scl[k] = 0.0;
      }
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    const double t = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    // p = t * A22 v, four threads per row
    for (int i0 = 0; i0 < m; i0 += EIG_THREADS / 4) {
      const int i = i0 + (tid >> 2), sub = tid & 3;
      double acc = 0.0;
      if (i < m) {
        const double* row = A + (int64_t)(k + 1 + i) * stride + (k + 1);
        for (int j = sub; j < m; j += 4) acc += row[j] * (j == 0 ? 1.0 : rowk[j] * scale);
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (i < m && sub == 0) p[i] = t * acc;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = lane; i < m; i += 64) pv += p[i] * (i == 0 ? 1.0 : rowk[i] * scale);
    const double kc = 0.5 * t * wave_sum(pv);
    // A22 -= v w^T + w v^T, rows over waves, columns over lanes
    for (int i = wave; i < m; i += EIG_WAVES) {
      const double vi = i == 0 ? 1.0 : rowk[i] * scale;
      const double wi = p[i] - kc * vi;
      double* row = A + (int64_t)(k + 1 + i) * stride + (k + 1);
      for (int j = lane; j < m; j += 64) {
        const double vj = j == 0 ? 1.0 : rowk[j] * scale;
        const double wj = p[j] - kc * vj;
        row[j] -= vi * wj + wi * vj;
      }
    }
    if (tid == 0) {
      d[k] = A[(int64_t)k * stride + k];
      e[k] = beta;
      tau[k] = t;
      scl[k] = scale;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(int64_t)(n - 2) * stride + (n - 2)];
      e[n - 2] = A[(int64_t)(n - 2) * stride + (n - 1)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = A[(int64_t)(n - 1) * stride + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += EIG_THREADS) e2[i] = e[i] * e[i];
  __syncthreads();

  // Gershgorin interval and scales (every thread, same order)
  double glo = 1e300, ghi = -1e300, emax = 0.0, tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    glo = fmin(glo, d[i] - r);
    ghi = fmax(ghi, d[i] + r);
    emax = fmax(emax, i + 1 < n ? e2[i] : 0.0);
    tnorm = fmax(tnorm, fabs(d[i]) + r);
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = fmax(2.2250738585072014e-308, eps * eps * emax);
  const double widen = 2.0 * eps * fmax(fabs(glo), fabs(ghi)) + pivmin;
  glo -= widen;
  ghi += widen;

  // 2. multisection: MS lanes (inside one wave) per eigenvalue, two points per lane
  {
    const int MS = K <= 8 ? 64 : (K <= 16 ? 32 : 16);
    const int NP = 2 * MS;                       // points per round -> NP + 1 sub-intervals
    const int g = tid / MS, q = tid % MS;
    const int gbase = lane & ~(MS - 1);
    const unsigned long long gmask = MS == 64 ? ~0ULL : (((1ULL << MS) - 1) << gbase);
    const double tol = 2.0 * eps * fmax(fabs(glo), fabs(ghi)) + pivmin;
    int rounds = 1;
    for (double w = ghi - glo; w > tol && rounds < 24; w /= (double)(NP + 1)) ++rounds;
    const bool act = g < K;
    const int idx = n - 1 - g;                   // ascending index of the g-th largest
    double a = glo, b = ghi;
    for (int r = 0; r < rounds; ++r) {
      const double h = (b - a) / (double)(NP + 1);
      const double x0 = a + h * (double)(2 * q + 1), x1 = a + h * (double)(2 * q + 2);
      int c0 = 0, c1 = 0;
      if (act) sturm_count2(d, e2, n, x0, x1, pivmin, c0, c1);
      // points with at most idx eigenvalues below them lie below the eigenvalue
      const unsigned long long m0 = __ballot(c0 <= idx) & gmask, m1 = __ballot(c1 <= idx) & gmask;
      const int P = __popcll(m0) + __popcll(m1);
      const double na = P == 0 ? a : a + h * (double)P;
      const double nb = P == NP ? b : a + h * (double)(P + 1);
      a = na;
      b = nb;
    }
    if (act && q == 0) lam[g] = 0.5 * (a + b);
  }
  __syncthreads();

  // 3. eigenvectors of T by inverse iteration, thread j for eigenvector j
  const double tiny = eps * fmax(tnorm, pivmin);
  for (int j = tid; j < K; j += EIG_THREADS) {
    double lj = lam[j];
    // separate (numerically) equal eigenvalues so the factorisations differ
    for (int i = 0; i < j; ++i)
      if (fabs(lam[i] - lj) < 10.0 * eps * fmax(tnorm, 1e-300)) lj -= 10.0 * eps * fmax(tnorm, 1e-300);
    double* ui = lu + (int64_t)j * 5 * n;   // 1/u0
    double* u1 = ui + n;
    double* u2 = u1 + n;
    double* ml = u2 + n;
    double* pv = ml + n;
    double* z = Z + (int64_t)j * n;
    double a0 = d[0] - lj, a1 = n > 1 ? e[0] : 0.0, a2 = 0.0;
    for (int i = 0; i < n - 1; ++i) {
      const double c = e[i], nd = d[i + 1] - lj, ns = i + 1 < n - 1 ? e[i + 1] : 0.0;
      if (fabs(c) > fabs(a0)) {         // swap rows i and i+1
        const double mlt = a0 / c;
        ui[i] = 1.0 / c; u1[i] = nd; u2[i] = ns; ml[i] = mlt; pv[i] = 1.0;
        a0 = a1 - mlt * nd;
        a1 = a2 - mlt * ns;
      } else {
        if (a0 == 0.0) a0 = tiny;
        const double mlt = c / a0;
        ui[i] = 1.0 / a0; u1[i] = a1; u2[i] = a2; ml[i] = mlt; pv[i] = 0.0;
        a0 = nd - mlt * a1;
        a1 = ns - mlt * a2;
      }
      a2 = 0.0;
    }
    if (a0 == 0.0) a0 = tiny;
    ui[n - 1] = 1.0 / a0; u1[n - 1] = 0.0; u2[n - 1] = 0.0; ml[n - 1] = 0.0; pv[n - 1] = 0.0;
    for (int i = 0; i < n; ++i) z[i] = start_entry(j, i);
    for (int it = 0; it < 2; ++it) {
      for (int i = 0; i < n - 1; ++i) {
        if (pv[i] != 0.0) {
          const double t0 = z[i];
          z[i] = z[i + 1];
          z[i + 1] = t0 - ml[i] * z[i + 1];
        } else {
          z[i + 1] -= ml[i] * z[i];
        }
      }
      double z1 = 0.0, z2 = 0.0, nrm = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        const double s = (z[i] - u1[i] * z1 - u2[i] * z2) * ui[i];
        z[i] = s;
        z2 = z1;
        z1 = s;
        nrm += s * s;
      }
      nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < n; ++i) z[i] *= nrm;
    }
  }
  __syncthreads();

  // 4. back-transformation, half a wave per vector (both halves run every
  // iteration: the shuffles need the whole wave)
  {
    const int half = lane >> 5, hl = lane & 31;
    for (int j0 = 0; j0 < K; j0 += 2 * EIG_WAVES) {
      const int j = j0 + 2 * wave + half;
      const bool on = j < K;
      double* z = Z + (int64_t)(on ? j : 0) * n;
      for (int k = n - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        const int m = n - k - 1;
        const double* rowk = A + (int64_t)k * stride + (k + 1);
        const double sc = scl[k];
        double s = 0.0;
        if (on)
          for (int i = hl; i < m; i += 32) s += (i == 0 ? 1.0 : rowk[i] * sc) * z[k + 1 + i];
        s = half_sum(s);
        if (on)
          for (int i = hl; i < m; i += 32) z[k + 1 + i] -= t * s * (i == 0 ? 1.0 : rowk[i] * sc);
      }
    }
  }
  __syncthreads();
  orth_rows(Z, K, n, gm, lu, red);
  for (int t = tid; t < n * K; t += EIG_THREADS) {
    const int i = t / K, j = t - i * K;
    VK[(int64_t)i * Kout + j] = Z[(int64_t)j * n + i];
  }
  for (int j = tid; j < K; j += EIG_THREADS) lam_out[j] = lam[j];
}

// ---- K-hat <= 128: fused, register-resident variant --------------------------------------------
//
// Lane l of every wave owns the columns J = l and J = l + 64.  Step k holds the
// reflector v_k and w_k = p_k - (tau_k/2)(p_k.v_k) v_k in registers (zero for
// J <= k).  One pass per step updates rows k+2.. of the trailing matrix with
// reflector k and, on the updated values, accumulates the product p_{k+1} =
// tau_{k+1} A v_{k+1} of the next reflector, which every wave builds from the
// updated row k+1 on its own.  The eight waves' partial products meet in LDS
// (double-buffered by step parity), so each step has a single barrier.
constexpr int SM_N = 128;

__device__ __forceinline__ double rl(double x, int l) { return lane_val(x, l); }

// value at column J of a two-register row (J wave-uniform)
__device__ __forceinline__ double col_of(const double (&x)[2], int J) { return rl(J < 64 ? x[0] : x[1], J & 63); }

struct SmallLayout {
  int64_t A, part, vec, d, e, e2, tau, scl, red, lam, Z, lu, gm, total;
};

static SmallLayout small_layout(int n, int K) {
  SmallLayout L{};
  int64_t o = 0;
  L.A = o; o += (int64_t)n * (n + 1);
  L.part = o; o += 2 * EIG_WAVES * SM_N;
  L.vec = o; o += 2 * 3 * SM_N;
  L.d = o; o += n;
  L.e = o; o += n;
  L.e2 = o; o += n;
  L.tau = o; o += n;
  L.scl = o; o += n;
  L.red = o; o += 64;
  L.lam = o; o += 32;
  L.Z = o; o += (int64_t)K * n;
  L.lu = o; o += (int64_t)K * 5 * n;
  L.gm = o; o += 2 * (int64_t)K * K + 2;
  L.total = o;
  return L;
}

// Reflector that maps the entries J >= j0 of a register row x to a multiple of
// e_{j0}: beta, tau, scale and v (v_{j0} = 1, v_J = x_J * scale for J > j0, 0 below).
__device__ __forceinline__ void reflector(const double (&x)[2], int j0, int n, double& beta, double& t, double& scale,
                                          double (&v)[2]) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int J = lane + 64 * c;
    if (J > j0 && J < n) s += x[c] * x[c];
  }
  const double xn2 = wave_sum_u(s);
  const double alpha = col_of(x, j0);
  if (xn2 == 0.0) {
    beta = alpha;
    t = 0.0;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    // Newton-refined reciprocals: the two divisions sit on every step's critical path
    double rb = __builtin_amdgcn_rcp(beta);
    rb = fma(fma(-beta, rb, 1.0), rb, rb);
    rb = fma(fma(-beta, rb, 1.0), rb, rb);
    const double am = alpha - beta;
    double ra = __builtin_amdgcn_rcp(am);
    ra = fma(fma(-am, ra, 1.0), ra, ra);
    ra = fma(fma(-am, ra, 1.0), ra, ra);
    t = (beta - alpha) * rb;
    scale = ra;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int J = lane + 64 * c;
    v[c] = J == j0 ? 1.0 : ((J > j0 && J < n) ? x[c] * scale : 0.0);
  }
}

// Sturm counts for the small kernel: q <- d_i - x - e_i^2 / q with a
// Newton-refined hardware reciprocal (two steps after the estimate).
// One Sturm count.
__device__ __forceinline__ int sturm_count1(const double* d, const double* e2, int n, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(fma(-q, r, 1.0), r, r);
    r = fma(fma(-q, r, 1.0), r, r);
    q = fma(-e2[i - 1], r, d[i] - x);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Two Sturm counts, interleaved, with the same arithmetic as sturm_count1.
__device__ __forceinline__ void sturm_count2r(const double* d, const double* e2, int n, double x0, double x1,
                                              double pivmin, int& c0, int& c1) {
  double q0 = d[0] - x0, q1 = d[0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  c0 = q0 < 0.0;
  c1 = q1 < 0.0;
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    const double di = d[i], ei = e2[i - 1];
    double r0 = __builtin_amdgcn_rcp(q0), r1 = __builtin_amdgcn_rcp(q1);
    r0 = fma(fma(-q0, r0, 1.0), r0, r0);
    r1 = fma(fma(-q1, r1, 1.0), r1, r1);
    r0 = fma(fma(-q0, r0, 1.0), r0, r0);
    r1 = fma(fma(-q1, r1, 1.0), r1, r1);
    q0 = fma(-ei, r0, di - x0);
    q1 = fma(-ei, r1, di - x1);
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    c0 += q0 < 0.0;
    c1 += q1 < 0.0;
  }
}

__global__ __launch_bounds__(EIG_THREADS) void k_syev_small(const double* __restrict__ G, int n, int K, int Kout,
                                                            SmallLayout L, double* __restrict__ lam_out,
                                                            double* __restrict__ VK) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int S = n + 1;
  double* A = sh + L.A;
  double* part = sh + L.part;
  double* vec = sh + L.vec;   // [v | w | v_next] of the current step, double-buffered by step parity
  double* d = sh + L.d;
  double* e = sh + L.e;
  double* e2 = sh + L.e2;
  double* tau = sh + L.tau;
  double* scl = sh + L.scl;
  double* red = sh + L.red;
  double* lam = sh + L.lam;
  double* Z = sh + L.Z;
  double* lu = sh + L.lu;
  double* gm = sh + L.gm;

  for (int i = wave; i < n; i += EIG_WAVES)
    for (int j = lane; j < n; j += 64) A[i * S + j] = G[(int64_t)i * n + j];
  __syncthreads();

  // 1. tridiagonalisation
  if (n <= 2) {
    if (tid == 0) {
      d[0] = A[0];
      e[0] = n == 2 ? A[1] : 0.0;
      tau[0] = 0.0;
      if (n == 2) { d[1] = A[S + 1]; e[1] = 0.0; tau[1] = 0.0; }
    }
  } else {
    double v[2], w[2], beta, t, scale;
    {
      double x[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int J = lane + 64 * c;
        x[c] = J < n ? A[J] : 0.0;
      }
      reflector(x, 1, n, beta, t, scale, v);
      double acc[2] = {0.0, 0.0};
      for (int I = 1 + wave; I < n; I += EIG_WAVES) {
        const double vI = col_of(v, I);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int J = lane + 64 * c;
          if (J >= 1 && J < n) acc[c] += A[I * S + J] * vI;
        }
      }
      double* pb = part + EIG_WAVES * SM_N;   // the odd buffer: step 0 writes the even one
#pragma unroll
      for (int c = 0; c < 2; ++c) pb[wave * SM_N + lane + 64 * c] = acc[c];
      __syncthreads();
      double pv = 0.0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double sp = 0.0;
        for (int ww = 0; ww < EIG_WAVES; ++ww) sp += pb[ww * SM_N + lane + 64 * c];
        const double pc = t * sp;
        w[c] = pc;
        pv += pc * v[c];
      }
      const double kc = 0.5 * t * wave_sum_u(pv);
#pragma unroll
      for (int c = 0; c < 2; ++c) w[c] -= kc * v[c];
      if (tid == 0) {
        d[0] = A[0];
        e[0] = beta;
        tau[0] = t;
        scl[0] = scale;
      }
    }
    for (int k = 0; k + 2 < n; ++k) {
      // row k+1 after reflector k (v_{k+1} = 1)
      const double wk1 = col_of(w, k + 1);
      double nr[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int J = lane + 64 * c;
        nr[c] = (J >= k + 1 && J < n) ? A[(k + 1) * S + J] - (w[c] + wk1 * v[c]) : 0.0;
      }
      const bool next = k + 3 < n;   // reflector k+1 exists
      double vn[2] = {0.0, 0.0}, bn = 0.0, tn = 0.0, sn = 0.0;
      if (next) reflector(nr, k + 2, n, bn, tn, sn, vn);
      // rows k+2.. : update with reflector k, accumulate A v_{k+1}
      double acc[2] = {0.0, 0.0};
      bool cok[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int J = lane + 64 * c;
        cok[c] = J >= k + 2 && J < n;
      }
      // the row constants v_I, w_I, v_next_I come from LDS as broadcast reads:
      // every wave stores the same vectors, and reads back only its own stores
      double* vb = vec + (k & 1) * 3 * SM_N;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        vb[lane + 64 * c] = v[c];
        vb[SM_N + lane + 64 * c] = w[c];
        vb[2 * SM_N + lane + 64 * c] = vn[c];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // four rows per iteration: all loads are issued before the first store;
      // lanes outside the trailing block load and store the row's unused
      // padding column, so no load or store is predicated
      int coff[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) coff[c] = cok[c] ? lane + 64 * c : n;
      for (int I0 = k + 2 + wave; I0 < n; I0 += 4 * EIG_WAVES) {
        double a[4][2], cv[4], cw[4], cn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int I = I0 + u * EIG_WAVES;
          const int Ic = I < n ? I : n - 1;
#pragma unroll
          for (int c = 0; c < 2; ++c) a[u][c] = A[Ic * S + coff[c]];
          cv[u] = vb[Ic];
          cw[u] = vb[SM_N + Ic];
          cn[u] = vb[2 * SM_N + Ic];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int I = I0 + u * EIG_WAVES;
          if (I < n) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double x = a[u][c] - (cv[u] * w[c] + cw[u] * v[c]);
              A[I * S + coff[c]] = x;
              acc[c] += x * cn[u];
            }
          }
        }
      }
      double* pb = part + (k & 1) * EIG_WAVES * SM_N;
#pragma unroll
      for (int c = 0; c < 2; ++c) pb[wave * SM_N + lane + 64 * c] = acc[c];
      __syncthreads();
      if (wave == 0) {
        // row k+1 keeps the next reflector's entries; the back-transformation reads them
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int J = lane + 64 * c;
          if (J >= k + 2 && J < n) A[(k + 1) * S + J] = nr[c];
        }
        const double dk1 = col_of(nr, k + 1), ek1 = next ? bn : col_of(nr, k + 2);   // whole wave active
        if (lane == 0) {
          d[k + 1] = dk1;
          e[k + 1] = ek1;
          tau[k + 1] = next ? tn : 0.0;
          scl[k + 1] = next ? sn : 0.0;
        }
      }
      if (!next) break;
      double pv = 0.0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double sp = 0.0;
        for (int ww = 0; ww < EIG_WAVES; ++ww) sp += pb[ww * SM_N + lane + 64 * c];
        const int J = lane + 64 * c;
        const double pc = (J >= k + 2 && J < n) ? tn * sp : 0.0;
        w[c] = pc;
        pv += pc * vn[c];
      }
      const double kc = 0.5 * tn * wave_sum_u(pv);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        w[c] -= kc * vn[c];
        v[c] = vn[c];
      }
    }
    __syncthreads();
    if (tid == 0) {
      d[n - 1] = A[(n - 1) * S + (n - 1)];
      e[n - 1] = 0.0;
      tau[n - 1] = 0.0;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += EIG_THREADS) e2[i] = e[i] * e[i];
  __syncthreads();

  double glo = 1e300, ghi = -1e300, emax = 0.0, tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    glo = fmin(glo, d[i] - r);
    ghi = fmax(ghi, d[i] + r);
    emax = fmax(emax, i + 1 < n ? e2[i] : 0.0);
    tnorm = fmax(tnorm, fabs(d[i]) + r);
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = fmax(2.2250738585072014e-308, eps * eps * emax);
  const double widen = 2.0 * eps * fmax(fabs(glo), fabs(ghi)) + pivmin;
  glo -= widen;
  ghi += widen;

  // 2. multisection, 16 lanes x 2 points per eigenvalue (33 sub-intervals per
  // round) until the interval is below 1e-11 of the spectrum's scale: inverse
  // iteration needs no more, and the eigenvalues only scale U's columns.  Two
  // interleaved recurrences per lane: a Sturm step is a chain of dependent
  // FP64 operations, so four points per lane cost twice the time of two for
  // one more bit per round.
  {
    const int g = tid >> 4, q = tid & 15;
    const int gbase = lane & ~15;
    const unsigned long long gmask = 0xFFFFULL << gbase;
    const double tol = 1e-11 * fmax(tnorm, pivmin);
    const bool act = g < K;
    const int idx = n - 1 - g;
    constexpr int NP = 32;
    // joint first round: one point per thread over the whole interval serves
    // every eigenvalue at once (the partial-product buffer is free by now)
    int* cnt0 = reinterpret_cast<int*>(part);
    const double h0 = (ghi - glo) / (double)(EIG_THREADS + 1);
    cnt0[tid] = sturm_count1(d, e2, n, glo + h0 * (double)(tid + 1), pivmin);
    __syncthreads();
    int t0 = -1, t1 = EIG_THREADS - 1;   // largest t with cnt0[t] <= idx (counts rise with x)
    while (t0 < t1) {
      const int mid = (t0 + t1 + 1) >> 1;
      if (cnt0[mid] <= idx) t0 = mid; else t1 = mid - 1;
    }
    double a = t0 < 0 ? glo : glo + h0 * (double)(t0 + 1);
    double b = t0 >= EIG_THREADS - 1 ? ghi : glo + h0 * (double)(t0 + 2);
    int rounds = 0;
    for (double wd = h0; wd > tol && rounds < 32; wd /= (double)(NP + 1)) ++rounds;
    for (int r = 0; r < rounds; ++r) {
      const double h = (b - a) / (double)(NP + 1);
      const double x0 = a + h * (double)(2 * q + 1), x1 = a + h * (double)(2 * q + 2);
      int c0 = 0, c1 = 0;
      if (act) sturm_count2r(d, e2, n, x0, x1, pivmin, c0, c1);
      const int P = __popcll(__ballot(c0 <= idx) & gmask) + __popcll(__ballot(c1 <= idx) & gmask);
      const double na = P == 0 ? a : a + h * (double)P;
      const double nb = P == NP ? b : a + h * (double)(P + 1);
      a = na;
      b = nb;
    }
    if (act && q == 0) lam[g] = 0.5 * (a + b);
  }
  __syncthreads();

  // 3. inverse iteration (as in the general kernel), one lane per vector.  The
  // recurrences are sequential, so their operands are loaded in chunks of
  // eight steps ahead of use (one LDS round trip per chunk instead of one
  // per step), the pivot choice is a select, and divisions are a
  // Newton-refined reciprocal.
  const double tiny = eps * fmax(tnorm, pivmin);
  for (int j = tid; j < K; j += EIG_THREADS) {
    double lj = lam[j];
    for (int i = 0; i < j; ++i)
      if (fabs(lam[i] - lj) < 10.0 * eps * fmax(tnorm, 1e-300)) lj -= 10.0 * eps * fmax(tnorm, 1e-300);
    double* ui = lu + (int64_t)j * 5 * n;
    double* u1 = ui + n;
    double* u2 = u1 + n;
    double* ml = u2 + n;
    double* pv = ml + n;
    double* z = Z + (int64_t)j * n;
    constexpr int CH = 8;
    auto rcp = [](double x) {
      double r = __builtin_amdgcn_rcp(x);
      r = fma(fma(-x, r, 1.0), r, r);
      return fma(fma(-x, r, 1.0), r, r);
    };
    // LU factorisation with partial pivoting of T - lj I; full chunks of CH
    // steps carry no bounds checks (a branch per step costs more than the
    // step), the remainder goes one step at a time
    double a0 = d[0] - lj, a1 = n > 1 ? e[0] : 0.0, a2 = 0.0;
    auto lu_step = [&](int i, double c, double ndl, double ns) __attribute__((always_inline)) {
      const double nd = ndl - lj;
      const bool sw = fabs(c) > fabs(a0);
      const double p0 = sw ? c : (a0 == 0.0 ? tiny : a0);
      const double r = rcp(p0);
      const double mlt = (sw ? a0 : c) * r;
      const double y1 = sw ? nd : a1, y2 = sw ? ns : a2;   // the pivot row's entries
      const double x1 = sw ? a1 : nd, x2 = sw ? a2 : ns;   // the other row's
      ui[i] = r; u1[i] = y1; u2[i] = y2; ml[i] = mlt; pv[i] = sw ? 1.0 : 0.0;
      a0 = x1 - mlt * y1;
      a1 = x2 - mlt * y2;
      a2 = 0.0;
    };
    const int nl = n - 1;                  // LU steps
    const int nfull = nl / CH * CH;
    for (int i0 = 0; i0 < nfull; i0 += CH) {
      double ce[CH], cd[CH], cs[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        ce[u] = e[i0 + u];
        cd[u] = d[i0 + u + 1];
        cs[u] = i0 + u + 1 < nl ? e[i0 + u + 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) lu_step(i0 + u, ce[u], cd[u], cs[u]);
    }
    for (int i = nfull; i < nl; ++i) lu_step(i, e[i], d[i + 1], i + 1 < nl ? e[i + 1] : 0.0);
    if (a0 == 0.0) a0 = tiny;
    ui[n - 1] = rcp(a0); u1[n - 1] = 0.0; u2[n - 1] = 0.0; ml[n - 1] = 0.0; pv[n - 1] = 0.0;
    for (int i = 0; i < n; ++i) z[i] = start_entry(j, i);
    for (int it = 0; it < 2; ++it) {
      // forward elimination with the row interchanges
      double cur = z[0];
      auto fw_step = [&](int i, double nx, double mi, double p) __attribute__((always_inline)) {
        const bool sw = p != 0.0;
        z[i] = sw ? nx : cur;
        cur = sw ? fma(-mi, nx, cur) : fma(-mi, cur, nx);
      };
      for (int i0 = 0; i0 < nfull; i0 += CH) {
        double cz[CH], cm[CH], cp[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          cz[u] = z[i0 + u + 1];
          cm[u] = ml[i0 + u];
          cp[u] = pv[i0 + u];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) fw_step(i0 + u, cz[u], cm[u], cp[u]);
      }
      for (int i = nfull; i < nl; ++i) fw_step(i, z[i + 1], ml[i], pv[i]);
      z[n - 1] = cur;
      // back substitution with U (three diagonals), then normalise
      double z1 = 0.0, z2 = 0.0, nrm = 0.0;
      auto bw_step = [&](int i, double zi, double a, double b, double r) __attribute__((always_inline)) {
        const double sv = (zi - a * z1 - b * z2) * r;
        z[i] = sv;
        z2 = z1;
        z1 = sv;
        nrm += sv * sv;
      };
      const int bfull = n / CH * CH;       // steps n-1 .. n-bfull in full chunks
      for (int i0 = n - 1; i0 > n - 1 - bfull; i0 -= CH) {
        double cz[CH], c1[CH], c2[CH], cr[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          cz[u] = z[i0 - u];
          c1[u] = u1[i0 - u];
          c2[u] = u2[i0 - u];
          cr[u] = ui[i0 - u];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) bw_step(i0 - u, cz[u], c1[u], c2[u], cr[u]);
      }
      for (int i = n - 1 - bfull; i >= 0; --i) bw_step(i, z[i], u1[i], u2[i], ui[i]);
      nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < n; ++i) z[i] *= nrm;
    }
  }
  __syncthreads();

  // 4. back-transformation: half a wave per vector, every half-wave's vectors
  // (K <= 16: at most two) in registers and reduced together, so the
  // latency of one reflector's reductions is paid once for both; the next
  // reflector's row is loaded while the current one is applied
  {
    const int half = lane >> 5, hl = lane & 31;
    constexpr int NV = 2;
    double z[NV][4];
    bool on[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int j = 2 * wave + half + 2 * EIG_WAVES * v;
      on[v] = j < K;
      const double* zr = Z + (int64_t)(on[v] ? j : 0) * n;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = hl + 32 * c;
        z[v][c] = (on[v] && i < n) ? zr[i] : 0.0;
      }
    }
    int ic[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) ic[c] = min(hl + 32 * c, n - 1);
    // reflector k's row, tau and scale are loaded one step ahead: LDS returns
    // in order, so a wait for this step's operands never waits for the next
    double xn[4], tn = 0.0, sn = 0.0;
    if (n >= 3) {
#pragma unroll
      for (int c = 0; c < 4; ++c) xn[c] = A[(n - 3) * S + ic[c]];
      tn = tau[n - 3];
      sn = scl[n - 3];
    }
    for (int k = n - 3; k >= 0; --k) {
      double x[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] = xn[c];
      const double t = tn, sc = sn;
      if (k > 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) xn[c] = A[(k - 1) * S + ic[c]];
        tn = tau[k - 1];
        sn = scl[k - 1];
      }
      if (t == 0.0) continue;
      double vv[4], sv[NV];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = hl + 32 * c;
        vv[c] = i == k + 1 ? 1.0 : ((i > k + 1 && i < n) ? x[c] * sc : 0.0);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += vv[c] * z[v][c];
        sv[v] = acc;
      }
      // the vectors' row sums stage by stage, interleaved
      row16_sum_n<NV>(sv);
      // each half-wave's sum: its two rows of 16 lanes
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double s0 = lane_val(sv[v], 0) + lane_val(sv[v], 16), s1 = lane_val(sv[v], 32) + lane_val(sv[v], 48);
        const double sh = t * (half ? s1 : s0);
#pragma unroll
        for (int c = 0; c < 4; ++c) z[v][c] -= sh * vv[c];
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!on[v]) continue;
      double* zr = Z + (int64_t)(2 * wave + half + 2 * EIG_WAVES * v) * n;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = hl + 32 * c;
        if (i < n) zr[i] = z[v][c];
      }
    }
  }
  __syncthreads();
  // inverse iteration leaves vectors of eigenvalues more than 1e-3 ||T|| apart
  // orthogonal to working accuracy; closer ones are orthonormalised together
  bool cluster = false;
  for (int j = 1; j < K; ++j) cluster |= fabs(lam[j - 1] - lam[j]) < 1e-3 * tnorm;
  if (cluster) orth_rows(Z, K, n, gm, lu, red);
  for (int t = tid; t < n * K; t += EIG_THREADS) {
    const int i = t / K, j = t - i * K;
    VK[(int64_t)i * Kout + j] = Z[(int64_t)j * n + i];
  }
  for (int j = tid; j < K; j += EIG_THREADS) lam_out[j] = lam[j];
}

void eig_topk_krylov(Ctx* c, const double* G, int n, int K, int Kout, double* lam_k, double* VK, int mode);

constexpr int KRYLOV_MIN_N = 192;   // above this, and for K <= 16, the block-Krylov solver

// Leading K eigenpairs of G (n0 x n0, FP64): lam_k[0..K) descending and VK (n0 x K).
// Eigenpairs beyond n0 (K > n0) are reported as zero eigenvalues.  mode >= 0
// lets the Krylov solver start from that mode's previous eigenvectors.
// The dense solvers (one workgroup): LDS-resident for K-hat up to about 128,
// otherwise with the matrix in LDS or global memory.
void eig_topk_dense(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK) {
  const int Ke = K < n0 ? K : n0;
  TK_REQUIRE(Ke <= 32, TK_ERR_UNSUPPORTED, "eigensolve: more than 32 eigenpairs");
  const size_t lim = c->lds_per_block;
  const SmallLayout SL = small_layout(n0, Ke);
  const bool small = n0 <= SM_N && Ke <= 16 && (size_t)SL.total * 8 <= lim;
  const EigLayout L = eig_layout(n0, Ke);
  ensure(c, c->work, sizeof(double) * (size_t)(L.total + 16));
  if (K > Ke) TK_HIP(hipMemsetAsync(lam_k, 0, sizeof(double) * K, c->stream));
  double* ws = c->work.as<double>();
  if (small) {
    hipLaunchKernelGGL(k_syev_small, dim3(1), dim3(EIG_THREADS), (size_t)SL.total * 8, c->stream, G, n0, Ke, K, SL,
                       lam_k, VK);
  } else if ((size_t)L.total * 8 <= lim) {
    hipLaunchKernelGGL(k_syev_topk<2>, dim3(1), dim3(EIG_THREADS), (size_t)L.total * 8, c->stream, G, n0, Ke, K, L,
                       ws, lam_k, VK);
  } else if ((size_t)(L.total - L.a_size) * 8 <= lim) {
    hipLaunchKernelGGL(k_syev_topk<1>, dim3(1), dim3(EIG_THREADS), (size_t)(L.total - L.a_size) * 8, c->stream,
                       G, n0, Ke, K, L, ws, lam_k, VK);
  } else {
    hipLaunchKernelGGL(k_syev_topk<0>, dim3(1), dim3(EIG_THREADS), 0, c->stream, G, n0, Ke, K, L, ws, lam_k, VK);
  }
  TK_CHECK_LAUNCH();
}

void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK, int mode) {
  const int Ke = K < n0 ? K : n0;
  TK_REQUIRE(Ke <= 32, TK_ERR_UNSUPPORTED, "eigensolve: more than 32 eigenpairs");
  const SmallLayout SL = small_layout(n0, Ke);
  const bool small = n0 <= SM_N && Ke <= 16 && (size_t)SL.total * 8 <= c->lds_per_block;
  if (!small && n0 >= KRYLOV_MIN_N && Ke <= 16) {
    eig_topk_krylov(c, G, n0, Ke, K, lam_k, VK, mode);
    return;
  }
  eig_topk_dense(c, G, n0, K, lam_k, VK);
}

}  // namespace tk
