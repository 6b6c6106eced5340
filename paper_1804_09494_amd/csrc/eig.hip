// FP64 symmetric eigensolver for the Gram matrix G = Y^T Y (Khat x Khat):
// the leading K_n eigenpairs give the leading K_n left singular vectors of Y
// (Section 2.2: the SVD step of an HOOI invocation) as Y V_K S_K^-1.
//
// One workgroup, data resident in LDS when it fits:
//   1. Householder tridiagonalisation G = Q T Q^T (lower variant: reflector k
//      is I - tau_k v_k v_k^T on rows/columns k+1..n-1, v_k[0] = 1, kept in
//      column k below the diagonal);
//   2. the K largest eigenvalues of T by multisection: 16 threads per
//      eigenvalue evaluate Sturm counts (eigenvalues of T below x, from the
//      signs of the LDL^T pivots) at 16 interior points and keep the
//      sub-interval that holds it, 17x narrower per round;
//   3. eigenvectors of T by inverse iteration (tridiagonal LU with partial
//      pivoting, distinct seeded starts), then modified Gram-Schmidt across the
//      K vectors, one more inverse-iteration step and a second pass;
//   4. back-transformation z <- H_0 ... H_{n-3} z, one wave per vector.
#include <cmath>

#include "common.hpp"

namespace tk {

struct EigLayout {
  // offsets (in doubles) into the LDS or global workspace
  int64_t A, d, e, e2, tau, p, v, red, Z, lu, lam, brk, cnt, gm;
  int64_t total;
};

static EigLayout eig_layout(int n, int K, bool a_in_ws) {
  EigLayout L{};
  int64_t o = 0;
  const int64_t stride = n + 1;
  L.A = a_in_ws ? o : -1;
  if (a_in_ws) o += (int64_t)n * stride;
  L.d = o; o += n;
  L.e = o; o += n;
  L.e2 = o; o += n;
  L.tau = o; o += n;
  L.p = o; o += n;
  L.v = o; o += n;
  L.red = o; o += 64;
  L.Z = o; o += (int64_t)K * n;
  L.lu = o; o += (int64_t)K * 3 * n;
  L.lam = o; o += K;
  L.brk = o; o += 2 * (int64_t)K;
  L.cnt = o; o += 32 * (int64_t)K;   // ints stored in doubles' space (generous)
  L.gm = o; o += 2 * (int64_t)K * K + 2;
  L.total = o;
  return L;
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

constexpr int EIG_THREADS = 512;
constexpr int EIG_WAVES = EIG_THREADS / 64;

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

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x.
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
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
__device__ void mgs_rows(double* Z, int K, int n, double* red) {
  for (int j = 0; j < K; ++j) {
    double* zj = Z + (int64_t)j * n;
    for (int i = 0; i < j; ++i) {
      const double* zi = Z + (int64_t)i * n;
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
// Gram-Schmidt when a pivot is not safely positive.  gm: 2*K*K doubles, tmp: K*n.
__device__ void orth_rows(double* Z, int K, int n, double* gm, double* tmp, double* red, int* flag) {
  double* R = gm + K * K;
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
      const int a = q / K, b = q % K;
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
        double d = gm[j * K + j];
        for (int k = 0; k < j; ++k) d -= R[k * K + j] * R[k * K + j];
        if (!(d > 1e-20 * dmax)) { ok = 0; break; }
        const double rjj = sqrt(d);
        R[j * K + j] = rjj;
        for (int i = j + 1; i < K; ++i) {
          double v = gm[j * K + i];
          for (int k = 0; k < j; ++k) v -= R[k * K + j] * R[k * K + i];
          R[j * K + i] = v / rjj;
        }
      }
      flag[0] = ok;
    }
    __syncthreads();
    if (!flag[0]) {  // (rare) nearly dependent vectors
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

__global__ __launch_bounds__(EIG_THREADS) void k_syev_topk(const double* __restrict__ G, int n, int K, int Kout,
                                                   int a_in_lds, int ws_in_lds, double* __restrict__ gws,
                                                   double* __restrict__ lam_out, double* __restrict__ VK) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x;
  const int stride = n + 1;
  // workspace layout mirrors eig_layout(n, K, a_in_lds)
  double* ws = ws_in_lds ? sh : gws;
  int64_t o = 0;
  double* A;
  if (a_in_lds) {
    A = ws;
    o += (int64_t)n * stride;
  } else {
    A = gws;  // A occupies the head of the global workspace
  }
  if (!a_in_lds && !ws_in_lds) o += (int64_t)n * stride;
  double* d = ws + o; o += n;
  double* e = ws + o; o += n;
  double* e2 = ws + o; o += n;
  double* tau = ws + o; o += n;
  double* p = ws + o; o += n;
  double* v = ws + o; o += n;
  double* red = ws + o; o += 64;
  double* Z = ws + o; o += (int64_t)K * n;
  double* lu = ws + o; o += (int64_t)K * 3 * n;
  double* lam = ws + o; o += K;
  double* brk = ws + o; o += 2 * K;
  int* cnt = reinterpret_cast<int*>(ws + o); o += 32 * K;
  double* gm = ws + o; o += 2 * K * K;
  int* oflag = reinterpret_cast<int*>(ws + o);

  for (int64_t t = tid; t < (int64_t)n * n; t += blockDim.x) {
    const int i = (int)(t / n), j = (int)(t % n);
    A[(int64_t)i * stride + j] = G[t];
  }
  __syncthreads();

  // 1. tridiagonalisation
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double s = 0.0;
    for (int i = tid + 1; i < m; i += blockDim.x) {
      const double x = A[(int64_t)(k + 1 + i) * stride + k];
      s += x * x;
    }
    const double xn2 = block_sum(s, red);
    const double alpha = A[(int64_t)(k + 1) * stride + k];
    if (tid == 0) d[k] = A[(int64_t)k * stride + k];
    if (xn2 == 0.0) {
      if (tid == 0) {
        tau[k] = 0.0;
        e[k] = alpha;
      }
      __syncthreads();
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    const double t = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    for (int i = tid; i < m; i += blockDim.x) {
      const double vi = i == 0 ? 1.0 : A[(int64_t)(k + 1 + i) * stride + k] * scale;
      v[i] = vi;
    }
    __syncthreads();
    for (int i = tid; i < m; i += blockDim.x) A[(int64_t)(k + 1 + i) * stride + k] = v[i];
    // p = t * A22 v, four threads per row (quad reduction)
    for (int i0 = 0; i0 < m; i0 += EIG_THREADS / 4) {
      const int i = i0 + (tid >> 2), sub = tid & 3;
      double acc = 0.0;
      if (i < m) {
        const double* row = A + (int64_t)(k + 1 + i) * stride + (k + 1);
        for (int j = sub; j < m; j += 4) acc += row[j] * v[j];
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (i < m && sub == 0) p[i] = t * acc;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += blockDim.x) pv += p[i] * v[i];
    pv = block_sum(pv, red);
    const double kc = 0.5 * t * pv;
    for (int i = tid; i < m; i += blockDim.x) p[i] -= kc * v[i];
    __syncthreads();
    for (int64_t q = tid; q < (int64_t)m * m; q += blockDim.x) {
      const int i = (int)(q / m), j = (int)(q % m);
      A[(int64_t)(k + 1 + i) * stride + (k + 1 + j)] -= v[i] * p[j] + p[i] * v[j];
    }
    if (tid == 0) {
      tau[k] = t;
      e[k] = beta;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(int64_t)(n - 2) * stride + (n - 2)];
      e[n - 2] = A[(int64_t)(n - 1) * stride + (n - 2)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = A[(int64_t)(n - 1) * stride + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) e2[i] = e[i] * e[i];
  __syncthreads();
  // Gershgorin bounds and scales
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
  __syncthreads();

  // 2. the K largest eigenvalues by multisection (32 threads per eigenvalue, 33x narrower per round)
  constexpr int MS = 32;
  for (int j0 = 0; j0 < K; j0 += EIG_THREADS / MS) {
    const int g = tid / MS, q = tid % MS;
    const int j = j0 + g;
    const bool act = j < K;
    if (act && q == 0) {
      brk[2 * j] = glo;
      brk[2 * j + 1] = ghi;
    }
    __syncthreads();
    for (int round = 0; round < 12; ++round) {
      if (act) {
        const double a = brk[2 * j], b = brk[2 * j + 1];
        const double x = a + (b - a) * (double)(q + 1) / (double)(MS + 1);
        cnt[MS * j + q] = sturm_count(d, e2, n, x, pivmin);
      }
      __syncthreads();
      if (act && q == 0) {
        const int idx = n - 1 - j;  // ascending index of the j-th largest
        const double a = brk[2 * j], b = brk[2 * j + 1];
        double na = a, nb = b;
        for (int r = 0; r < MS; ++r) {
          const double x = a + (b - a) * (double)(r + 1) / (double)(MS + 1);
          if (cnt[MS * j + r] <= idx) na = x;  // eigenvalue idx is at or above x
          else { nb = x; break; }
        }
        brk[2 * j] = na;
        brk[2 * j + 1] = nb;
      }
      __syncthreads();
    }
    if (act && q == 0) lam[j] = 0.5 * (brk[2 * j] + brk[2 * j + 1]);
    __syncthreads();
  }

  // 3. eigenvectors of T by inverse iteration, thread j for eigenvector j
  const double tiny = eps * fmax(tnorm, pivmin);
  for (int j = tid; j < K; j += blockDim.x) {
    double lj = lam[j];
    // separate (numerically) equal eigenvalues so the factorisations differ
    for (int i = 0; i < j; ++i)
      if (fabs(lam[i] - lj) < 10.0 * eps * fmax(tnorm, 1e-300)) lj -= 10.0 * eps * fmax(tnorm, 1e-300);
    double* u0 = lu + (int64_t)j * 3 * n;
    double* u1 = u0 + n;
    double* u2 = u1 + n;
    double* z = Z + (int64_t)j * n;
    for (int i = 0; i < n; ++i) z[i] = start_entry(j, i);
    for (int it = 0; it < 3; ++it) {
      // LU of T - lj I with partial pivoting, applied to z as it is formed, then back substitution
      double a0 = d[0] - lj, a1 = n > 1 ? e[0] : 0.0, a2 = 0.0;
      for (int i = 0; i < n - 1; ++i) {
        const double c = e[i], nd = d[i + 1] - lj, ns = i + 1 < n - 1 ? e[i + 1] : 0.0;
        if (fabs(c) > fabs(a0)) {
          u0[i] = c; u1[i] = nd; u2[i] = ns;
          const double mlt = a0 / c;
          const double t0 = z[i];
          z[i] = z[i + 1];
          z[i + 1] = t0 - mlt * z[i + 1];
          a0 = a1 - mlt * nd;
          a1 = a2 - mlt * ns;
          a2 = 0.0;
        } else {
          if (a0 == 0.0) a0 = tiny;
          u0[i] = a0; u1[i] = a1; u2[i] = a2;
          const double mlt = c / a0;
          z[i + 1] -= mlt * z[i];
          a0 = nd - mlt * a1;
          a1 = ns - mlt * a2;
          a2 = 0.0;
        }
      }
      if (a0 == 0.0) a0 = tiny;
      u0[n - 1] = a0; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        if (i + 1 < n) s -= u1[i] * z[i + 1];
        if (i + 2 < n) s -= u2[i] * z[i + 2];
        z[i] = s / u0[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += z[i] * z[i];
      nrm = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = 0; i < n; ++i) z[i] *= nrm;
    }
  }
  __syncthreads();
  orth_rows(Z, K, n, gm, lu, red, oflag);

  // 4. back-transformation, one wave per vector
  const int wave = tid >> 6, lane = tid & 63;
  for (int j = wave; j < K; j += blockDim.x >> 6) {
    double* z = Z + (int64_t)j * n;
    for (int k = n - 3; k >= 0; --k) {
      const double t = tau[k];
      if (t == 0.0) continue;
      const int m = n - k - 1;
      double s = 0.0;
      for (int i = lane; i < m; i += 64) s += A[(int64_t)(k + 1 + i) * stride + k] * z[k + 1 + i];
      s = wave_sum(s);
      for (int i = lane; i < m; i += 64) z[k + 1 + i] -= t * s * A[(int64_t)(k + 1 + i) * stride + k];
    }
  }
  __syncthreads();
  orth_rows(Z, K, n, gm, lu, red, oflag);   // restore orthonormality after back-transformation
  for (int64_t t = tid; t < (int64_t)n * K; t += blockDim.x) {
    const int i = (int)(t / K), j = (int)(t % K);
    VK[(int64_t)i * Kout + j] = Z[(int64_t)j * n + i];
  }
  for (int j = tid; j < K; j += blockDim.x) lam_out[j] = lam[j];
}

// Leading K eigenpairs of G (n0 x n0, FP64): lam_k[0..K) descending and VK (n0 x K).
// Eigenpairs beyond n0 (K > n0) are reported as zero eigenvalues.
void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK) {
  const int Ke = K < n0 ? K : n0;
  const EigLayout with_a = eig_layout(n0, Ke, true), no_a = eig_layout(n0, Ke, false);
  const size_t lim = c->lds_per_block;
  int a_in_lds = 0, ws_in_lds = 0;
  size_t lds = 0;
  if ((size_t)with_a.total * 8 <= lim) {
    a_in_lds = 1;
    ws_in_lds = 1;
    lds = (size_t)with_a.total * 8;
  } else if ((size_t)no_a.total * 8 <= lim) {
    ws_in_lds = 1;
    lds = (size_t)no_a.total * 8;
  }
  ensure(c, c->work, sizeof(double) * (size_t)(with_a.total + 16));
  if (K > Ke) TK_HIP(hipMemsetAsync(lam_k, 0, sizeof(double) * K, c->stream));
  hipLaunchKernelGGL(k_syev_topk, dim3(1), dim3(EIG_THREADS), lds, c->stream, G, n0, Ke, K, a_in_lds, ws_in_lds,
                     c->work.as<double>(), lam_k, VK);
  TK_CHECK_LAUNCH();
}

}  // namespace tk
