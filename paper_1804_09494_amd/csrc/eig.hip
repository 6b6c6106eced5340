// FP64 symmetric eigensolver for the Gram matrix (Khat x Khat): cyclic
// two-sided Jacobi in one workgroup, parallel over disjoint rotation pairs.
//
// The leading K_n left singular vectors of Y (Section 2.2: the SVD step of an
// HOOI invocation) are Y V_K S_K^-1 for the K_n largest eigenpairs (V, S^2)
// of G = Y^T Y.  Jacobi is used for its high relative accuracy on a small
// dense matrix.  A warm start rotates G into the previous invocation's
// eigenbasis first (A = V0^T G V0, V = V0), which leaves it nearly diagonal
// once HOOI settles.
//
// Parallel ordering: a round-robin tournament over n (even) indices; round r
// pairs (r, n-1) and ((r+k) mod (n-1), (r-k) mod (n-1)) for k = 1..n/2-1, so
// the n/2 pairs of a round are disjoint and n-1 rounds cover every pair once.
// A round computes all rotations from the current diagonal blocks, then
// updates every 2x2 block (pair k1, pair k2) of A as J_k1^T B J_k2, with
// J = [[c, s], [-s, c]] in rows/columns (p, q).  A is kept as a packed upper
// triangle; V (row-major, column j = eigenvector j) is rotated alongside.
#include "common.hpp"

namespace tk {

__device__ __forceinline__ int64_t pk(int i, int j, int n) {
  if (i > j) { int t = i; i = j; j = t; }
  return (int64_t)i * (2 * n - i + 1) / 2 + (j - i);
}

__device__ __forceinline__ void round_pair(int r, int k, int n, int& p, int& q) {
  int a, b;
  if (k == 0) {
    a = r;
    b = n - 1;
  } else {
    a = (r + k) % (n - 1);
    b = (r - k + (n - 1)) % (n - 1);
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// G: n x n FP64 (full), V0: n x n warm start (row-major) or null.
// Outputs: lam[j] (eigenvalues, unsorted), Vout n x n (row-major), sweeps used in info[0].
// Workspace: A (packed) and V in LDS when `lds_mode` bits allow, else in gA/gV.
__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ G, const double* __restrict__ V0, int n0,
                                                 int n, int max_sweeps, double tol, int lds_mode,
                                                 double* __restrict__ gA, double* __restrict__ gV,
                                                 double* __restrict__ lam, double* __restrict__ Vout,
                                                 int* __restrict__ info) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t npk = (int64_t)n * (n + 1) / 2;
  double* cs = sh;                   // c[k], s[k]: 2 * (n/2)
  int* pr = reinterpret_cast<int*>(sh + n);   // p[k], q[k]: n ints (= n/2 doubles)
  double* red = sh + n + (n + 1) / 2;         // 1024 doubles of reduction space
  double* base = red + 1024;
  double* A = (lds_mode & 1) ? base : gA;
  double* V = (lds_mode & 2) ? ((lds_mode & 1) ? base + npk : base) : gV;

  // A = V0^T G V0 (or G), V = V0 (or I); padded index n0..n-1 gets a zero row/column.
  // With a warm start, V first holds T = G V0 (n0 x n0, row-major, stride n).
  if (V0) {
    for (int64_t e = tid; e < (int64_t)n0 * n0; e += nt) {
      const int a = (int)(e / n0), j = (int)(e % n0);
      double t = 0.0;
      for (int b = 0; b < n0; ++b) t += G[(int64_t)a * n0 + b] * V0[(int64_t)b * n0 + j];
      V[(int64_t)a * n + j] = t;
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < npk; e += nt) {
    int i = (int)((2.0 * n + 1 - sqrt((2.0 * n + 1) * (2.0 * n + 1) - 8.0 * (double)e)) / 2);
    while (i > 0 && pk(i, i, n) > e) --i;
    while (i + 1 < n && pk(i + 1, i + 1, n) <= e) ++i;
    const int j = i + (int)(e - pk(i, i, n));
    double s = 0.0;
    if (i < n0 && j < n0) {
      if (V0) {
        for (int a = 0; a < n0; ++a) s += V0[(int64_t)a * n0 + i] * V[(int64_t)a * n + j];
      } else {
        s = G[(int64_t)i * n0 + j];
      }
    }
    A[e] = s;
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
    const int i = (int)(e / n), j = (int)(e % n);
    double v;
    if (i < n0 && j < n0) v = V0 ? V0[(int64_t)i * n0 + j] : (i == j ? 1.0 : 0.0);
    else v = (i == j) ? 1.0 : 0.0;
    V[e] = v;
  }
  __syncthreads();

  const int half = n / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal Frobenius^2 <= tol^2 * diagonal Frobenius^2
    double off = 0.0, dia = 0.0;
    for (int64_t e = tid; e < npk; e += nt) {
      int i = (int)((2.0 * n + 1 - sqrt((2.0 * n + 1) * (2.0 * n + 1) - 8.0 * (double)e)) / 2);
      while (i > 0 && pk(i, i, n) > e) --i;
      while (i + 1 < n && pk(i + 1, i + 1, n) <= e) ++i;
      double x = A[e];
      if (pk(i, i, n) == e) dia += x * x; else off += x * x;
    }
    red[tid] = off;
    if (tid + nt < 1024) red[tid + nt] = 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && tid + w < 1024) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = dia;
    if (tid + nt < 1024) red[tid + nt] = 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && tid + w < 1024) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double dias = red[0];
    __syncthreads();
    if (offs <= tol * tol * dias || offs == 0.0) break;

    for (int r = 0; r < n - 1; ++r) {
      if (tid < half) {
        int p, q;
        round_pair(r, tid, n, p, q);
        const double app = A[pk(p, p, n)], aqq = A[pk(q, q, n)], apq = A[pk(p, q, n)];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double theta = (aqq - app) / (2.0 * apq);
          double t;
          if (fabs(theta) > 1e150) t = 0.5 / theta;
          else t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;
      }
      __syncthreads();
      // 2x2 blocks (k1 <= k2)
      const int nblk = half * (half + 1) / 2;
      for (int b = tid; b < nblk; b += nt) {
        int k1 = (int)((2.0 * half + 1 - sqrt((2.0 * half + 1) * (2.0 * half + 1) - 8.0 * b)) / 2);
        auto start = [&](int k) { return k * (2 * half - k + 1) / 2; };
        while (k1 > 0 && start(k1) > b) --k1;
        while (k1 + 1 < half && start(k1 + 1) <= b) ++k1;
        const int k2 = k1 + (b - start(k1));
        const int p1 = pr[2 * k1], q1 = pr[2 * k1 + 1];
        const double c1 = cs[2 * k1], s1 = cs[2 * k1 + 1];
        if (k1 == k2) {
          const int64_t ipp = pk(p1, p1, n), iqq = pk(q1, q1, n), ipq = pk(p1, q1, n);
          const double app = A[ipp], aqq = A[iqq], apq = A[ipq];
          A[ipp] = c1 * c1 * app - 2.0 * c1 * s1 * apq + s1 * s1 * aqq;
          A[iqq] = s1 * s1 * app + 2.0 * c1 * s1 * apq + c1 * c1 * aqq;
          A[ipq] = 0.0;
        } else {
          const int p2 = pr[2 * k2], q2 = pr[2 * k2 + 1];
          const double c2 = cs[2 * k2], s2 = cs[2 * k2 + 1];
          const int64_t i11 = pk(p1, p2, n), i12 = pk(p1, q2, n), i21 = pk(q1, p2, n), i22 = pk(q1, q2, n);
          const double x11 = A[i11], x12 = A[i12], x21 = A[i21], x22 = A[i22];
          const double y11 = c1 * x11 - s1 * x21, y12 = c1 * x12 - s1 * x22;
          const double y21 = s1 * x11 + c1 * x21, y22 = s1 * x12 + c1 * x22;
          A[i11] = c2 * y11 - s2 * y12;
          A[i12] = s2 * y11 + c2 * y12;
          A[i21] = c2 * y21 - s2 * y22;
          A[i22] = s2 * y21 + c2 * y22;
        }
      }
      // V <- V J
      for (int e = tid; e < n * half; e += nt) {
        const int i = e / half, k = e - i * half;
        const int p = pr[2 * k], q = pr[2 * k + 1];
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double vp = V[(int64_t)i * n + p], vq = V[(int64_t)i * n + q];
        V[(int64_t)i * n + p] = c * vp - s * vq;
        V[(int64_t)i * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < n; j += nt) lam[j] = A[pk(j, j, n)];
  for (int64_t e = tid; e < (int64_t)n * n; e += nt) Vout[e] = V[e];
  if (tid == 0) info[0] = sweep;
}

// Order eigenpairs by eigenvalue, largest first (ties: lower index first), over
// the first n0 indices (padding excluded); write the leading K values and
// vectors: lam_k[k], VK[i * K + k] (n0 x K), and the full sorted basis Vs (n0 x n0)
// for the next warm start.
__global__ void k_eig_select(const double* __restrict__ lam, const double* __restrict__ V, int n0, int n, int K,
                             double* __restrict__ lam_k, double* __restrict__ VK, double* __restrict__ Vs) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += gridDim.x * blockDim.x) {
    const double li = lam[i];
    int rank = 0;
    for (int j = 0; j < n0; ++j) {
      const double lj = lam[j];
      rank += (lj > li) || (lj == li && j < i);
    }
    if (rank < K) lam_k[rank] = li;
    for (int r = 0; r < n0; ++r) {
      const double v = V[(int64_t)r * n + i];
      if (rank < K) VK[(int64_t)r * K + rank] = v;
      Vs[(int64_t)r * n0 + rank] = v;
    }
  }
}

// Eigen-decomposition of G (n0 x n0) -> leading K eigenpairs; warm start from
// and update of Vwarm (n0 x n0, may be null on the first call: then *have_warm = false).
void eig_topk(Ctx* c, const double* G, int n0, int K, double* Vwarm, bool have_warm, double* lam_k, double* VK,
              int* info_dev) {
  const int n = n0 + (n0 & 1);
  const int64_t npk = (int64_t)n * (n + 1) / 2;
  const size_t head = sizeof(double) * ((size_t)n + (size_t)(n + 1) / 2 + 1024);
  const size_t bA = sizeof(double) * (size_t)npk, bV = sizeof(double) * (size_t)n * n;
  const size_t lim = c->lds_per_block;
  int mode = 0;
  size_t lds = head;
  if (head + bA + bV <= lim) { mode = 3; lds = head + bA + bV; }
  else if (head + bA <= lim) { mode = 1; lds = head + bA; }
  ensure(c, c->work, (bA + bV + sizeof(double) * ((size_t)n * n + n)) );
  double* gA = c->work.as<double>();
  double* gV = gA + npk;
  double* lam = gV + (size_t)n * n;
  double* Vout = lam + n;
  const int threads = 1024;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(threads), lds, c->stream, G, have_warm ? Vwarm : nullptr, n0, n,
                     c->opt.max_jacobi_sweeps > 0 ? c->opt.max_jacobi_sweeps : 30,
                     c->opt.eig_tol > 0 ? c->opt.eig_tol : 1e-15, mode, gA, gV, lam, Vout, info_dev);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_eig_select, dim3((n0 + 255) / 256), dim3(256), 0, c->stream, lam, Vout, n0, n, K, lam_k, VK,
                     Vwarm);
  TK_CHECK_LAUNCH();
}

}  // namespace tk
