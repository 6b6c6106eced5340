// Leading K eigenpairs of a large Gram matrix G = Y^T Y (Khat above what one
// workgroup holds), the SVD step of an HOOI invocation (Section 2.2) for wide
// penultimate matrices.  The paper queries Y through a Lanczos method
// (Section 3, "SVD Component"); here the Krylov method runs on G itself, in
// blocks, with everything in FP64:
//   Q_0 = orthonormal start block (the previous invocation's eigenvectors of
//         this mode when there are any, seeded directions otherwise);
//   for j < KR_S:  GQ_j = G Q_j;  W = GQ_j - Q_{0..j} (Q_{0..j}^T GQ_j), twice
//         (full re-orthogonalisation);  Q_{j+1} = W R^-1 by CholeskyQR, three
//         passes (a block that has no independent directions left is zeroed);
//   Rayleigh-Ritz: H = Q^T (G Q)  (KR_S*KR_B square), its leading K eigenpairs by
//         the dense solver, V = Q S;
//   the largest residual ||G v - theta v|| / theta_1 decides a restart from V.
// The tall-skinny products are plain FP64 kernels with fixed-order partial sums.
#include <cmath>

#include "common.hpp"

namespace tk {

void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK, int mode);

constexpr int KR_B = 16;    // block width
constexpr int KR_S = 6;     // blocks per cycle (subspace KR_S * KR_B = 96: the dense solver's LDS path)
constexpr int KR_M = KR_B * KR_S;
constexpr int KR_CYCLES = 4;

// D[r][c] (=, or -= when SUB) sum_{i<J} A[r*lda + i] * C[i*ldc + c], c < nc
template <bool SUB>
__global__ __launch_bounds__(256) void k_kr_nn(const double* __restrict__ A, int lda, int J,
                                               const double* __restrict__ C, int ldc, double* __restrict__ D,
                                               int ldd, int n, int nc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * nc) return;
  const int r = (int)(idx / nc), cc = (int)(idx - (int64_t)r * nc);
  const double* a = A + (int64_t)r * lda;
  double s = 0.0;
  for (int i = 0; i < J; ++i) s += a[i] * C[(int64_t)i * ldc + cc];
  double* d = D + (int64_t)r * ldd + cc;
  *d = SUB ? *d - s : s;
}

// part[wg][i*nc + c] = sum over the workgroup's rows of A[r*lda + i] * B[r*ldb + c]
__global__ __launch_bounds__(256) void k_kr_tn(const double* __restrict__ A, int lda, int J,
                                               const double* __restrict__ B, int ldb, int nc, int n, int rows_per_wg,
                                               double* __restrict__ part) {
  const int r0 = blockIdx.x * rows_per_wg, r1 = min(r0 + rows_per_wg, n);
  const int nout = J * nc;
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    const int i = o / nc, cc = o - i * nc;
    double s = 0.0;
    for (int r = r0; r < r1; ++r) s += A[(int64_t)r * lda + i] * B[(int64_t)r * ldb + cc];
    part[(int64_t)blockIdx.x * nout + o] = s;
  }
}

__global__ void k_kr_sum(const double* __restrict__ part, int nparts, int cnt, double* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= cnt) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * cnt + o];
  out[o] = s;
}

// Cholesky of the b x b Gram A = R^T R and Rinv = R^-1; a pivot that is not
// safely positive (no independent direction left) zeroes Rinv, and so the block.
__global__ void k_kr_chol(const double* __restrict__ A, int b, double* __restrict__ Rinv) {
  __shared__ double R[KR_B * KR_B], Ri[KR_B * KR_B];
  if (threadIdx.x != 0) return;
  double dmax = 0.0;
  for (int i = 0; i < b; ++i) dmax = fmax(dmax, A[i * b + i]);
  bool ok = dmax > 0.0;
  for (int i = 0; i < b * b; ++i) R[i] = 0.0;
  for (int j = 0; j < b && ok; ++j) {
    double d = A[j * b + j];
    for (int k = 0; k < j; ++k) d -= R[k * b + j] * R[k * b + j];
    if (!(d > 1e-14 * dmax)) { ok = false; break; }
    const double rjj = sqrt(d);
    R[j * b + j] = rjj;
    for (int i = j + 1; i < b; ++i) {
      double s = A[j * b + i];
      for (int k = 0; k < j; ++k) s -= R[k * b + j] * R[k * b + i];
      R[j * b + i] = s / rjj;
    }
  }
  for (int i = 0; i < b * b; ++i) Ri[i] = 0.0;
  if (ok) {
    for (int j = 0; j < b; ++j) {
      Ri[j * b + j] = 1.0 / R[j * b + j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += R[i * b + k] * Ri[k * b + j];
        Ri[i * b + j] = -s / R[i * b + i];
      }
    }
  }
  for (int i = 0; i < b * b; ++i) Rinv[i] = Ri[i];
}

// Start block: columns 0..kw-1 from the warm vectors (n x kw, row-major), the
// rest seeded directions (SplitMix64 of (column, row), uniform in [-1, 1)).
__global__ void k_kr_start(const double* __restrict__ warm, int kw, int n, double* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * KR_B) return;
  const int r = (int)(idx / KR_B), cc = (int)(idx % KR_B);
  if (cc < kw) {
    W[idx] = warm[(int64_t)r * kw + cc];
  } else {
    unsigned long long z = 0x9E3779B97F4A7C15ULL * (unsigned long long)((cc + 1) * 2654435761u + r + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    W[idx] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// max_k ||GV[:,k] - lam_k V[:,k]|| / lam_0, one workgroup
__global__ __launch_bounds__(256) void k_kr_resid(const double* __restrict__ GV, const double* __restrict__ V, int ldv,
                                                  const double* __restrict__ lam, int n, int K,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double worst = 0.0;
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const double d = GV[(int64_t)r * K + k] - lam[k] * V[(int64_t)r * ldv + k];
      s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    worst = fmax(worst, sqrt(red[0]));
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = lam[0] > 0.0 ? worst / lam[0] : 0.0;
}

namespace {
struct KrBufs {
  double *Q, *GQ, *W, *part, *small, *H, *lamH, *S, *GV, *res;
  int nwg, rows_per_wg;
};

unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

// out (J x nc) = A^T B over n rows
void tn(Ctx* c, const KrBufs& b, const double* A, int lda, int J, const double* B, int ldb, int nc, int n,
        double* out) {
  hipLaunchKernelGGL(k_kr_tn, dim3(b.nwg), dim3(256), 0, c->stream, A, lda, J, B, ldb, nc, n, b.rows_per_wg, b.part);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_kr_sum, dim3(g1((int64_t)J * nc)), dim3(256), 0, c->stream, b.part, b.nwg, J * nc, out);
  TK_CHECK_LAUNCH();
}

// Q[:, q0:q0+B] = orthonormal basis of W (three CholeskyQR passes in place, then copied)
void cholqr(Ctx* c, const KrBufs& b, int n, int q0) {
  double* A = b.small;              // B x B Gram
  double* Ri = b.small + KR_B * KR_B;
  for (int pass = 0; pass < 3; ++pass) {
    tn(c, b, b.W, KR_B, KR_B, b.W, KR_B, KR_B, n, A);
    hipLaunchKernelGGL(k_kr_chol, dim3(1), dim3(64), 0, c->stream, A, KR_B, Ri);
    TK_CHECK_LAUNCH();
    double* dst = pass == 2 ? b.Q + q0 : b.GV;   // GV doubles as scratch here
    const int ldd = pass == 2 ? KR_M : KR_B;
    hipLaunchKernelGGL(k_kr_nn<false>, dim3(g1((int64_t)n * KR_B)), dim3(256), 0, c->stream, b.W, KR_B, KR_B, Ri,
                       KR_B, dst, ldd, n, KR_B);
    TK_CHECK_LAUNCH();
    if (pass < 2) TK_HIP(hipMemcpyAsync(b.W, b.GV, sizeof(double) * (size_t)n * KR_B, hipMemcpyDeviceToDevice,
                                        c->stream));
  }
}
}  // namespace

// Leading K (<= KR_B) eigenpairs of G (n x n FP64): lam_k descending, VK (n x Kout).
// mode >= 0 keeps the eigenvectors for that mode's next call.
void eig_topk_krylov(Ctx* c, const double* G, int n, int K, int Kout, double* lam_k, double* VK, int mode) {
  TK_REQUIRE(K <= KR_B, TK_ERR_UNSUPPORTED, "Krylov eigensolve: more than 16 eigenpairs");
  KrBufs b{};
  b.rows_per_wg = std::max(64, (int)ceil_div(n, 256));
  b.nwg = (int)ceil_div(n, b.rows_per_wg);
  const size_t nQ = (size_t)n * KR_M;
  const size_t need = 2 * nQ + (size_t)n * KR_B + (size_t)b.nwg * KR_M * KR_M + 4 * KR_B * KR_B + KR_M * KR_M +
                      64 + (size_t)KR_M * KR_B + (size_t)n * KR_B + 8;
  ensure(c, c->kr_work, sizeof(double) * need);
  double* p = c->kr_work.as<double>();
  b.Q = p; p += nQ;
  b.GQ = p; p += nQ;
  b.W = p; p += (size_t)n * KR_B;
  b.part = p; p += (size_t)b.nwg * KR_M * KR_M;
  b.small = p; p += 4 * KR_B * KR_B;
  b.H = p; p += KR_M * KR_M;
  b.lamH = p; p += 64;
  b.S = p; p += (size_t)KR_M * KR_B;
  b.GV = p; p += (size_t)n * KR_B;
  b.res = p;
  Buf* warm = mode >= 0 ? &c->eig_warm[mode] : nullptr;
  int kw = (warm && c->eig_warm_k[mode] == K && warm->bytes() >= sizeof(double) * (size_t)n * K) ? K : 0;
  for (int cycle = 0; cycle < KR_CYCLES; ++cycle) {
    // start block: the warm vectors (first cycle) or the last Ritz vectors (restart), then seeded directions
    const double* wsrc = nullptr;
    int kws = 0;
    if (cycle == 0 && kw) {
      wsrc = warm->as<double>();
      kws = kw;
    } else if (cycle > 0) {
      TK_HIP(hipMemcpy2DAsync(b.GV, sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K, n,
                              hipMemcpyDeviceToDevice, c->stream));
      wsrc = b.GV;
      kws = K;
    }
    hipLaunchKernelGGL(k_kr_start, dim3(g1((int64_t)n * KR_B)), dim3(256), 0, c->stream, wsrc, kws, n, b.W);
    TK_CHECK_LAUNCH();
    TK_HIP(hipMemsetAsync(b.Q, 0, sizeof(double) * nQ, c->stream));
    cholqr(c, b, n, 0);
    for (int j = 0; j < KR_S; ++j) {
      const int q0 = j * KR_B, J = q0 + KR_B;
      // GQ_j = G Q_j
      hipLaunchKernelGGL(k_kr_nn<false>, dim3(g1((int64_t)n * KR_B)), dim3(256), 0, c->stream, G, n, n, b.Q + q0,
                         KR_M, b.GQ + q0, KR_M, n, KR_B);
      TK_CHECK_LAUNCH();
      if (j == KR_S - 1) break;
      TK_HIP(hipMemcpy2DAsync(b.W, sizeof(double) * KR_B, b.GQ + q0, sizeof(double) * KR_M,
                              sizeof(double) * KR_B, n, hipMemcpyDeviceToDevice, c->stream));
      for (int rep = 0; rep < 2; ++rep) {
        double* Cm = b.H;   // J x B coefficients; H is free until the Rayleigh-Ritz step
        tn(c, b, b.Q, KR_M, J, b.W, KR_B, KR_B, n, Cm);
        hipLaunchKernelGGL(k_kr_nn<true>, dim3(g1((int64_t)n * KR_B)), dim3(256), 0, c->stream, b.Q, KR_M, J, Cm,
                           KR_B, b.W, KR_B, n, KR_B);
        TK_CHECK_LAUNCH();
      }
      cholqr(c, b, n, J);
    }
    // Rayleigh-Ritz on span(Q)
    tn(c, b, b.Q, KR_M, KR_M, b.GQ, KR_M, KR_M, n, b.H);
    eig_topk(c, b.H, KR_M, K, b.lamH, b.S, -1);
    hipLaunchKernelGGL(k_kr_nn<false>, dim3(g1((int64_t)n * K)), dim3(256), 0, c->stream, b.Q, KR_M, KR_M, b.S, K,
                       VK, Kout, n, K);
    TK_CHECK_LAUNCH();
    TK_HIP(hipMemcpyAsync(lam_k, b.lamH, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
    // residual check
    hipLaunchKernelGGL(k_kr_nn<false>, dim3(g1((int64_t)n * K)), dim3(256), 0, c->stream, G, n, n, VK, Kout, b.GV, K,
                       n, K);
    TK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_kr_resid, dim3(1), dim3(256), 0, c->stream, b.GV, VK, Kout, lam_k, n, K, b.res);
    TK_CHECK_LAUNCH();
    double res = 0.0;
    TK_HIP(hipMemcpyAsync(&res, b.res, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (res <= 1e-10) break;
  }
  if (warm) {
    ensure(c, *warm, sizeof(double) * (size_t)n * K);
    TK_HIP(hipMemcpy2DAsync(warm->as<double>(), sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K,
                            n, hipMemcpyDeviceToDevice, c->stream));
    c->eig_warm_k[mode] = K;
  }
}

}  // namespace tk
