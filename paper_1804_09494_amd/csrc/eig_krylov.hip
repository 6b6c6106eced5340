// Leading K eigenpairs of a large Gram matrix G = Y^T Y (Khat above what one
// workgroup holds), the SVD step of an HOOI invocation (Section 2.2) for wide
// penultimate matrices.  The paper queries Y through a Lanczos method
// (Section 3, "SVD Component"); here the Krylov method runs on G itself, in
// blocks, with everything in FP64:
//   Q_0 = orthonormal start block (the previous invocation's eigenvectors of
//         this mode when there are any, seeded directions otherwise);
//   for j < KR_S:  GQ_j = G Q_j;  W = GQ_j - Q_{0..j} (Q_{0..j}^T GQ_j), twice
//         (full re-orthogonalisation);  Q_{j+1} = W R^-1 by shifted
//         CholeskyQR3 (the first pass on the shifted Gram; an exactly zero
//         block is zeroed);
//   Rayleigh-Ritz: H = Q^T (G Q)  (KR_S*KR_B square), its leading K eigenpairs by
//         the dense solver, V = Q S;
//   the largest residual ||G v - theta v|| / theta_1 decides a restart from V
//   (up to KR_CYCLES cycles, ending early once a restart stops improving it);
//   the cycle with the smallest residual is kept.  Its subspace error is
//   bounded through the sin-theta theorem (Davis-Kahan) by
//   sqrt(2) * residual * theta_1 / (theta_K - theta_{K+1}); above the
//   context's eig_tol the dense solver is run on G instead.
// The tall-skinny products are plain FP64 kernels with fixed-order partial sums.
#include <cmath>

#include "common.hpp"

namespace tk {

void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK, int mode);
void eig_topk_dense(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK);

constexpr int KR_B = 16;    // block width
constexpr int KR_S = 6;     // blocks per cycle (subspace KR_S * KR_B = 96: the dense solver's LDS path)
constexpr int KR_M = KR_B * KR_S;
constexpr int KR_CYCLES = 4;
constexpr int KR_TN_WAVES = 16;   // waves splitting the rows of one A^T B tile

typedef double doublex4_k __attribute__((ext_vector_type(4)));

// The tall-skinny products run on the FP64 matrix cores (v_mfma_f64_16x16x4_f64:
// lane l supplies A[i = l%16][k = l/16] and B[k = l/16][j = l%16]; register r
// of the result holds D[l/16 + 4r][l%16]).  The k range is split over the
// waves of a workgroup and their tiles are summed in LDS in wave order, so
// every result is deterministic.

// D (n x nc, ldd) = A (n x J, lda) C (J x nc, ldc), or D = S - A C when SUB
// (S may be D itself); nc <= 16.  One workgroup per 16-row block, whose NW
// waves take consecutive parts of the k range.
template <bool SUB, int NW>
__global__ __launch_bounds__(NW * 64) void k_kr_nn(const double* __restrict__ A, int lda, int J,
                                                  const double* __restrict__ C, int ldc, const double* S, int lds,
                                                  double* D, int ldd, int n, int nc) {
  __shared__ double red[NW * 256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  const int r0 = blockIdx.x * 16;
  const int row = r0 + i16;
  const int Jw = ((J + 4 * NW - 1) / (4 * NW)) * 4;   // k per wave, a multiple of 4
  const int k0 = wave * Jw, k1 = min(k0 + Jw, J);
  doublex4_k acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int k = k0; k < k1; k += 4) {
    const int kk = k + q;
    const double a = (row < n && kk < k1) ? A[(int64_t)row * lda + kk] : 0.0;
    const double b = (kk < k1 && i16 < nc) ? C[(int64_t)kk * ldc + i16] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // the waves' partials, summed by wave 0 in wave order
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + r * 64 + lane] = acc[r];
  __syncthreads();
  if (wave == 0 && i16 < nc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += red[w * 256 + r * 64 + lane];
      const int rr = r0 + q + 4 * r;
      if (rr < n) D[(int64_t)rr * ldd + i16] = SUB ? S[(int64_t)rr * lds + i16] - t : t;
    }
  }
}

// out (J x nc, row-major) = A^T B over n rows (A: n x J, lda; B: n x nc, ldb).
// One workgroup per 16 x 16 output tile (blockIdx.x: rows of out, blockIdx.y: columns);
// its sixteen waves take consecutive row ranges, so the chain of dependent
// matrix-core steps per wave is short (a handful of tiles fill few CUs).
__global__ __launch_bounds__(KR_TN_WAVES * 64) void k_kr_tn(const double* __restrict__ A, int lda, int J,
                                                           const double* __restrict__ B, int ldb, int nc, int n,
                                                           double* __restrict__ out) {
  __shared__ double red[KR_TN_WAVES * 256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
  const int nw = ((n + 4 * KR_TN_WAVES - 1) / (4 * KR_TN_WAVES)) * 4;   // rows per wave, a multiple of 4
  const int s0 = wave * nw, s1 = min(s0 + nw, n);
  const bool aok = i0 + i16 < J, bok = c0 + i16 < nc;
  doublex4_k acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int r = s0; r < s1; r += 4) {
    const int rr = r + q;
    const bool rok = rr < s1;
    const double a = (rok && aok) ? A[(int64_t)rr * lda + i0 + i16] : 0.0;
    const double b = (rok && bok) ? B[(int64_t)rr * ldb + c0 + i16] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // the waves' partials, summed by wave 0 in wave order
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + r * 64 + lane] = acc[r];
  __syncthreads();
  if (wave == 0 && bok) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double t = 0.0;
      for (int w = 0; w < KR_TN_WAVES; ++w) t += red[w * 256 + r * 64 + lane];
      const int ii = i0 + q + 4 * r;
      if (ii < J) out[(int64_t)ii * nc + c0 + i16] = t;
    }
  }
}

// Cholesky of the b x b Gram A = R^T R (b <= 16) and Rinv = R^-1, one wave.
// shift_rows > 0: the shifted form for the first of the three CholeskyQR
// passes (Fukaya et al., shifted CholeskyQR3): A + s I with
// s = 11 (m b + b (b + 1)) u tr(A), m = shift_rows, u = 2^-53, which is safely
// positive definite whatever the condition of the block, so a block whose
// directions are nearly spanned already still yields its remaining (tiny or
// noise) directions, normalised by the next two passes.  Without the shift a
// restart from converged vectors fails the pivot test on every later block
// and the Krylov space stops growing.  A column whose pivot is not safely
// positive in a later pass (a direction at rounding level) is dropped alone:
// its row of R is set to e_j and its column of Rinv to zero, so it adds
// nothing to the other columns and comes out zero.  An all-zero block zeroes
// Rinv.
// x of lane l (l wave-uniform)
__device__ __forceinline__ double kr_lane(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(v & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Lane k keeps column k of the block in registers (x[i] = A[i][k], then
// R[i][k] in the upper triangle); an entry of another column is read across
// lanes, so the factorisation and the inverse need no LDS and no barrier.
__global__ __launch_bounds__(64) void k_kr_chol(const double* __restrict__ A, int b, double* __restrict__ Rinv,
                                               int shift_rows) {
  const int l = threadIdx.x;
  double x[KR_B];
#pragma unroll
  for (int i = 0; i < KR_B; ++i) x[i] = (i < b && l < b) ? A[i * b + l] : 0.0;
  if (shift_rows > 0) {
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < KR_B; ++i)
      if (i < b) tr += kr_lane(x[i], i);
    const double sh = 11.0 * ((double)shift_rows * b + (double)b * (b + 1)) * 0x1p-53 * tr;
#pragma unroll
    for (int i = 0; i < KR_B; ++i)
      if (i == l && l < b) x[i] += sh;
  }
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < KR_B; ++i)
    if (i < b) dmax = fmax(dmax, kr_lane(x[i], i));
  if (!(dmax > 0.0)) {
    for (int i = l; i < b * b; i += 64) Rinv[i] = 0.0;
    return;
  }
  // R in the upper triangle, row j: R[j][j..b-1] (lane k holds R[j][k] in x[j])
  int dead = 0;
#pragma unroll
  for (int j = 0; j < KR_B; ++j) {
    if (j < b) {
      const double d = kr_lane(x[j], j);
      if (!(d > 1e-14 * dmax)) {   // dependent column: dropped
        dead |= 1 << j;
        if (l == j) x[j] = 1.0;
        if (l > j && l < b) x[j] = 0.0;
      } else {
        const double rjj = sqrt(d), ri = 1.0 / rjj;
        if (l > j && l < b) x[j] *= ri;
        if (l == j) x[j] = rjj;
        // trailing update A[i][k] -= R[j][i] R[j][k], j < i <= k
#pragma unroll
        for (int i = j + 1; i < KR_B; ++i) {
          if (i < b) {
            const double rji = kr_lane(x[j], i);
            if (l >= i && l < b) x[i] -= rji * x[j];
          }
        }
      }
    }
  }
  // column c = l of R^-1 by back substitution; x[k] = 0 for k > c leaves the
  // sums as they are
  double y[KR_B];
#pragma unroll
  for (int i = 0; i < KR_B; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = KR_B - 1; i >= 0; --i) {
    if (i < b) {
      double s = 0.0;   // minus the sum
#pragma unroll
      for (int k = i + 1; k < KR_B; ++k)
        if (k < b) s -= kr_lane(x[i], k) * y[k];
      const double rii = kr_lane(x[i], i);
      y[i] = i == l ? 1.0 / rii : (i < l ? s / rii : 0.0);
    }
  }
  if (l < b) {
    const bool dc = (dead >> l) & 1;
#pragma unroll
    for (int i = 0; i < KR_B; ++i)
      if (i < b) Rinv[i * b + l] = dc ? 0.0 : y[i];
  }
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
  double *Q, *GQ, *W, *W2, *small, *H, *lamH, *S, *GV, *res, *bestV, *bestLam;
};

unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }
unsigned g16(int64_t n) { return (unsigned)((n + 15) / 16); }

// out (J x nc) = A^T B over n rows
void tn(Ctx* c, const double* A, int lda, int J, const double* B, int ldb, int nc, int n, double* out) {
  hipLaunchKernelGGL(k_kr_tn, dim3(g16(J), g16(nc)), dim3(KR_TN_WAVES * 64), 0, c->stream, A, lda, J, B, ldb, nc, n,
                     out);
  TK_CHECK_LAUNCH();
}

// D = A C (SUB: D = S - A C); nc <= 16
template <bool SUB>
void nn(Ctx* c, const double* A, int lda, int J, const double* C, int ldc, const double* S, int lds, double* D,
        int ldd, int n, int nc) {
  // a long k range (G Q) goes over sixteen waves, so each wave's chain of dependent steps is short
  if (J >= 256)
    hipLaunchKernelGGL((k_kr_nn<SUB, 16>), dim3(g16(n)), dim3(16 * 64), 0, c->stream, A, lda, J, C, ldc, S, lds, D, ldd,
                       n, nc);
  else
    hipLaunchKernelGGL((k_kr_nn<SUB, 4>), dim3(g16(n)), dim3(4 * 64), 0, c->stream, A, lda, J, C, ldc, S, lds, D, ldd,
                       n, nc);
  TK_CHECK_LAUNCH();
}

// Q[:, q0:q0+B] = orthonormal basis of W (three CholeskyQR passes, W and W2
// alternating, the last one written into Q)
void cholqr(Ctx* c, const KrBufs& b, int n, int q0) {
  double* A = b.small;              // B x B Gram
  double* Ri = b.small + KR_B * KR_B;
  double* src = b.W;
  for (int pass = 0; pass < 3; ++pass) {
    tn(c, src, KR_B, KR_B, src, KR_B, KR_B, n, A);
    hipLaunchKernelGGL(k_kr_chol, dim3(1), dim3(64), 0, c->stream, A, KR_B, Ri, pass == 0 ? n : 0);
    TK_CHECK_LAUNCH();
    double* dst = pass == 2 ? b.Q + q0 : (src == b.W ? b.W2 : b.W);
    nn<false>(c, src, KR_B, KR_B, Ri, KR_B, nullptr, 0, dst, pass == 2 ? KR_M : KR_B, n, KR_B);
    src = dst;
  }
}
}  // namespace

// Leading K (<= KR_B) eigenpairs of G (n x n FP64): lam_k descending, VK (n x Kout).
// mode >= 0 keeps the eigenvectors for that mode's next call.
void eig_topk_krylov(Ctx* c, const double* G, int n, int K, int Kout, double* lam_k, double* VK, int mode) {
  TK_REQUIRE(K <= KR_B, TK_ERR_UNSUPPORTED, "Krylov eigensolve: more than 16 eigenpairs");
  // the Rayleigh-Ritz step also yields theta_{K+1}, the gap estimate
  const int Kr = K + 1;
  KrBufs b{};
  const size_t nQ = (size_t)n * KR_M;
  const size_t need = 2 * nQ + 2 * (size_t)n * KR_B + 4 * KR_B * KR_B + KR_M * KR_M + 64 +
                      (size_t)KR_M * (KR_B + 1) + (size_t)n * KR_B + 8 + (size_t)n * KR_B + KR_B;
  ensure(c, c->kr_work, sizeof(double) * need);
  double* p = c->kr_work.as<double>();
  b.Q = p; p += nQ;
  b.GQ = p; p += nQ;
  b.W = p; p += (size_t)n * KR_B;
  b.W2 = p; p += (size_t)n * KR_B;
  b.small = p; p += 4 * KR_B * KR_B;
  b.H = p; p += KR_M * KR_M;
  b.lamH = p; p += 64;
  b.S = p; p += (size_t)KR_M * (KR_B + 1);
  b.GV = p; p += (size_t)n * KR_B;
  b.res = p; p += 8;
  b.bestV = p; p += (size_t)n * KR_B;
  b.bestLam = p;
  Buf* warm = mode >= 0 ? &c->eig_warm[mode] : nullptr;
  int kw = (warm && c->eig_warm_k[mode] == K && warm->bytes() >= sizeof(double) * (size_t)n * K) ? K : 0;
  double prev_res = 0.0, best_res = 0.0, best_err = 0.0;
  int best_cycle = -1, last_cycle = -1;
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
      nn<false>(c, G, n, n, b.Q + q0, KR_M, nullptr, 0, b.GQ + q0, KR_M, n, KR_B);
      if (j == KR_S - 1) break;
      // W = GQ_j - Q_{0..j} (Q_{0..j}^T GQ_j), then once more on W (full re-orthogonalisation)
      for (int rep = 0; rep < 2; ++rep) {
        double* Cm = b.H;   // J x B coefficients; H is free until the Rayleigh-Ritz step
        const double* src = rep == 0 ? b.GQ + q0 : b.W;
        const int ls = rep == 0 ? KR_M : KR_B;
        tn(c, b.Q, KR_M, J, src, ls, KR_B, n, Cm);
        nn<true>(c, b.Q, KR_M, J, Cm, KR_B, src, ls, b.W, KR_B, n, KR_B);
      }
      cholqr(c, b, n, J);
    }
    // Rayleigh-Ritz on span(Q): K + 1 Ritz pairs, the first K kept
    tn(c, b.Q, KR_M, KR_M, b.GQ, KR_M, KR_M, n, b.H);
    eig_topk(c, b.H, KR_M, Kr, b.lamH, b.S, -1);
    nn<false>(c, b.Q, KR_M, KR_M, b.S, Kr, nullptr, 0, VK, Kout, n, K);
    TK_HIP(hipMemcpyAsync(lam_k, b.lamH, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
    // residual check
    nn<false>(c, G, n, n, VK, Kout, nullptr, 0, b.GV, K, n, K);
    hipLaunchKernelGGL(k_kr_resid, dim3(1), dim3(256), 0, c->stream, b.GV, VK, Kout, lam_k, n, K, b.res);
    TK_CHECK_LAUNCH();
    double hres[3] = {0.0, 0.0, 0.0};   // residual / theta_1, theta_1, theta_{K+1}
    TK_HIP(hipMemcpyAsync(&hres[0], b.res, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    TK_HIP(hipMemcpyAsync(&hres[1], b.lamH, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    double thK[2] = {0.0, 0.0};
    TK_HIP(hipMemcpyAsync(thK, b.lamH + K - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    const double res = hres[0];
    const double gap = thK[0] - thK[1];
    // estimated projector distance of the Ritz subspace from the eigenspace
    const double err = hres[1] > 0.0 ? (gap > 0.0 ? std::sqrt(2.0) * res * hres[1] / gap : HUGE_VAL) : 0.0;
    last_cycle = cycle;
    ++c->counters.eig_krylov_cycles;
    if (best_cycle < 0 || res < best_res) {
      best_res = res;
      best_err = err;
      best_cycle = cycle;
      TK_HIP(hipMemcpy2DAsync(b.bestV, sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K, n,
                              hipMemcpyDeviceToDevice, c->stream));
      TK_HIP(hipMemcpyAsync(b.bestLam, lam_k, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
    }
    // converged, or a restart that no longer improves (rounding floor)
    if ((res <= 1e-10 && err <= c->eig_tol()) || (cycle > 0 && res > 0.5 * prev_res)) break;
    prev_res = res;
  }
  ++c->counters.eig_krylov_solves;
  if (best_cycle != last_cycle) {
    TK_HIP(hipMemcpy2DAsync(VK, sizeof(double) * Kout, b.bestV, sizeof(double) * K, sizeof(double) * K, n,
                            hipMemcpyDeviceToDevice, c->stream));
    TK_HIP(hipMemcpyAsync(lam_k, b.bestLam, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
  }
  if (!(best_err <= c->eig_tol())) {
    // the Krylov subspace is not accurate enough (slow convergence or a tight
    // gap at K): the dense solver on G
    ++c->counters.eig_dense_fallbacks;
    eig_topk_dense(c, G, n, Kout, lam_k, VK);
  }
  if (warm) {
    ensure(c, *warm, sizeof(double) * (size_t)n * K);
    TK_HIP(hipMemcpy2DAsync(warm->as<double>(), sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K,
                            n, hipMemcpyDeviceToDevice, c->stream));
    c->eig_warm_k[mode] = K;
  }
}

}  // namespace tk
