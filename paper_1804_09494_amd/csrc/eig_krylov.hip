// Leading K eigenpairs of Y^T Y for a wide penultimate matrix Y (Khat above
// what one workgroup holds), the SVD step of an HOOI invocation (Section 2.2).
// The paper queries Y through a Lanczos method (Section 3, "SVD Component").
// Two operators feed the same block Krylov method:
//   * the Gram G = Y^T Y, formed beforehand (Khat x Khat): X -> G X;
//   * matrix-free, Y itself (R x Khat FP32, never squared): X -> Y^T (Y X),
//     two passes over Y per block, for Khat where G's Khat^2 memory and
//     2 R Khat^2 flops outgrow the passes over Y.
// With everything in FP64:
//   Q_0 = orthonormal start block (the previous invocation's eigenvectors of
//         this mode when there are any, seeded directions otherwise);
//   for j < S:  GQ_j = A Q_j  (A the operator, blocks of B columns);  W = GQ_j - Q_{0..j} (Q_{0..j}^T GQ_j), twice
//         (full re-orthogonalisation);  Q_{j+1} = W R^-1 by shifted
//         CholeskyQR3 (the first pass on the shifted Gram; an exactly zero
//         block is zeroed);
//   Rayleigh-Ritz: H = Q^T (A Q)  (S*B square), its leading K eigenpairs by
//         the dense solver, V = Q S;
//   the largest residual ||A v - theta v|| / theta_1 decides a restart from V
//   (up to 4 cycles with 16-column blocks, 12 with 32-column ones, ending
//   early once a restart stops improving it);
//   the cycle with the smallest residual is kept.  It is accepted once its
//   relative residual is at the rounding level of the FP32 data the operator
//   comes from (4 u): the Ritz vectors are then exact for an operator within
//   that rounding of the given one, as good as the dense solver's on the same
//   data.  A caller's positive eig_tol instead bounds the subspace error
//   estimated through the sin-theta theorem (Davis-Kahan),
//   sqrt(2) * residual * theta_1 / (theta_K - theta_{K+1}).  A rejected
//   result is replaced by the Gram route's (the dense solver on G; for the
//   matrix-free operator, G is formed first).
// B = 16, S = 6 for K <= 16 and B = 32, S = 3 up to K = 31: the subspace is
// 96 columns either way.
// The tall-skinny products are plain FP64 kernels with fixed-order partial sums.
#include <cmath>

#include "common.hpp"

namespace tk {

void eig_topk(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK, int mode);
void eig_topk_dense(Ctx* c, const double* G, int n0, int K, double* lam_k, double* VK);

void gram(Ctx* c, const float* Y, int64_t R, int khat, double* G, bool bf16);

constexpr int KR_M = 96;    // subspace columns per cycle (the dense solver's LDS path)
constexpr int KR_TN_WAVES = 16;   // waves splitting the rows of one A^T B tile

typedef double doublex4_k __attribute__((ext_vector_type(4)));

// The tall-skinny products run on the FP64 matrix cores (v_mfma_f64_16x16x4_f64:
// lane l supplies A[i = l%16][k = l/16] and B[k = l/16][j = l%16]; register r
// of the result holds D[l/16 + 4r][l%16]).  The k range is split over the
// waves of a workgroup and their tiles are summed in LDS in wave order, so
// every result is deterministic.

// D (n x nc, ldd) = A (n x J, lda) C (J x nc, ldc), or D = S - A C when SUB
// (S may be D itself); nc <= 16.  One workgroup per 16-row block, whose NW
// waves take consecutive parts of the k range.  A is FP64 or FP32 (Y, widened
// exactly).
template <bool SUB, int NW, class TA>
__global__ __launch_bounds__(NW * 64) void k_kr_nn(const TA* __restrict__ A, int64_t lda, int J,
                                                  const double* __restrict__ C, int ldc, const double* S, int lds,
                                                  double* D, int ldd, int64_t n, int nc) {
  __shared__ double red[NW * 256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  const int64_t row = r0 + i16;
  const int Jw = ((J + 4 * NW - 1) / (4 * NW)) * 4;   // k per wave, a multiple of 4
  const int k0 = wave * Jw, k1 = min(k0 + Jw, J);
  doublex4_k acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int k = k0; k < k1; k += 4) {
    const int kk = k + q;
    const double a = (row < n && kk < k1) ? (double)A[row * lda + kk] : 0.0;
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
      const int64_t rr = r0 + q + 4 * r;
      if (rr < n) D[rr * ldd + i16] = SUB ? S[rr * lds + i16] - t : t;
    }
  }
}

// part[z] (J x nc, row-major) = A^T B over rows [z*rows, (z+1)*rows) of n
// (A: n x J, lda; B: n x nc, ldb).  One workgroup per 16 x 16 output tile and
// row range (blockIdx.x: rows of out, blockIdx.y: columns, blockIdx.z: row
// range); its sixteen waves take consecutive parts of the range, so the chain
// of dependent matrix-core steps per wave is short.  With one row range, part
// is the product itself.
template <class TA>
__global__ __launch_bounds__(KR_TN_WAVES * 64) void k_kr_tn(const TA* __restrict__ A, int64_t lda, int J,
                                                           const double* __restrict__ B, int ldb, int nc, int64_t n,
                                                           int64_t rows, double* __restrict__ part) {
  __shared__ double red[KR_TN_WAVES * 256];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i16 = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
  const int64_t z0 = (int64_t)blockIdx.z * rows, z1 = min(z0 + rows, n);
  const int64_t nw = ((z1 - z0 + 4 * KR_TN_WAVES - 1) / (4 * KR_TN_WAVES)) * 4;   // rows per wave, a multiple of 4
  const int64_t s0 = z0 + wave * nw, s1 = min(s0 + nw, z1);
  const bool aok = i0 + i16 < J, bok = c0 + i16 < nc;
  doublex4_k acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int64_t r = s0; r < s1; r += 4) {
    const int64_t rr = r + q;
    const bool rok = rr < s1;
    const double a = (rok && aok) ? (double)A[rr * lda + i0 + i16] : 0.0;
    const double b = (rok && bok) ? B[rr * ldb + c0 + i16] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // the waves' partials, summed by wave 0 in wave order
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + r * 64 + lane] = acc[r];
  __syncthreads();
  if (wave == 0 && bok) {
    double* out = part + (int64_t)blockIdx.z * J * nc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double t = 0.0;
      for (int w = 0; w < KR_TN_WAVES; ++w) t += red[w * 256 + r * 64 + lane];
      const int ii = i0 + q + 4 * r;
      if (ii < J) out[(int64_t)ii * nc + c0 + i16] = t;
    }
  }
}

// out[e] = sum over p < nparts of part[p * count + e], in p order
__global__ __launch_bounds__(256) void k_kr_sum_parts(const double* __restrict__ part, int nparts, int64_t count,
                                                      double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
    double t = 0.0;
    for (int p = 0; p < nparts; ++p) t += part[(int64_t)p * count + e];
    out[e] = t;
  }
}

// part[z][k] = sum over rows [z*rows, (z+1)*rows) of Y[r][k]^2 (FP64), the
// diagonal of Y^T Y in pieces
__global__ __launch_bounds__(256) void k_colsq_part(const float* __restrict__ Y, int64_t R, int khat, int64_t rows,
                                                    double* __restrict__ part) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= khat) return;
  const int64_t z0 = (int64_t)blockIdx.y * rows, z1 = min(z0 + rows, R);
  double t = 0.0;
  for (int64_t r = z0; r < z1; ++r) {
    const double y = Y[r * khat + k];
    t += y * y;
  }
  part[(int64_t)blockIdx.y * khat + k] = t;
}

// Cholesky of the b x b Gram A = R^T R (b <= B <= 64) and Rinv = R^-1, one wave.
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
template <int B>
__global__ __launch_bounds__(64) void k_kr_chol(const double* __restrict__ A, int b, double* __restrict__ Rinv,
                                               int shift_rows) {
  const int l = threadIdx.x;
  double x[B];
#pragma unroll
  for (int i = 0; i < B; ++i) x[i] = (i < b && l < b) ? A[i * b + l] : 0.0;
  if (shift_rows > 0) {
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (i < b) tr += kr_lane(x[i], i);
    const double sh = 11.0 * ((double)shift_rows * b + (double)b * (b + 1)) * 0x1p-53 * tr;
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (i == l && l < b) x[i] += sh;
  }
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < B; ++i)
    if (i < b) dmax = fmax(dmax, kr_lane(x[i], i));
  if (!(dmax > 0.0)) {
    for (int i = l; i < b * b; i += 64) Rinv[i] = 0.0;
    return;
  }
  // R in the upper triangle, row j: R[j][j..b-1] (lane k holds R[j][k] in x[j])
  unsigned long long dead = 0;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (j < b) {
      const double d = kr_lane(x[j], j);
      if (!(d > 1e-14 * dmax)) {   // dependent column: dropped
        dead |= 1ull << j;
        if (l == j) x[j] = 1.0;
        if (l > j && l < b) x[j] = 0.0;
      } else {
        const double rjj = sqrt(d), ri = 1.0 / rjj;
        if (l > j && l < b) x[j] *= ri;
        if (l == j) x[j] = rjj;
        // trailing update A[i][k] -= R[j][i] R[j][k], j < i <= k
#pragma unroll
        for (int i = j + 1; i < B; ++i) {
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
  double y[B];
#pragma unroll
  for (int i = 0; i < B; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = B - 1; i >= 0; --i) {
    if (i < b) {
      double s = 0.0;   // minus the sum
#pragma unroll
      for (int k = i + 1; k < B; ++k)
        if (k < b) s -= kr_lane(x[i], k) * y[k];
      const double rii = kr_lane(x[i], i);
      y[i] = i == l ? 1.0 / rii : (i < l ? s / rii : 0.0);
    }
  }
  if (l < b) {
    const bool dc = (dead >> l) & 1;
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (i < b) Rinv[i * b + l] = dc ? 0.0 : y[i];
  }
}

// Start block (n x B): columns 0..kw-1 from the warm vectors (n x kw,
// row-major), the rest seeded directions (SplitMix64 of (column, row),
// uniform in [-1, 1)).
__global__ void k_kr_start(const double* __restrict__ warm, int kw, int n, int B, double* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * B) return;
  const int r = (int)(idx / B), cc = (int)(idx % B);
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

// max_k ||AV[:,k] - lam_k V[:,k]|| / lam_0, one workgroup
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

// out (J x nc) = A^T B over n rows, in one launch (no row ranges)
void tn(Ctx* c, const double* A, int lda, int J, const double* B, int ldb, int nc, int n, double* out) {
  hipLaunchKernelGGL(k_kr_tn<double>, dim3(g16(J), g16(nc), 1), dim3(KR_TN_WAVES * 64), 0, c->stream, A,
                     (int64_t)lda, J, B, ldb, nc, (int64_t)n, (int64_t)n, out);
  TK_CHECK_LAUNCH();
}

// D = A C (SUB: D = S - A C), 16 columns per launch
template <bool SUB, class TA>
void nn(Ctx* c, const TA* A, int64_t lda, int J, const double* C, int ldc, const double* S, int lds, double* D,
        int ldd, int64_t n, int nc) {
  for (int c0 = 0; c0 < nc; c0 += 16) {
    const int w = std::min(16, nc - c0);
    const double* Sc = SUB ? S + c0 : nullptr;
    // a long k range goes over sixteen waves, so each wave's chain of dependent steps is short
    if (J >= 256)
      hipLaunchKernelGGL((k_kr_nn<SUB, 16, TA>), dim3(g16(n)), dim3(16 * 64), 0, c->stream, A, lda, J, C + c0, ldc,
                         Sc, lds, D + c0, ldd, n, w);
    else
      hipLaunchKernelGGL((k_kr_nn<SUB, 4, TA>), dim3(g16(n)), dim3(4 * 64), 0, c->stream, A, lda, J, C + c0, ldc,
                         Sc, lds, D + c0, ldd, n, w);
    TK_CHECK_LAUNCH();
  }
}

// Q[:, q0:q0+B] = orthonormal basis of W (three CholeskyQR passes, W and W2
// alternating, the last one written into Q)
template <int B>
void cholqr(Ctx* c, const KrBufs& b, int n, int q0) {
  double* A = b.small;            // B x B Gram
  double* Ri = b.small + B * B;
  double* src = b.W;
  for (int pass = 0; pass < 3; ++pass) {
    tn(c, src, B, B, src, B, B, n, A);
    hipLaunchKernelGGL(k_kr_chol<B>, dim3(1), dim3(64), 0, c->stream, A, B, Ri, pass == 0 ? n : 0);
    TK_CHECK_LAUNCH();
    double* dst = pass == 2 ? b.Q + q0 : (src == b.W ? b.W2 : b.W);
    nn<false, double>(c, src, B, B, Ri, B, nullptr, 0, dst, pass == 2 ? KR_M : B, n, B);
    src = dst;
  }
}

// The operator G X with G formed (n x n).
struct GramOp {
  const double* G;
  int n;
  void apply(Ctx* c, const double* X, int ldx, double* out, int ldo, int nc) const {
    nn<false, double>(c, G, n, n, X, ldx, nullptr, 0, out, ldo, n, nc);
  }
};

// The operator Y^T (Y X) from Y (R x khat FP32), never squared: T = Y X
// (R x nc, FP64), then Y^T T in row ranges summed in range order.
struct MatFreeOp {
  const float* Y;
  int64_t R;
  int khat;
  double* T;       // R x 32
  double* part;    // splits x khat x 32
  int splits;
  void apply(Ctx* c, const double* X, int ldx, double* out, int ldo, int nc) const {
    nn<false, float>(c, Y, khat, khat, X, ldx, nullptr, 0, T, nc, R, nc);
    const int64_t rows = ceil_div(std::max<int64_t>(R, 1), splits);
    hipLaunchKernelGGL(k_kr_tn<float>, dim3(g16(khat), g16(nc), splits), dim3(KR_TN_WAVES * 64), 0, c->stream, Y,
                       (int64_t)khat, khat, T, nc, nc, R, rows, part);
    TK_CHECK_LAUNCH();
    const int64_t cnt = (int64_t)khat * nc;
    double* dst = ldo == nc ? out : part + (int64_t)splits * cnt;   // a strided destination: sum, then copy
    hipLaunchKernelGGL(k_kr_sum_parts, dim3(grid_for(cnt, 256, 4096)), dim3(256), 0, c->stream, part, splits, cnt,
                       dst);
    TK_CHECK_LAUNCH();
    if (dst != out)
      TK_HIP(hipMemcpy2DAsync(out, sizeof(double) * ldo, dst, sizeof(double) * nc, sizeof(double) * nc, khat,
                              hipMemcpyDeviceToDevice, c->stream));
  }
};

// Block Krylov with B-column blocks and S blocks per cycle (S * B = KR_M) on
// the operator; Kout >= K columns of VK are written (the first K).  Returns
// false when the best cycle's result is not accepted (krylov_accepts).
template <int B, int S, class Op>
bool krylov_run(Ctx* c, const Op& op, int n, int K, int Kout, double* lam_k, double* VK, int mode) {
  static_assert(B * S == KR_M, "subspace size");
  // cycles, and the residual reduction a restart must bring to go on: the
  // 32-column block's cycle is a degree-3 Krylov space, which gains less per
  // cycle than the 16-column block's degree 6
  constexpr int KR_CYCLES = B == 16 ? 4 : 12;
  constexpr double KR_GAIN = B == 16 ? 0.5 : 0.85;
  TK_REQUIRE(K < B || (B == 16 && K == 16), TK_ERR_UNSUPPORTED, "Krylov eigensolve: block too narrow");
  // the Rayleigh-Ritz step also yields theta_{K+1}, the gap estimate
  const int Kr = K + 1;
  KrBufs b{};
  const size_t nQ = (size_t)n * KR_M;
  const size_t need = 2 * nQ + 2 * (size_t)n * B + 4 * B * B + KR_M * KR_M + 64 + (size_t)KR_M * (B + 1) +
                      (size_t)n * Kr + 8 + (size_t)n * B + B;
  ensure(c, c->kr_work, sizeof(double) * need);
  double* p = c->kr_work.as<double>();
  b.Q = p; p += nQ;
  b.GQ = p; p += nQ;
  b.W = p; p += (size_t)n * B;
  b.W2 = p; p += (size_t)n * B;
  b.small = p; p += 4 * B * B;
  b.H = p; p += KR_M * KR_M;
  b.lamH = p; p += 64;
  b.S = p; p += (size_t)KR_M * (B + 1);
  b.GV = p; p += (size_t)n * Kr;
  b.res = p; p += 8;
  b.bestV = p; p += (size_t)n * B;
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
    hipLaunchKernelGGL(k_kr_start, dim3(g1((int64_t)n * B)), dim3(256), 0, c->stream, wsrc, kws, n, B, b.W);
    TK_CHECK_LAUNCH();
    TK_HIP(hipMemsetAsync(b.Q, 0, sizeof(double) * nQ, c->stream));
    cholqr<B>(c, b, n, 0);
    for (int j = 0; j < S; ++j) {
      const int q0 = j * B, J = q0 + B;
      // GQ_j = A Q_j
      op.apply(c, b.Q + q0, KR_M, b.GQ + q0, KR_M, B);
      if (j == S - 1) break;
      // W = GQ_j - Q_{0..j} (Q_{0..j}^T GQ_j), then once more on W (full re-orthogonalisation)
      for (int rep = 0; rep < 2; ++rep) {
        double* Cm = b.H;   // J x B coefficients; H is free until the Rayleigh-Ritz step
        const double* src = rep == 0 ? b.GQ + q0 : b.W;
        const int ls = rep == 0 ? KR_M : B;
        tn(c, b.Q, KR_M, J, src, ls, B, n, Cm);
        nn<true, double>(c, b.Q, KR_M, J, Cm, B, src, ls, b.W, B, n, B);
      }
      cholqr<B>(c, b, n, J);
    }
    // Rayleigh-Ritz on span(Q): K + 1 Ritz pairs, the first K kept
    tn(c, b.Q, KR_M, KR_M, b.GQ, KR_M, KR_M, n, b.H);
    eig_topk(c, b.H, KR_M, Kr, b.lamH, b.S, -1);
    nn<false, double>(c, b.Q, KR_M, KR_M, b.S, Kr, nullptr, 0, VK, Kout, n, K);
    TK_HIP(hipMemcpyAsync(lam_k, b.lamH, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
    // residual check
    op.apply(c, VK, Kout, b.GV, K, K);
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
    // converged to the FP64 level (and acceptable), or a restart that no
    // longer improves (the rounding floor)
    if ((res <= 1e-10 && c->krylov_accepts(res, err)) || (cycle > 0 && res > KR_GAIN * prev_res)) break;
    prev_res = res;
  }
  ++c->counters.eig_krylov_solves;
  if (best_cycle != last_cycle) {
    TK_HIP(hipMemcpy2DAsync(VK, sizeof(double) * Kout, b.bestV, sizeof(double) * K, sizeof(double) * K, n,
                            hipMemcpyDeviceToDevice, c->stream));
    TK_HIP(hipMemcpyAsync(lam_k, b.bestLam, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
  }
  const bool ok = c->krylov_accepts(best_res, best_err);
  if (ok && warm) {
    ensure(c, *warm, sizeof(double) * (size_t)n * K);
    TK_HIP(hipMemcpy2DAsync(warm->as<double>(), sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K,
                            n, hipMemcpyDeviceToDevice, c->stream));
    c->eig_warm_k[mode] = K;
  }
  return ok;
}

void keep_warm(Ctx* c, int mode, int n, int K, int Kout, const double* VK) {
  if (mode < 0) return;
  Buf* warm = &c->eig_warm[mode];
  ensure(c, *warm, sizeof(double) * (size_t)n * K);
  TK_HIP(hipMemcpy2DAsync(warm->as<double>(), sizeof(double) * K, VK, sizeof(double) * Kout, sizeof(double) * K, n,
                          hipMemcpyDeviceToDevice, c->stream));
  c->eig_warm_k[mode] = K;
}
}  // namespace

// U (R x K, FP64) = Y (R x khat FP32) W (khat x K FP64) on the FP64 matrix
// cores, for factor steps whose W does not fit in LDS.
void tall_times_small(Ctx* c, const float* Y, int64_t R, int khat, const double* W, int K, double* U) {
  if (R == 0) return;
  nn<false, float>(c, Y, khat, khat, W, K, nullptr, 0, U, K, R, K);
}

// Leading K (<= 16) eigenpairs of G (n x n FP64): lam_k descending, VK (n x Kout).
// mode >= 0 keeps the eigenvectors for that mode's next call.
void eig_topk_krylov(Ctx* c, const double* G, int n, int K, int Kout, double* lam_k, double* VK, int mode) {
  TK_REQUIRE(K <= 16, TK_ERR_UNSUPPORTED, "Krylov eigensolve: more than 16 eigenpairs");
  if (!krylov_run<16, 6>(c, GramOp{G, n}, n, K, Kout, lam_k, VK, mode)) {
    // the Krylov subspace is not accurate enough (slow convergence or a tight
    // gap at K): the dense solver on G
    ++c->counters.eig_dense_fallbacks;
    eig_topk_dense(c, G, n, Kout, lam_k, VK);
    keep_warm(c, mode, n, K, Kout, VK);
  }
}

// Matrix-free: leading K (<= 31) eigenpairs of Y^T Y from Y (R x khat FP32),
// and diag(Y^T Y) (khat FP64, for the rank floor).  The Gram (the context's
// Gram buffer) is formed only on the fallback.
void eig_topk_matfree(Ctx* c, const float* Y, int64_t R, int khat, int K, double* lam_k, double* VK, int mode,
                      double* diag) {
  TK_REQUIRE(K <= 31, TK_ERR_UNSUPPORTED, "matrix-free eigensolve: more than 31 eigenpairs");
  TK_REQUIRE(khat >= 2 * KR_M, TK_ERR_UNSUPPORTED, "matrix-free eigensolve: Khat below 192");
  if (R == 0) {   // no rows: the Gram route (G = 0)
    ensure(c, c->gram64, sizeof(double) * (size_t)khat * khat);
    gram(c, Y, R, khat, c->gram64.as<double>(), false);
    TK_HIP(hipMemsetAsync(diag, 0, sizeof(double) * khat, c->stream));
    eig_topk(c, c->gram64.as<double>(), khat, K, lam_k, VK, mode);
    return;
  }
  const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(R, 8192)));
  const size_t need = (size_t)std::max<int64_t>(R, 1) * 32 + (size_t)(splits + 1) * khat * 32;
  ensure(c, c->mf_work, sizeof(double) * need);
  MatFreeOp op{Y, R, khat, c->mf_work.as<double>(), c->mf_work.as<double>() + (size_t)std::max<int64_t>(R, 1) * 32,
               splits};
  // diag(Y^T Y)
  {
    const int64_t rows = ceil_div(std::max<int64_t>(R, 1), splits);
    hipLaunchKernelGGL(k_colsq_part, dim3(g1(khat), splits), dim3(256), 0, c->stream, Y, R, khat, rows, op.part);
    TK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_kr_sum_parts, dim3(grid_for(khat, 256, 4096)), dim3(256), 0, c->stream, op.part, splits,
                       (int64_t)khat, diag);
    TK_CHECK_LAUNCH();
  }
  const bool ok = K <= 16 ? krylov_run<16, 6>(c, op, khat, K, K, lam_k, VK, mode)
                          : krylov_run<32, 3>(c, op, khat, K, K, lam_k, VK, mode);
  if (!ok) {
    // the Gram route: form G, then its own solver (with its dense fallback)
    ++c->counters.eig_dense_fallbacks;
    ensure(c, c->gram64, sizeof(double) * (size_t)khat * khat);
    double* G = c->gram64.as<double>();
    gram(c, Y, R, khat, G, false);
    eig_topk(c, G, khat, K, lam_k, VK, -1);
    keep_warm(c, mode, khat, K, K, VK);
  }
}

}  // namespace tk
