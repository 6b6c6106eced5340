// Gram matrix G = Y^T Y of the compact penultimate matrix (R rows x Khat
// columns, FP32 row-major) on the matrix cores.  It replaces the paper's
// Lanczos queries (Section 3, "SVD Component"): the leading left singular
// vectors of Y are Y V S^-1 for the leading eigenpairs (V, S^2) of G.
//
// v_mfma_f32_16x16x4_f32: lane l supplies A[i = l%16][k = l/16] and
// B[k = l/16][j = l%16]; with A = Y^T and B = Y both operands are
// Y[row0 + l/16][col0 + l%16], i.e. one coalesced load of four 64-byte row
// pieces feeds every tile in the same column block.  The result tile holds
// D[4*(l/16) + r][l%16] in register r.
//
// Precision form: the same tiles on v_mfma_f32_16x16x32_bf16, where lane l
// supplies eight consecutive rows (k = 8*(l/16) .. +7) of column l%16 rounded
// to BF16 (round to nearest even); products accumulate in FP32.  A and B take
// their k values from the same rows, so the order of k inside a step does not
// matter.
//
// Wide Grams (Khat > 128, several macro tile pairs) in the precision form
// first write a BF16 copy of Y in that operand order (k_y_bf16_blocked), so
// that each operand is one 16-byte load instead of eight 4-byte ones, and the
// copy that every macro pair re-reads is half the bytes (k_gram_bf16b, same
// tiles and order, same partials bit for bit).
//
// Each wave accumulates its share of 4-row steps for a set of 16x16 tiles;
// the four waves of a workgroup are combined in LDS in fixed order and each
// workgroup writes one FP32 partial; a second kernel sums the partials in
// FP64 in workgroup order (deterministic) and mirrors the upper triangle.
#include "common.hpp"

namespace tk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int GRAM_BATCH = 4;   // FP32 Gram: 4-row steps whose loads are issued together

// Tiles (bi, bj) of the macro pair: bi in [I0, I0+NBA), bj in [J0, J0+NBB);
// DIAG = the pair is on the diagonal and only bi <= bj is computed.
template <int NBA, int NBB, bool DIAG>
struct TileSet {
  static constexpr int count = DIAG ? NBA * (NBA + 1) / 2 : NBA * NBB;
  __device__ static constexpr int ti(int t) {
    if (!DIAG) return t / NBB;
    int i = 0;
    while (t >= NBA - i) { t -= NBA - i; ++i; }
    return i;
  }
  __device__ static constexpr int tj(int t) {
    if (!DIAG) return t % NBB;
    int i = 0;
    while (t >= NBA - i) { t -= NBA - i; ++i; }
    return i + t;
  }
};

// Macro pair of blockIdx.y: diagonal launches take (p, p); off-diagonal
// launches enumerate I < J row by row.
__device__ __forceinline__ void macro_pair(bool diag, int p, int MB, int& I, int& J) {
  if (diag) { I = J = p; return; }
  I = 0;
  while (p >= MB - 1 - I) { p -= MB - 1 - I; ++I; }
  J = I + 1 + p;
}

// Macro pairs of up to 4 x 4 tiles are capped at four waves per SIMD (at most
// 128 registers per lane; the compiler's own choice, 154, allows three): the
// waves wait on their loads for most of their cycles, and the fourth hides
// more of it (the wide c3 Gram 34.7 -> 32.2 ms).  Larger macro pairs would spill.
template <int NBA, int NBB, bool DIAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NBA * NBB <= 16 ? 4 : 1))) void k_gram(
    const float* __restrict__ Y, int64_t R, int khat, int rows_per_wg,
                                              int MB, float* __restrict__ part) {
  using TS = TileSet<NBA, NBB, DIAG>;
  constexpr int T = TS::count;
  extern __shared__ float red[];  // T * 256 floats
  const int pair = blockIdx.y;
  int PI, PJ;
  macro_pair(DIAG, pair, MB, PI, PJ);
  const int I0 = PI * NBA, J0 = PJ * NBB;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(r0 + rows_per_wg, R);
  floatx4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lr = lane >> 4, lc = lane & 15;
  // software pipeline: the next 4-row step is loaded while this one's MFMAs run
  // buffer loads over this workgroup's rows: a row past r1 lies beyond the
  // resource and a column past khat carries an out-of-range offset, so both
  // read as zero with no condition on the load
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Y + r0 * khat, (uint32_t)((r1 - r0) * khat * 4));
  uint32_t ca[NBA], cb[NBB];
#pragma unroll
  for (int b = 0; b < NBA; ++b) {
    const int col = (I0 + b) * 16 + lc;
    ca[b] = col < khat ? 4u * col : BUF_OOB;
  }
#pragma unroll
  for (int b = 0; b < NBB; ++b) {
    const int col = (J0 + b) * 16 + lc;
    cb[b] = col < khat ? 4u * col : BUF_OOB;
  }
  auto load = [&](int64_t r, float (&xa)[NBA], float (&xb)[NBB]) {
    const uint32_t rb = 4u * (uint32_t)((r + lr - r0) * khat);
#pragma unroll
    for (int b = 0; b < NBA; ++b) xa[b] = buf_f32(rs, rb + ca[b]);
    if constexpr (DIAG) {
#pragma unroll
      for (int b = 0; b < NBB; ++b) xb[b] = xa[b];
    } else {
#pragma unroll
      for (int b = 0; b < NBB; ++b) xb[b] = buf_f32(rs, rb + cb[b]);
    }
  };
  // batches of GRAM_BATCH steps: every load of a batch is issued first, then
  // each step waits only for its own loads; no register value crosses an
  // iteration (a loop-carried load forces a full wait); steps past r1 read zeros
  for (int64_t r = r0 + 4 * wave; r < r1; r += 16 * GRAM_BATCH) {
    float xa[GRAM_BATCH][NBA], xb[GRAM_BATCH][NBB];
#pragma unroll
    for (int d = 0; d < GRAM_BATCH; ++d) load(r + 16 * d, xa[d], xb[d]);
#pragma unroll
    for (int d = 0; d < GRAM_BATCH; ++d) {
      int t = 0;
#pragma unroll
      for (int a = 0; a < NBA; ++a)
#pragma unroll
        for (int bj = DIAG ? a : 0; bj < NBB; ++bj, ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[d][a], xb[d][bj], acc[t], 0, 0, 0);
    }
  }
  // combine the four waves in fixed order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float* dst = red + t * 256 + q * 64 + lane;
          *dst = (w == 0) ? acc[t][q] : *dst + acc[t][q];
        }
    }
    __syncthreads();
  }
  float* out = part + ((int64_t)blockIdx.x * gridDim.y + pair) * (int64_t)T * 256;
  for (int i = threadIdx.x; i < T * 256; i += blockDim.x) out[i] = red[i];
}

// BF16 operands, FP32 accumulation: 32 rows per MFMA step, each wave takes
// every fourth 32-row step of the workgroup's rows.
template <int NBA, int NBB, bool DIAG>
__global__ __launch_bounds__(256) void k_gram_bf16(const float* __restrict__ Y, int64_t R, int khat,
                                                   int rows_per_wg, int MB, float* __restrict__ part) {
  using TS = TileSet<NBA, NBB, DIAG>;
  constexpr int T = TS::count;
  constexpr int NL = DIAG ? NBA : NBA + NBB;   // column blocks loaded per step
  extern __shared__ float red[];
  const int pair = blockIdx.y;
  int PI, PJ;
  macro_pair(DIAG, pair, MB, PI, PJ);
  const int I0 = PI * NBA, J0 = PJ * NBB;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(r0 + rows_per_wg, R);
  floatx4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lr = lane >> 4, lc = lane & 15;
  int cols[NL];
#pragma unroll
  for (int b = 0; b < NL; ++b) cols[b] = (b < NBA ? (I0 + b) : (J0 + b - NBA)) * 16 + lc;
  // FP32 values of the next step stay in flight while this step's MFMAs run
  // buffer loads over this workgroup's rows: rows past r1 lie beyond the
  // resource, columns past khat carry an out-of-range offset (both read zero)
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Y + r0 * khat, (uint32_t)((r1 - r0) * khat * 4));
  uint32_t coff[NL];
#pragma unroll
  for (int b = 0; b < NL; ++b) coff[b] = cols[b] < khat ? 4u * cols[b] : BUF_OOB;
  auto load = [&](int64_t r, float (&f)[NL][8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t rb = 4u * (uint32_t)((r + 8 * lr + q - r0) * khat);
#pragma unroll
      for (int b = 0; b < NL; ++b) f[b][q] = buf_f32(rs, rb + coff[b]);
    }
  };
  // batches of two 32-row steps: both steps' loads issued first, no register
  // value crossing an iteration; steps past r1 read zeros
  for (int64_t r = r0 + 32 * wave; r < r1; r += 256) {
    float f[2][NL][8];
    load(r, f[0]);
    load(r + 128, f[1]);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      bf16x8 x[NL];
#pragma unroll
      for (int b = 0; b < NL; ++b)
#pragma unroll
        for (int q = 0; q < 8; ++q) x[b][q] = (__bf16)f[d][b][q];
      int t = 0;
#pragma unroll
      for (int a = 0; a < NBA; ++a)
#pragma unroll
        for (int bj = DIAG ? a : 0; bj < NBB; ++bj, ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[a], x[DIAG ? bj : NBA + bj], acc[t], 0, 0, 0);
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float* dst = red + t * 256 + q * 64 + lane;
          *dst = (w == 0) ? acc[t][q] : *dst + acc[t][q];
        }
    }
    __syncthreads();
  }
  float* out = part + ((int64_t)blockIdx.x * gridDim.y + pair) * (int64_t)T * 256;
  for (int i = threadIdx.x; i < T * 256; i += blockDim.x) out[i] = red[i];
}

// BF16 copy of Y for the wide precision-form Gram, in the operand order of
// v_mfma_f32_16x16x32_bf16: for each block of 32 rows and each column c (of
// KP, Khat rounded up to 16) the 32 rows' values are contiguous, so lane l's
// operand (column c, rows 8*(l/16) .. +7 of the block) is one 16-byte load.
// Values are rounded to nearest even, as the direct kernel rounds them in
// registers; rows past R and columns past Khat are zero.  One workgroup turns
// 32 rows x 256 columns around through LDS, 64 columns at a time, reading Y
// with 16-byte loads when Khat is a multiple of 4.
constexpr int YB_COLS = 256;   // columns per workgroup
__global__ __launch_bounds__(256) void k_y_bf16_blocked(const float* __restrict__ Y, int64_t R, int khat, int KP,
                                                        __bf16* __restrict__ Yb) {
  __shared__ float t[32][65];
  const int64_t rb = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = tid >> 3, cq = (tid & 7) * 8;
  const int64_t row = rb * 32 + r;
  const bool vec = (khat & 3) == 0;
  const int cend = min(KP, (int)(blockIdx.y + 1) * YB_COLS);
  for (int c0 = blockIdx.y * YB_COLS; c0 < cend; c0 += 64) {
    const int col = c0 + cq;
    if (row < R && vec && col + 8 <= khat) {
      const float4* src = reinterpret_cast<const float4*>(Y + row * khat + col);
      const float4 a = src[0], b = src[1];
      t[r][cq + 0] = a.x; t[r][cq + 1] = a.y; t[r][cq + 2] = a.z; t[r][cq + 3] = a.w;
      t[r][cq + 4] = b.x; t[r][cq + 5] = b.y; t[r][cq + 6] = b.z; t[r][cq + 7] = b.w;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) t[r][cq + q] = (row < R && col + q < khat) ? Y[row * khat + col + q] : 0.f;
    }
    __syncthreads();
    const int c = tid >> 2, g = tid & 3;
    if (c0 + c < KP) {
      bf16x8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (__bf16)t[8 * g + q][c];
      *reinterpret_cast<bf16x8*>(Yb + ((rb * KP + c0 + c) * 32 + 8 * g)) = v;
    }
    __syncthreads();
  }
}

// The precision-form Gram from the blocked BF16 copy: the tiles, steps and
// order of k_gram_bf16 (so the same partials, bit for bit), with each operand
// one 16-byte load instead of eight 4-byte ones.
template <int NBA, int NBB, bool DIAG>
__global__ __launch_bounds__(256) void k_gram_bf16b(const __bf16* __restrict__ Yb, int64_t R, int KP,
                                                    int rows_per_wg, int MB, float* __restrict__ part) {
  using TS = TileSet<NBA, NBB, DIAG>;
  constexpr int T = TS::count;
  constexpr int NL = DIAG ? NBA : NBA + NBB;   // column blocks loaded per step
  extern __shared__ float red[];
  const int pair = blockIdx.y;
  int PI, PJ;
  macro_pair(DIAG, pair, MB, PI, PJ);
  const int I0 = PI * NBA, J0 = PJ * NBB;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;   // a multiple of 128
  const int64_t r1 = min(r0 + rows_per_wg, R);
  floatx4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lr = lane >> 4, lc = lane & 15;
  // the workgroup's row blocks form one buffer resource: steps past r1 read zeros
  const int64_t nrb = (r1 - r0 + 31) / 32;
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Yb + (r0 / 32) * KP * 32, (uint32_t)(nrb * KP * 64));
  uint32_t coff[NL];
#pragma unroll
  for (int b = 0; b < NL; ++b) {
    const int blk = b < NBA ? I0 + b : J0 + b - NBA;   // blocks past the last one read zeros
    coff[b] = blk * 16 < KP ? 2u * (uint32_t)((blk * 16 + lc) * 32 + 8 * lr) : BUF_OOB;
  }
  auto load = [&](int64_t r, bf16x8 (&x)[NL]) {
    const uint32_t rb = 2u * (uint32_t)(((r - r0) >> 5) * KP * 32);
#pragma unroll
    for (int b = 0; b < NL; ++b)
      x[b] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, rb + coff[b], 0, 0));
  };
  for (int64_t r = r0 + 32 * wave; r < r1; r += 256) {
    bf16x8 x[2][NL];
    load(r, x[0]);
    load(r + 128, x[1]);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      int t = 0;
#pragma unroll
      for (int a = 0; a < NBA; ++a)
#pragma unroll
        for (int bj = DIAG ? a : 0; bj < NBB; ++bj, ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[d][a], x[d][DIAG ? bj : NBA + bj], acc[t], 0, 0, 0);
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float* dst = red + t * 256 + q * 64 + lane;
          *dst = (w == 0) ? acc[t][q] : *dst + acc[t][q];
        }
    }
    __syncthreads();
  }
  float* out = part + ((int64_t)blockIdx.x * gridDim.y + pair) * (int64_t)T * 256;
  for (int i = threadIdx.x; i < T * 256; i += blockDim.x) out[i] = red[i];
}

// Level 1: sum groups of `group` consecutive chunk partials in FP64 (fixed order).
__global__ void k_colsum_groups(const float* __restrict__ in, int64_t P, int64_t M, int group,
                                double* __restrict__ out) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= M) return;
  const int64_t p0 = (int64_t)blockIdx.y * group;
  const int64_t p1 = min<int64_t>(p0 + group, P);
  double s = 0.0;
  for (int64_t p = p0; p < p1; ++p) s += (double)in[p * M + col];
  out[(int64_t)blockIdx.y * M + col] = s;
}

// Level 2: sum the group partials and scatter into the full symmetric G.
template <int NBA, int NBB, bool DIAG>
__global__ void k_gram_reduce(const double* __restrict__ part, int nchunks, int MB, int khat,
                              double* __restrict__ G) {
  using TS = TileSet<NBA, NBB, DIAG>;
  constexpr int T = TS::count;
  const int pair = blockIdx.y;
  int PI, PJ;
  macro_pair(DIAG, pair, MB, PI, PJ);
  const int I0 = PI * NBA, J0 = PJ * NBB;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // element of the T x 256 tile set
  if (i >= T * 256) return;
  const int t = i >> 8, e = i & 255;
  const int q = e >> 6, lane = e & 63;
  // register q of lane holds D[4*(lane/16) + q][lane%16]
  const int rr = 4 * (lane >> 4) + q, cc = lane & 15;
  const int gi = (I0 + TS::ti(t)) * 16 + rr;
  const int gj = (J0 + TS::tj(t)) * 16 + cc;
  if (gi >= khat || gj >= khat) return;
  if (DIAG && TS::ti(t) == TS::tj(t) && rr > cc) return;  // the (cc, rr) thread writes both halves
  double s = 0.0;
  // part is [group][pair][T*256]
  const double* p = part + (int64_t)pair * T * 256 + i;
  const int64_t stride = (int64_t)gridDim.y * T * 256;
  for (int k = 0; k < nchunks; ++k) s += p[k * stride];
  G[(int64_t)gi * khat + gj] = s;
  G[(int64_t)gj * khat + gi] = s;
}

template <int NBA, int NBB, bool DIAG, bool BF16>
static void run_gram(Ctx* c, const float* Y, int64_t R, int khat, int npairs, int MB, double* G,
                     const __bf16* Yb = nullptr, int KP = 0) {
  using TS = TileSet<NBA, NBB, DIAG>;
  constexpr int T = TS::count;
  if (npairs == 0) return;
  // about 1024 workgroups for the many-pair FP32 Gram (matrix-core bound: every
  // SIMD busy), about 512 for the BF16 and the single-pair ones (fewer, longer
  // row chunks and half the partials: 12-15% faster there)
  const int64_t target_wgs = std::max<int64_t>(1, ((BF16 || npairs == 1) ? 512 : 1024) / npairs);
  const int64_t gran = BF16 ? 128 : 16;   // rows per workgroup-wide step
  int64_t rpw = std::max<int64_t>(BF16 ? 128 : 64, ceil_div(ceil_div(R, target_wgs), gran) * gran);
  // a workgroup's rows form one buffer resource: keep them below 2^31 bytes
  rpw = std::min<int64_t>(rpw, std::max<int64_t>(gran, ((int64_t)0x7fff0000 / (4 * (int64_t)khat)) / gran * gran));
  const int rows_per_wg = (int)rpw;
  const int nchunks = (int)std::max<int64_t>(1, ceil_div(R, rows_per_wg));
  const int group = 32;
  const int ngroups = (nchunks + group - 1) / group;
  const int64_t M = (int64_t)npairs * T * 256;   // the chunk partials are [chunk][pair][T*256]
  const size_t b1 = sizeof(float) * (size_t)nchunks * M, b2 = sizeof(double) * (size_t)ngroups * M;
  ensure(c, c->gram_part, b1 + b2 + 256);
  float* part = c->gram_part.as<float>();
  double* part2 = reinterpret_cast<double*>(c->gram_part.as<char>() + ((b1 + 255) & ~(size_t)255));
  TK_REQUIRE(((b1 + 255) & ~(size_t)255) + b2 <= c->gram_part.bytes(), TK_ERR_DEVICE, "gram scratch");
  if (BF16 && Yb)
    hipLaunchKernelGGL((k_gram_bf16b<NBA, NBB, DIAG>), dim3(nchunks, npairs), dim3(256), T * 256 * sizeof(float),
                       c->stream, Yb, R, KP, rows_per_wg, MB, part);
  else if (BF16)
    hipLaunchKernelGGL((k_gram_bf16<NBA, NBB, DIAG>), dim3(nchunks, npairs), dim3(256), T * 256 * sizeof(float),
                       c->stream, Y, R, khat, rows_per_wg, MB, part);
  else
    hipLaunchKernelGGL((k_gram<NBA, NBB, DIAG>), dim3(nchunks, npairs), dim3(256), T * 256 * sizeof(float),
                       c->stream, Y, R, khat, rows_per_wg, MB, part);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_colsum_groups, dim3((unsigned)ceil_div(M, 256), ngroups), dim3(256), 0, c->stream, part,
                     (int64_t)nchunks, M, group, part2);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_gram_reduce<NBA, NBB, DIAG>), dim3((T * 256 + 255) / 256, npairs), dim3(256), 0, c->stream,
                     part2, ngroups, MB, khat, G);
  TK_CHECK_LAUNCH();
}

template <bool BF16>
static void gram_impl(Ctx* c, const float* Y, int64_t R, int khat, double* G) {
  const int NB = (khat + 15) / 16;
  if (R == 0) {
    TK_HIP(hipMemsetAsync(G, 0, sizeof(double) * (size_t)khat * khat, c->stream));
    return;
  }
  if (NB <= 8) {
    switch (NB) {
      case 1: run_gram<1, 1, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 2: run_gram<2, 2, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 3: run_gram<3, 3, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 4: run_gram<4, 4, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 5: run_gram<5, 5, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 6: run_gram<6, 6, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      case 7: run_gram<7, 7, true, BF16>(c, Y, R, khat, 1, 1, G); break;
      default: run_gram<8, 8, true, BF16>(c, Y, R, khat, 1, 1, G); break;
    }
    return;
  }
  // macro blocks of 4 column blocks (64 columns): diagonal pairs and the upper off-diagonal pairs
  const int MB = (NB + 3) / 4;
  const __bf16* Yb = nullptr;
  int KP = 0;
  if (BF16) {
    // Y is read once per macro pair: a BF16 copy in operand order first, so
    // that every operand is one 16-byte load of half the bytes
    KP = NB * 16;
    const int64_t RB = ceil_div(R, 32);
    ensure(c, c->ybf, sizeof(uint16_t) * (size_t)RB * KP * 32);
    hipLaunchKernelGGL(k_y_bf16_blocked, dim3((unsigned)RB, (unsigned)ceil_div(KP, YB_COLS)), dim3(256), 0, c->stream, Y, R,
                       khat, KP, c->ybf.as<__bf16>());
    TK_CHECK_LAUNCH();
    Yb = c->ybf.as<__bf16>();
  }
  run_gram<4, 4, true, BF16>(c, Y, R, khat, MB, MB, G, Yb, KP);
  run_gram<4, 4, false, BF16>(c, Y, R, khat, MB * (MB - 1) / 2, MB, G, Yb, KP);
}

// G (khat x khat FP64, full) = Y^T Y; bf16 = operands rounded to BF16 (FP32 accumulation).
void gram(Ctx* c, const float* Y, int64_t R, int khat, double* G, bool bf16) {
  if (bf16) gram_impl<true>(c, Y, R, khat, G);
  else gram_impl<false>(c, Y, R, khat, G);
}

}  // namespace tk
