// TTM-chain along mode n through the Kronecker reformulation (eq. 1,
// Appendix A): row l of Y_(n) is the sum over the elements e of slice l of
// val(e) * (F_a[l_a] (x) F_b[l_b] (x) ...), the first remaining mode fastest.
//
// One workgroup per Lite bin (and per column tile when Khat is wide).  A bin
// holds at most `limit` elements and at most ceil(L/P) + 2 distinct slices
// (Theorem 6.1), so its rows of Y live in LDS for the whole bin:
//   * each thread takes a contiguous run of the bin's elements (the layout is
//     slice-sorted, so a run crosses few slice boundaries) and keeps the
//     running Kronecker sum of its current slice in registers;
//   * at a slice boundary the thread adds its registers into that slice's LDS
//     row (ds_add_f32) and starts over;
//   * after the bin, rows of slices the bin owns alone are written straight to
//     Y; rows of slices split over several bins go to a partial slot, and the
//     fixup kernel sums those slots in bin order.
// Factor rows are gathered with 16-byte loads from FP32 copies whose row
// stride is padded to a multiple of four floats.
#include "common.hpp"

namespace tk {

struct TtmArgs {
  const int64_t* bin_ptr;
  const int32_t* seg_ptr;
  const int32_t* seg_row;
  const int64_t* seg_begin;
  const int32_t* seg_slot;
  const int32_t* lay[7];    // other modes' coordinates in layout order (ascending mode)
  const float* val;
  const float* F[7];        // FP32 factor copies of the other modes
  int fstride[7];
  int Kj[7];
  int div[7];               // prod of Kj[1..j-1] (digit divisors of the slow index)
  int n_other;
  int KA;                   // rank of the first remaining mode (runtime, <= template KA)
  int KW;                   // product of the remaining ranks after the first
  int khat;
  float* Y;
  float* partial;
  int64_t P;
};

template <int K>
__device__ __forceinline__ void load_row4(const float* __restrict__ p, float (&r)[K]) {
  constexpr int NV = (K + 3) / 4;
  float t[NV * 4];
  const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float4 x = p4[i];
    t[4 * i + 0] = x.x;
    t[4 * i + 1] = x.y;
    t[4 * i + 2] = x.z;
    t[4 * i + 3] = x.w;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) r[i] = t[i];
}

// Map the linear block id to a bin so that each XCD (blocks are dealt to the
// 8 XCDs round robin) works on a contiguous range of bins: consecutive bins
// of a large slice then share factor rows in the same L2.
__device__ __forceinline__ int64_t xcd_bin(int64_t b, int64_t G) {
  const int64_t q = G >> 3, r = G & 7;
  const int64_t x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// MODE 1: two-mode tensors (one remaining mode).  MODE 2: three modes, the
// slow factor is one row.  MODE 3: four or more modes, the slow factor is the
// Kronecker of several rows, formed per element for the tile's columns.
// EXACT: KA equals the runtime rank; otherwise KA is an upper bound.
template <int KA, int TW, int MODE, bool EXACT>
__global__ __launch_bounds__(256) void k_ttm(TtmArgs A) {
  extern __shared__ float lds[];
  constexpr int TILEW = KA * TW;
  const int64_t bin = xcd_bin(blockIdx.x, gridDim.x);
  const int tile = blockIdx.y;
  const int cw0 = tile * TW;
  const int ka = EXACT ? KA : A.KA;
  const int64_t e0 = A.bin_ptr[bin], e1 = A.bin_ptr[bin + 1];
  const int s0 = A.seg_ptr[bin], s1 = A.seg_ptr[bin + 1];
  const int nseg = s1 - s0;
  float* rows = lds;                                        // nseg x TILEW
  int* send = reinterpret_cast<int*>(lds + (size_t)nseg * TILEW);  // local end offset per segment
  for (int i = threadIdx.x; i < nseg * TILEW; i += blockDim.x) rows[i] = 0.f;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) send[i] = (int)(A.seg_begin[s0 + i + 1] - e0);
  __syncthreads();

  const int E = (int)(e1 - e0);
  const int q = (E + (int)blockDim.x - 1) / (int)blockDim.x;
  const int lo = (int)threadIdx.x * q;
  const int hi = min(lo + q, E);
  if (lo < hi) {
    int a = 0, b = nseg - 1;  // first segment whose end exceeds lo
    while (a < b) {
      int mid = (a + b) >> 1;
      if (send[mid] > lo) b = mid; else a = mid + 1;
    }
    int sg = a;
    int end = send[sg];
    float acc[TW][KA];
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
      for (int c = 0; c < KA; ++c) acc[t][c] = 0.f;

    auto flush = [&](int s) {
      float* row = rows + (size_t)s * TILEW;
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        if (cw0 + t < A.KW) {
#pragma unroll
          for (int c = 0; c < KA; ++c) {
            if (EXACT || c < ka) atomicAdd(row + t * ka + c, acc[t][c]);
            acc[t][c] = 0.f;
          }
        }
      }
    };

    const float* __restrict__ Fa = A.F[0];
    const int sa = A.fstride[0];
    const int32_t* __restrict__ la = A.lay[0];
    const float* __restrict__ vv = A.val;
    for (int e = lo; e < hi; ++e) {
      if (e == end) {
        flush(sg);
        ++sg;
        end = send[sg];
      }
      const int64_t g = e0 + e;
      const float v = vv[g];
      float ar[KA];
      if constexpr (EXACT) {
        load_row4<KA>(Fa + (int64_t)la[g] * sa, ar);   // row stride >= KA rounded up to 4
      } else {
        const float* ap = Fa + (int64_t)la[g] * sa;
#pragma unroll
        for (int c = 0; c < KA; ++c) ar[c] = (c < ka) ? ap[c] : 0.f;
      }
#pragma unroll
      for (int c = 0; c < KA; ++c) ar[c] *= v;
      float w[TW];
      if constexpr (MODE == 1) {
#pragma unroll
        for (int t = 0; t < TW; ++t) w[t] = (t == 0) ? 1.f : 0.f;
      } else if constexpr (MODE == 2) {
        const float* wr = A.F[1] + (int64_t)A.lay[1][g] * A.fstride[1] + cw0;
        if ((cw0 & 3) == 0 && cw0 + ((TW + 3) & ~3) <= A.fstride[1]) {
          load_row4<TW>(wr, w);
        } else {
#pragma unroll
          for (int t = 0; t < TW; ++t) w[t] = (cw0 + t < A.KW) ? wr[t] : 0.f;
        }
      } else {
        int64_t base[7];
        for (int j = 1; j < A.n_other; ++j) base[j] = (int64_t)A.lay[j][g] * A.fstride[j];
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          const int cw = cw0 + t;
          float p = 0.f;
          if (cw < A.KW) {
            p = 1.f;
            for (int j = 1; j < A.n_other; ++j) p *= A.F[j][base[j] + (cw / A.div[j]) % A.Kj[j]];
          }
          w[t] = p;
        }
      }
#pragma unroll
      for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int c = 0; c < KA; ++c) acc[t][c] = fmaf(ar[c], w[t], acc[t][c]);
    }
    flush(sg);
  }
  __syncthreads();

  // write the bin's rows: owned slices to Y, split slices to their partial slot
  const int tilew = ka * TW;
  const int col0 = ka * cw0;
  for (int i = threadIdx.x; i < nseg * tilew; i += blockDim.x) {
    const int s = i / tilew;
    const int j = i - s * tilew;
    const int col = col0 + j;
    if (col >= A.khat) continue;
    const float x = rows[(size_t)s * TILEW + j];
    const int slot = A.seg_slot[s0 + s];
    if (slot < 0)
      A.Y[(int64_t)A.seg_row[s0 + s] * A.khat + col] = x;
    else
      A.partial[(int64_t)slot * A.khat + col] = x;
  }
}

// Sum the partial rows of every split slice in bin order (deterministic).
__global__ void k_fixup(const int32_t* __restrict__ bad_row, const int32_t* __restrict__ bad_slot,
                        const float* __restrict__ partial, int khat, float* __restrict__ Y) {
  const int k = blockIdx.x;
  const int a = bad_slot[k], b = bad_slot[k + 1];
  const int64_t row = bad_row[k];
  for (int c = threadIdx.x; c < khat; c += blockDim.x) {
    float s = 0.f;
    for (int t = a; t < b; ++t) s += partial[(int64_t)t * khat + c];
    Y[row * khat + c] = s;
  }
}

// ---- dispatch -----------------------------------------------------------------------------------

struct TtmShape {
  int KA, TW, ntiles, mode;
  bool exact;
};

static TtmShape ttm_shape(int N, const int32_t* K, int n) {
  TtmShape s{};
  int first = (n == 0) ? 1 : 0;
  int KA = K[first];
  int KW = 1;
  for (int j = 0; j < N; ++j)
    if (j != n && j != first) KW *= K[j];
  s.mode = (N == 2) ? 1 : (N == 3 ? 2 : 3);
  s.KA = KA;
  // exact instantiations for the common ranks, bounded ones otherwise
  if (s.mode == 2 && KA == 10 && KW == 10) { s.TW = 10; s.exact = true; }
  else if (s.mode == 2 && KA == 5 && KW == 5) { s.TW = 5; s.exact = true; }
  else if (s.mode == 2 && KA == 16 && KW == 16) { s.TW = 8; s.exact = true; }
  else if (s.mode == 3 && KA == 10) { s.TW = 10; s.exact = true; }
  else if (s.mode == 1) { s.TW = 1; s.exact = false; }
  else if (KA <= 16) { s.TW = 8; s.exact = false; }
  else { s.TW = 4; s.exact = false; }
  s.ntiles = (s.mode == 1) ? 1 : (int)ceil_div(KW, s.TW);
  return s;
}

int ttm_tile_width(int N, const int32_t* K, int n) {
  TtmShape s = ttm_shape(N, K, n);
  int kmax = s.exact ? s.KA : (s.mode == 1 ? 32 : (s.KA <= 16 ? 16 : 32));
  return kmax * s.TW;
}

int ttm_rows_cap(Ctx* c, int64_t tile_w) {
  // LDS budget per bin: about 40 KB so three bins share a CU, never past the hardware limit
  int64_t budget = 40960;
  if ((int64_t)c->lds_per_block < budget) budget = (int64_t)c->lds_per_block;
  int64_t cap = budget / (4 * tile_w + 4);
  if (cap > 512) cap = 512;
  if (cap < 3) cap = 3;
  return (int)cap;
}

template <int KA, int TW, int MODE, bool EXACT>
static void launch_ttm(Ctx* c, const TtmArgs& a, const ModePlan& pl, int ntiles, int tilew_alloc) {
  size_t lds = (size_t)pl.R_max * (4 * (size_t)tilew_alloc + 4);
  if (lds == 0) lds = 4;
  dim3 grid((unsigned)pl.P, (unsigned)ntiles);
  hipLaunchKernelGGL((k_ttm<KA, TW, MODE, EXACT>), grid, dim3(256), lds, c->stream, a);
  TK_CHECK_LAUNCH();
}

// TTM-chain of the elements of plan `pl` along mode n with FP32 factor copies
// F32[j] (row stride kp[j]) of every mode j != n; values are the plan's layout values.
void ttm_run(Ctx* c, const ModePlan& pl, int N, int n, const int32_t* K, const float* const* F32, const int* kp,
             const float* lay_val, int64_t m, float* Y) {
  TtmShape s = ttm_shape(N, K, n);
  TK_REQUIRE(s.KA <= 32, TK_ERR_UNSUPPORTED, "rank of the first remaining mode above 32");
  TtmArgs a{};
  a.bin_ptr = pl.bin_ptr.as<int64_t>();
  a.seg_ptr = pl.seg_ptr.as<int32_t>();
  a.seg_row = pl.seg_row.as<int32_t>();
  a.seg_begin = pl.seg_begin.as<int64_t>();
  a.seg_slot = pl.seg_slot.as<int32_t>();
  int no = 0, prod = 1;
  for (int j = 0; j < N; ++j) {
    if (j == n) continue;
    a.lay[no] = pl.lay_idx[no].as<int32_t>();
    a.F[no] = F32[j];
    a.fstride[no] = kp[j];
    a.Kj[no] = K[j];
    if (no >= 1) { a.div[no] = prod; prod *= K[j]; }
    ++no;
  }
  a.n_other = no;
  a.KA = s.KA;
  a.KW = (s.mode == 1) ? 1 : prod;
  a.khat = (int)pl.khat;
  a.val = lay_val;
  a.Y = Y;
  ensure(c, c->partial, sizeof(float) * (size_t)(pl.n_slots > 0 ? pl.n_slots : 1) * (size_t)pl.khat);
  a.partial = c->partial.as<float>();
  a.P = pl.P;
  if (m == 0) {
    if (pl.L_nz > 0) TK_HIP(hipMemsetAsync(Y, 0, sizeof(float) * (size_t)pl.L_nz * pl.khat, c->stream));
    return;
  }
  const int tw = ttm_tile_width(N, K, n);
  if (c->ev_ttm[0]) TK_HIP(hipEventRecord(c->ev_ttm[0], c->stream));
  if (s.exact) {
    if (s.mode == 2 && s.KA == 10) launch_ttm<10, 10, 2, true>(c, a, pl, s.ntiles, tw);
    else if (s.mode == 2 && s.KA == 5) launch_ttm<5, 5, 2, true>(c, a, pl, s.ntiles, tw);
    else if (s.mode == 2 && s.KA == 16) launch_ttm<16, 8, 2, true>(c, a, pl, s.ntiles, tw);
    else launch_ttm<10, 10, 3, true>(c, a, pl, s.ntiles, tw);
  } else if (s.mode == 1) {
    launch_ttm<32, 1, 1, false>(c, a, pl, s.ntiles, tw);
  } else if (s.KA <= 16) {
    if (s.mode == 2) launch_ttm<16, 8, 2, false>(c, a, pl, s.ntiles, tw);
    else launch_ttm<16, 8, 3, false>(c, a, pl, s.ntiles, tw);
  } else {
    if (s.mode == 2) launch_ttm<32, 4, 2, false>(c, a, pl, s.ntiles, tw);
    else launch_ttm<32, 4, 3, false>(c, a, pl, s.ntiles, tw);
  }
  if (c->ev_ttm[1]) TK_HIP(hipEventRecord(c->ev_ttm[1], c->stream));
  if (pl.n_bad > 0) {
    hipLaunchKernelGGL(k_fixup, dim3((unsigned)pl.n_bad), dim3(128), 0, c->stream, pl.bad_row.as<int32_t>(),
                       pl.bad_slot.as<int32_t>(), c->partial.as<float>(), (int)pl.khat, Y);
    TK_CHECK_LAUNCH();
  }
}

void ttm_chain(Ctx* c, int n, float* Y, bool bf16) {
  (void)bf16;
  const float* F[8];
  for (int j = 0; j < c->N; ++j) F[j] = c->F32[j].as<float>();
  ttm_run(c, c->plan[n], c->N, n, c->K, F, c->kp32, c->plan[n].lay_val.as<float>(), c->m, Y);
}

}  // namespace tk
