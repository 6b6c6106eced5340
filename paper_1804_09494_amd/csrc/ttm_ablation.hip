// TTM-chain kernels kept as ablations of the Lite-bin kernels in ttm.hip:
//   * k_ttm_atomic: no partition, FP32 atomics into Y (TK_TTM_ATOMIC);
//   * k_ttm_fiber:  eq. 1 grouped by fibers on the vector ALUs (TK_TTM_FIBER).
#include "ttm_common.hpp"

namespace tk {

// ---- TTM-chain without a partition (ablation baseline) ---------------------------------------
//
// The merged element list in canonical order, cut into contiguous chunks of
// TTMA_CHUNK elements per wave; lanes over columns as in k_ttm_cols.  A wave
// keeps the running sum of the current mode-n slice in registers and adds it
// to Y with FP32 atomics when the slice changes (in canonical order the
// mode-1 index changes rarely, the others almost every element).  The order
// of the atomic additions depends on timing: results are not deterministic.
constexpr int TTMA_CHUNK = 512;

struct TtmAtomicArgs {
  const int32_t* idx[8];    // canonical coordinates of every mode
  const int32_t* label[8];  // storage label of each index (the factor copies' row order)
  const float* val;
  const float* F[8];
  int fstride[8];
  int Kj[8];
  int N, n;
  const int32_t* row_of;    // compact row of each mode-n slice
  int khat;
  int64_t m;
  float* Y;
};

template <int NO>
__global__ __launch_bounds__(256) void k_ttm_atomic(TtmAtomicArgs A) {
  const int no = NO > 0 ? NO : A.N - 1;
  const int lane = threadIdx.x & 63;
  const int64_t wave_id = (int64_t)blockIdx.x * 4 + uni(threadIdx.x >> 6);
  const int col0 = blockIdx.y * TTMV_TILE;
  const int64_t cs = wave_id * TTMA_CHUNK;
  if (cs >= A.m) return;
  const int64_t ce = min(cs + (int64_t)TTMA_CHUNK, A.m);
  int oj[7];                // the other modes, ascending
  {
    int q = 0;
    for (int j = 0; j < A.N; ++j)
      if (j != A.n) oj[q++] = j;
  }
  int off[TTMV_CPL][7];
  bool colok[TTMV_CPL];
#pragma unroll
  for (int u = 0; u < TTMV_CPL; ++u) {
    const int col = col0 + lane + 64 * u;
    colok[u] = col < A.khat;
    int rest = colok[u] ? col : 0;
    for (int q = 0; q < no; ++q) {
      off[u][q] = rest % A.Kj[oj[q]];
      rest /= A.Kj[oj[q]];
    }
  }
  float acc[TTMV_CPL] = {};
  int cur = -1;
  auto flush = [&]() __attribute__((always_inline)) {
    if (cur >= 0) {
      float* y = A.Y + (int64_t)A.row_of[cur] * A.khat + col0 + lane;
#pragma unroll
      for (int u = 0; u < TTMV_CPL; ++u)
        if (colok[u]) atomicAdd(y + 64 * u, acc[u]);
    }
#pragma unroll
    for (int u = 0; u < TTMV_CPL; ++u) acc[u] = 0.f;
  };
  for (int64_t e = cs; e < ce; ++e) {
    const int l = A.idx[A.n][e];            // uniform: every lane reads the same element
    if (l != cur) {
      flush();
      cur = l;
    }
    const float v = A.val[e];
    float p[TTMV_CPL];
#pragma unroll
    for (int u = 0; u < TTMV_CPL; ++u) p[u] = v;
    for (int q = 0; q < no; ++q) {
      const int j = oj[q];
      const int64_t r = (int64_t)A.label[j][A.idx[j][e]] * A.fstride[j];
#pragma unroll
      for (int u = 0; u < TTMV_CPL; ++u) p[u] *= A.F[j][r + off[u][q]];
    }
#pragma unroll
    for (int u = 0; u < TTMV_CPL; ++u) acc[u] += p[u];
  }
  flush();
}

// ---- fiber-factored TTM-chain (three or four modes, other ranks <= 16) -----------------------------
//
// Elements of one slice that agree on every remaining coordinate but the last
// (mode c) form a fiber; within a segment they are contiguous (the layout
// keeps the canonical order inside each slice).  Eq. 1 then factors by fibers:
//   Y[l] = sum over fibers f of slice l of  F_a[l_a(f)] (x) F_b[l_b(f)] (x) t_f,
//   t_f = sum over elements e of f of val(e) F_c[l_c(e)],
// with F_b absent for three modes.  A fiber costs K_c multiply-adds per
// element and one rank-one update of K_a K_b K_c entries, instead of a
// Kronecker row of K-hat entries per element.
//
// One wave per Lite bin.  The bin's coordinates and values are staged in LDS
// and its fiber starts found with ballots.  Fibers go in batches of sixteen:
// lane group g (four lanes, lane q holding columns 4q..4q+3 of a 16-float
// row) forms t of fiber 16i + g with 16-byte gathers of the F_c rows and
// gathers the fiber's F_a and F_b rows; the three rows go to an LDS stage.
// Then every lane updates its accumulators for the batch's fibers in order,
// one (a, b) pair per lane and pair slot (pair = a + K_a b), reading the
// fiber's rows from the stage as broadcasts.  A segment's row goes straight
// from the accumulators to Y (or to its partial slot when the slice is split
// across bins) when the next fiber belongs to a later segment; the column of
// entry (pair, c) is pair + K_a K_b c, the first remaining mode fastest.  Sums
// run in element order within a fiber and in fiber order within a slice:
// deterministic.
constexpr int TTMF_MAXP = 4;   // pair slots per lane: K_a K_b <= 256
constexpr int TTMF_BATCH = 16; // fibers per batch (one per four-lane group)

template <int NP>
__global__ __launch_bounds__(64) void k_ttm_fiber(TtmArgs A, int Epad) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t bin = xcd_bin(blockIdx.x, gridDim.x);
  const int64_t e0 = A.bin_ptr[bin];
  const int E = (int)(A.bin_ptr[bin + 1] - e0);   // multiple of 4
  const int s0 = A.seg_ptr[bin];
  const int nseg = A.seg_ptr[bin + 1] - s0;
  if (nseg == 0) return;
  const bool four = A.n_other == 3;
  const int ka = A.Kj[0], kb = four ? A.Kj[1] : 1, kc = A.Kj[A.n_other - 1];
  const int P = ka * kb, khat = A.khat;
  float* stage = reinterpret_cast<float*>(smem);            // TTMF_BATCH x 48: F_a, F_b, t rows
  int* sia = reinterpret_cast<int*>(stage + TTMF_BATCH * 48);   // Epad
  int* sib = sia + Epad;                     // Epad (four modes)
  int* sic = sib + Epad;                     // Epad
  float* sv = reinterpret_cast<float*>(sic + Epad);
  int* fst = reinterpret_cast<int*>(sv + Epad);   // Epad + 1: fiber starts, then E
  int* send = fst + Epad + 1;                     // nseg: segment ends (bin-relative)
  unsigned char* sflag = reinterpret_cast<unsigned char*>(send + nseg);   // Epad: segment starts
  const int lane = threadIdx.x;
  {
    const u32x4* la4 = reinterpret_cast<const u32x4*>(A.lay[0] + e0);
    const u32x4* lb4 = reinterpret_cast<const u32x4*>(A.lay[1] + e0);
    const u32x4* lc4 = reinterpret_cast<const u32x4*>(A.lay[A.n_other - 1] + e0);
    const u32x4* v4 = reinterpret_cast<const u32x4*>(A.val + e0);
    for (int i = lane; 4 * i < E; i += 64) {
      reinterpret_cast<u32x4*>(sia)[i] = __builtin_nontemporal_load(la4 + i);
      if (four) reinterpret_cast<u32x4*>(sib)[i] = __builtin_nontemporal_load(lb4 + i);
      reinterpret_cast<u32x4*>(sic)[i] = __builtin_nontemporal_load(lc4 + i);
      reinterpret_cast<u32x4*>(sv)[i] = __builtin_nontemporal_load(v4 + i);
    }
    for (int i = lane; i < nseg; i += 64) send[i] = (int)(A.seg_begin[s0 + i + 1] - e0);
    for (int i = lane; i < E; i += 64) sflag[i] = 0;
  }
  wave_lds_sync();
  for (int i = lane; i < nseg; i += 64) sflag[i == 0 ? 0 : send[i - 1]] = 1;
  wave_lds_sync();
  // fiber starts: a segment start, or a change of the coordinates other than the last
  int nf = 0;
  for (int b0 = 0; b0 < E; b0 += 64) {
    const int e = b0 + lane;
    bool start = false;
    if (e < E) {
      const int ep = e > 0 ? e - 1 : 0;   // e = 0 is a segment start
      start = sflag[e] || sia[e] != sia[ep] || (four && sib[e] != sib[ep]);
    }
    const uint64_t m = __ballot(start);
    if (start) fst[nf + __popcll(m & ((1ull << lane) - 1))] = e;
    nf += __popcll(m);
  }
  if (lane == 0) fst[nf] = E;
  wave_lds_sync();
  const int g = lane >> 2, q = lane & 3;
  const float* Fa = A.F[0];
  const float* Fb = A.F[1];
  const float* Fc = A.F[A.n_other - 1];
  float acc[NP][16];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[p][c] = 0.f;
  int po[NP];    // stage offsets of this lane's pairs: a | (16 + b) << 8, or -1 past K_a K_b
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int pair = lane + 64 * p;
    po[p] = pair < P ? (pair % ka) | ((16 + pair / ka) << 8) : -1;
  }
  int cur = 0;   // segment of the accumulators
  const uintptr_t ybase = reinterpret_cast<uintptr_t>(A.Y);
  const uintptr_t pdiff = reinterpret_cast<uintptr_t>(A.partial) - ybase;
  auto flush = [&]() __attribute__((always_inline)) {
    const int slot = A.seg_slot[s0 + cur];
    const int64_t r64 = slot < 0 ? A.seg_row[s0 + cur] : slot;
    float* dst = reinterpret_cast<float*>(ybase + (slot < 0 ? 0 : pdiff) + (uintptr_t)(r64 * khat) * 4);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int pair = lane + 64 * p;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (c < kc && pair < P) __builtin_nontemporal_store(acc[p][c], dst + pair + P * c);
        acc[p][c] = 0.f;
      }
    }
  };
  auto row4 = [&](const float* F, int r) __attribute__((always_inline)) {
    return *reinterpret_cast<const floatx4_c*>(F + ((size_t)(uint32_t)r * 16 + 4 * q));
  };
  for (int fb = 0; fb < nf; fb += TTMF_BATCH) {
    // phase 1: lane group g forms t of fiber fb + g and stages its rows
    const int f = fb + g;
    if (f < nf) {
      const int fs = fst[f], fe = fst[f + 1];
      const floatx4_c xa = row4(Fa, sia[fs]);
      const floatx4_c xb = four ? row4(Fb, sib[fs]) : floatx4_c{1.f, 1.f, 1.f, 1.f};
      floatx4_c t = {0.f, 0.f, 0.f, 0.f};
      int e = fs;
      for (; e + 4 <= fe; e += 4) {   // four gathers in flight, then their sum in element order
        floatx4_c x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = row4(Fc, sic[e + u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) t += sv[e + u] * x[u];
      }
      for (; e < fe; ++e) t += sv[e] * row4(Fc, sic[e]);
      float* st = stage + g * 48 + 4 * q;
      *reinterpret_cast<floatx4_c*>(st) = xa;
      *reinterpret_cast<floatx4_c*>(st + 16) = xb;
      *reinterpret_cast<floatx4_c*>(st + 32) = t;
    }
    wave_lds_sync();
    // phase 2: the batch's rank-one updates, in fiber order
    const int nb = min(TTMF_BATCH, nf - fb);
    for (int gg = 0; gg < nb; ++gg) {
      const int fs = uni(fst[fb + gg]);
      while (fs >= uni(send[cur])) {   // the fiber belongs to a later segment: the row is complete
        flush();
        ++cur;
      }
      const float* st = stage + gg * 48;
      float tc[16];
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const floatx4_c v = reinterpret_cast<const floatx4_c*>(st + 32)[c4];
        tc[4 * c4] = v[0];
        tc[4 * c4 + 1] = v[1];
        tc[4 * c4 + 2] = v[2];
        tc[4 * c4 + 3] = v[3];
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const float fab = po[p] >= 0 ? st[po[p] & 0xff] * st[po[p] >> 8] : 0.f;
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < kc) acc[p][c] = fmaf(fab, tc[c], acc[p][c]);
      }
    }
    wave_lds_sync();   // the next batch's stage writes follow these reads
  }
  // the last segment (every segment holds at least one element, hence one fiber)
  while (cur < nseg) {
    flush();
    ++cur;
  }
}

// Which shapes the fiber-factored kernel takes: three or four modes, other
// ranks <= 16 with 16-float factor rows.
bool ttm_uses_fiber(int N, const int32_t* K, int n, const int* kp) {
  if (N != 3 && N != 4) return false;
  for (int j = 0; j < N; ++j)
    if (j != n && (K[j] > 16 || kp[j] != 16)) return false;
  return true;
}

// TTM-chain of the whole merged list along mode n with atomics (TK_TTM_ATOMIC).
void ttm_atomic(Ctx* c, int n, float* Y) {
  const ModePlan& pl = c->plan[n];
  TtmAtomicArgs a{};
  for (int j = 0; j < c->N; ++j) {
    a.idx[j] = c->idx_c[j].as<int32_t>();
    a.label[j] = c->plan[j].label.as<int32_t>();
    a.F[j] = c->F32[j].as<float>();
    a.fstride[j] = c->kp32[j];
    a.Kj[j] = c->K[j];
  }
  a.val = c->val_c.as<float>();
  a.N = c->N;
  a.n = n;
  a.row_of = pl.row_of.as<int32_t>();
  a.khat = (int)pl.khat;
  a.m = c->m;
  a.Y = Y;
  const int64_t ny = pl.L_nz * pl.khat;
  if (ny > 0) {
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(ny, 256, 4096)), dim3(256), 0, c->stream, Y, ny);
    TK_CHECK_LAUNCH();
  }
  if (c->m == 0) return;
  if (c->ev_ttm[0]) TK_HIP(hipEventRecord(c->ev_ttm[0], c->stream));
  const int64_t waves = ceil_div(c->m, TTMA_CHUNK);
  const dim3 g((unsigned)ceil_div(waves, 4), (unsigned)ceil_div(pl.khat, TTMV_TILE)), b(256);
  switch (c->N - 1) {
    case 1: hipLaunchKernelGGL(k_ttm_atomic<1>, g, b, 0, c->stream, a); break;
    case 2: hipLaunchKernelGGL(k_ttm_atomic<2>, g, b, 0, c->stream, a); break;
    case 3: hipLaunchKernelGGL(k_ttm_atomic<3>, g, b, 0, c->stream, a); break;
    default: hipLaunchKernelGGL(k_ttm_atomic<0>, g, b, 0, c->stream, a); break;
  }
  TK_CHECK_LAUNCH();
  if (c->ev_ttm[1]) TK_HIP(hipEventRecord(c->ev_ttm[1], c->stream));
}

void ttm_fiber_launch(Ctx* c, const ModePlan& pl, const TtmArgs& a, int N) {
  const int Epad = (int)((pl.E_pad_max + 15) & ~(int64_t)15);
  const size_t lds = 4 * (TTMF_BATCH * 48 + 5 * (size_t)Epad + 1 + (size_t)pl.R_max) + (size_t)Epad + 64;
  TK_REQUIRE(lds <= c->lds_per_block, TK_ERR_UNSUPPORTED, "TTM-chain: bin too large for LDS");
  const int P = N == 4 ? a.Kj[0] * a.Kj[1] : a.Kj[0];
  if (P <= 64)
    hipLaunchKernelGGL(k_ttm_fiber<1>, dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
  else if (P <= 128)
    hipLaunchKernelGGL(k_ttm_fiber<2>, dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
  else
    hipLaunchKernelGGL(k_ttm_fiber<TTMF_MAXP>, dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
  TK_CHECK_LAUNCH();
}

}  // namespace tk
