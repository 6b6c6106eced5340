// TTM-chain along mode n through the Kronecker reformulation (eq. 1,
// Appendix A): row l of Y_(n) is the sum over the elements e of slice l of
// val(e) * (F_a[l_a] (x) F_b[l_b] (x) ...), the first remaining mode fastest.
//
// One workgroup (or one wave) per Lite bin.  A bin holds at most `limit`
// elements and at most ceil(L/P) + 2 distinct slices (Theorem 6.1), so its
// rows of Y live in LDS for the whole bin; after the bin, rows of slices the
// bin owns alone are written straight to Y and rows of slices split over
// several bins go to a partial slot, which the fixup kernels sum in bin order.
// Three kernels:
//   * k_ttm3_mfma: three modes, other ranks <= 16, on the matrix cores;
//   * k_ttm4_mfma: four modes, other ranks <= 16, on the matrix cores;
//   * k_ttm_cols:  every other shape, on the vector ALUs.
// None of them uses atomics: every sum runs in a fixed order.
#include <mutex>

#include "ttm_common.hpp"

namespace tk {

// ---- TTM-chain on the vector ALUs (every shape the matrix-core kernels do not take) -------------
//
// One workgroup of four waves per (Lite bin, tile of TTMV_TILE columns of Y).
// The waves take contiguous quarters of the bin's elements and stream them in
// order; a lane owns TTMV_CPL columns of the tile and accumulates, for the
// current slice, val(e) * prod_j F_j[l_j(e)][digit_j(col)] for each of them
// (the Kronecker column of Appendix A, first remaining mode fastest).  The
// coordinates and values of 64 elements at a time are loaded by the lanes
// together and broadcast with readlane; the gathers of TTMV_U elements are
// issued before their products are added.
// When a slice ends, its row goes to the bin's LDS rows: stored when the slice
// lies inside the wave's quarter, added at once when it began in an earlier
// quarter (no other wave writes that row before the barrier), kept in
// registers when it continues into a later quarter.  After the barrier the
// waves add those kept rows in wave order.  Every sum therefore runs in a
// fixed order: no atomics, bit-identical reruns.
constexpr int TTMV_U = 8;                    // elements whose gathers are in flight together


// NO: number of other modes (1, 2, 3), or 0 for any number up to 7 (runtime).
template <int NO>
__global__ __launch_bounds__(256) void k_ttm_cols(TtmArgs A) {
  extern __shared__ __align__(16) float lds[];
  const int no = NO > 0 ? NO : A.n_other;
  const int64_t bin = xcd_bin(blockIdx.x, gridDim.x);
  const int col0 = blockIdx.y * TTMV_TILE;
  const int khat = A.khat;
  const int64_t e0 = A.bin_ptr[bin];
  const int E = (int)(A.bin_ptr[bin + 1] - e0);
  const int s0 = A.seg_ptr[bin];
  const int nseg = A.seg_ptr[bin + 1] - s0;
  float* rows = lds;                                                   // nseg x TTMV_TILE
  int* send = reinterpret_cast<int*>(rows + (size_t)nseg * TTMV_TILE);  // end of each segment in the bin
  for (int i = threadIdx.x; i < nseg * TTMV_TILE; i += 256) rows[i] = 0.f;
  for (int i = threadIdx.x; i < nseg; i += 256) send[i] = (int)(A.seg_begin[s0 + i + 1] - e0);
  __syncthreads();

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uni(tid >> 6);
  const int Q = (E + 3) >> 2;
  const int cs = min(wave * Q, E), ce = min(cs + Q, E);
  // the lane's columns: Kronecker digits of col = i + K_a (d_1 + K_1 (d_2 + ...))
  int off[TTMV_CPL][7];
  bool colok[TTMV_CPL];
#pragma unroll
  for (int u = 0; u < TTMV_CPL; ++u) {
    const int col = col0 + lane + 64 * u;
    colok[u] = col < khat;
    int rest = colok[u] ? col : 0;
    off[u][0] = rest % A.Kj[0];
    rest /= A.Kj[0];
    for (int j = 1; j < no; ++j) {
      off[u][j] = rest % A.Kj[j];
      rest /= A.Kj[j];
    }
  }
  float acc[TTMV_CPL];
#pragma unroll
  for (int u = 0; u < TTMV_CPL; ++u) acc[u] = 0.f;
  bool has_right = false;
  int right_sg = 0;
  if (cs < ce) {
    int lo = 0, hi = nseg - 1;   // first segment ending after cs
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uni(send[mid]) > cs) hi = mid; else lo = mid + 1;
    }
    int sg = lo;
    int seg_lo = sg > 0 ? uni(send[sg - 1]) : 0;
    int seg_hi = uni(send[sg]);
    auto flush = [&]() __attribute__((always_inline)) {
      const bool left = seg_lo < cs, right = seg_hi > ce;
      float* row = rows + (size_t)sg * TTMV_TILE + lane;
      if (right) {   // the quarter's last slice continues in a later quarter: kept in registers
        has_right = true;
        right_sg = sg;
        return;
      }
#pragma unroll
      for (int u = 0; u < TTMV_CPL; ++u) {
        if (left) row[64 * u] += acc[u];
        else row[64 * u] = acc[u];
        acc[u] = 0.f;
      }
    };
    const float* __restrict__ vv = A.val + e0;
    for (int g = cs; g < ce; g += 64) {
      // coordinates and values of elements g .. g+63, one per lane
      const int ge = min(g + lane, ce - 1);
      const float vl = vv[ge];
      int li[7];
#pragma unroll
      for (int j = 0; j < (NO > 0 ? NO : 7); ++j)
        if (j < no) li[j] = A.lay[j][e0 + ge];
      const int cnt = min(64, ce - g);
      for (int k0 = 0; k0 < cnt; k0 += TTMV_U) {
        float p[TTMV_U][TTMV_CPL];
#pragma unroll
        for (int q = 0; q < TTMV_U; ++q) {
          const int k = min(k0 + q, cnt - 1);
          const float v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, vl), k));
          const int64_t ra = (int64_t)__builtin_amdgcn_readlane(li[0], k) * A.fstride[0];
#pragma unroll
          for (int u = 0; u < TTMV_CPL; ++u) p[q][u] = v * A.F[0][ra + off[u][0]];
#pragma unroll
          for (int j = 1; j < (NO > 0 ? NO : 7); ++j) {
            if (j < no) {
              const int64_t rj = (int64_t)__builtin_amdgcn_readlane(li[j], k) * A.fstride[j];
#pragma unroll
              for (int u = 0; u < TTMV_CPL; ++u) p[q][u] *= A.F[j][rj + off[u][j]];
            }
          }
        }
#pragma unroll
        for (int q = 0; q < TTMV_U; ++q) {
          const int e = g + k0 + q;
          if (k0 + q >= cnt) break;
          if (e >= seg_hi) {   // a new slice starts at element e
            flush();
            ++sg;
            seg_lo = seg_hi;
            seg_hi = uni(send[sg]);
          }
#pragma unroll
          for (int u = 0; u < TTMV_CPL; ++u) acc[u] += p[q][u];
        }
      }
    }
    flush();   // the quarter's last slice
  }
  __syncthreads();
  // rows of slices continued by a later quarter, added in wave order
  for (int w = 0; w < 4; ++w) {
    if (wave == w && has_right) {
      float* row = rows + (size_t)right_sg * TTMV_TILE + lane;
#pragma unroll
      for (int u = 0; u < TTMV_CPL; ++u) row[64 * u] += acc[u];
    }
    __syncthreads();
  }
  // the bin's rows out: owned slices to Y, split slices to their partial slot
  const int tw = min(TTMV_TILE, khat - col0);
  for (int i = threadIdx.x; i < nseg * tw; i += 256) {
    const int sgi = i / tw;
    const int j = i - sgi * tw;
    const float x = rows[(size_t)sgi * TTMV_TILE + j];
    const int slot = A.seg_slot[s0 + sgi];
    if (slot < 0)
      A.Y[(int64_t)A.seg_row[s0 + sgi] * khat + col0 + j] = x;
    else
      A.partial[(int64_t)slot * khat + col0 + j] = x;
  }
}

// ---- three-mode TTM-chain on the matrix cores ----------------------------------------------
//
// For the elements of one slice, Y[row] viewed as K_a x K_b is
//   sum_e (val_e F_a[l_a(e)]) F_b[l_b(e)]^T,
// a contraction over the slice's elements: v_mfma_f32_16x16x4_f32 with lane l
// supplying A[i = l%16][k = l/16] = val_k F_a[l_a(k)][i] and
// B[k = l/16][j = l%16] = F_b[l_b(k)][j] (factor rows padded to 16 floats).
// The result D[4*(l/16)+r][l%16] is Y[row][i + K_a j].
//
// Gathers: the address unit takes a fixed number of lanes per cycle whatever
// the width of each lane's load, so the rows of a block of 16 elements are
// fetched with 16-byte loads (four lanes per 64-byte row, one instruction per
// factor) and turned into the operand layout through a 2 KB LDS tile per wave
// (one 16-byte write and four 4-byte reads per lane and factor).
//
// The layout this kernel streams pads every slice segment to a multiple of 4
// elements (zero values), so one MFMA step (4 consecutive elements) lies in one
// slice: a slice change is a scalar compare per step, with no masking.  Each of
// the four waves streams a contiguous quarter of the bin in blocks of 16
// elements from the LDS copy of the bin.  When a slice ends its accumulator
// goes to the bin's LDS rows; the at most two slices a wave shares with its
// neighbours keep their partial rows in registers and are added to the
// (zeroed) LDS rows in wave order after the main loop.  No atomics: the result
// is deterministic.
constexpr int TTM3_RING = 3;   // blocks of 16 elements with gathers in flight per wave
constexpr int TTM4_RING = 3;   // the same for the four-mode kernel (three 16-byte loads per lane per block)

// Three-mode TTM-chain on the matrix cores, one wave per Lite bin.
//
// The bin's layout (coordinates of the two other modes and values) is staged
// in LDS.  The wave streams it in blocks of 16 elements with a ring of
// TTM3_RING blocks of gathers in flight: four lanes fetch one 64-byte factor
// row with a 16-byte load, and the block's F_a rows (times the value) and F_b
// rows go through a 2 KB LDS tile into the MFMA operand layout.  When a slice
// ends its row goes to the bin's LDS rows; at the end the rows are written to
// Y (or to the partial slots of slices split across bins) with 16-byte stores.
// All slices of a bin belong to its one wave: no barriers and no merging of
// partial rows between waves.  The slice table (end, partial slot, row) is
// held across the lanes, lane i for slice base + i, and read with readlane.
//
// BFM = false: each 4-element step is one v_mfma_f32_16x16x4_f32
// accumulating (val F_a)^T F_b of the current slice (segments are padded to
// multiples of 4, so a step never straddles two slices).
// BFM = true (the precision form): the operands are rounded once to BF16
// (round to nearest even) and a block of 16 elements is one
// v_mfma_f32_16x16x16_bf16 with FP32 accumulation: lane group q = l/16
// supplies the block's four elements 4q .. 4q+3 (one padded quad, so one
// slice).  A block whose quads belong to several slices issues one MFMA per
// slice, the other lane groups' A operands zeroed.
// GATHER: the values come from A.val in another order (A.val_order), each
// fetched on its own while the bin is staged (the completion adjoint's
// residuals, kept in observation order).
//
// The occupancy attribute (51 registers, none spilled) makes the compiler
// keep the accumulator in VGPRs.  Without it the accumulator lives in AGPRs
// and every step copies it out before testing for a slice boundary: four
// moves and a wait on the MFMA result per step, 16 of the 40 vector-ALU
// instructions of a 16-element block (c5 mode 0: 20.2 -> 18.9 ms).
template <bool BFM, bool GATHER = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_ttm3_mfma(TtmArgs A, int Epad) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ka = A.KA, kb = A.KW;
  const int64_t bin = xcd_bin(blockIdx.x, gridDim.x);
  const int64_t e0 = A.bin_ptr[bin];
  const int E = (int)(A.bin_ptr[bin + 1] - e0);   // multiple of 4
  const int s0 = A.seg_ptr[bin];
  const int nseg = A.seg_ptr[bin + 1] - s0;
  if (nseg == 0) return;
  int* sia = reinterpret_cast<int*>(smem);                  // Epad
  int* sib = sia + Epad;                                    // Epad
  float* sv = reinterpret_cast<float*>(sib + Epad);         // Epad
  float* tile = sv + Epad;                                  // 512: F_a and F_b rows of one block
  float* rows = tile + 512;                                 // nseg x khat: the bin's rows of Y
  const int khat = A.khat;
  const int lane = threadIdx.x;
  int base = 0, v_end = 0, v_slot = 0, v_row = 0;
  auto load_segs = [&](int b) __attribute__((always_inline)) {
    const int i = min(b + lane, nseg - 1);
    v_end = (int)(A.seg_begin[s0 + i + 1] - e0);
    v_slot = A.seg_slot[s0 + i];
    v_row = A.seg_row[s0 + i];
    // wait here: the table is then known to be in registers, and the waits
    // inside the ring count only its gathers
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
  };
  const int Ep = (E + 15) & ~15;
  // the layout is read once, four elements per lane (bins start at multiples
  // of four): non-temporal loads keep it from evicting factor rows in L2
  {
    const u32x4* la4 = reinterpret_cast<const u32x4*>(A.lay[0] + e0);
    const u32x4* lb4 = reinterpret_cast<const u32x4*>(A.lay[1] + e0);
    const u32x4* v4 = reinterpret_cast<const u32x4*>(A.val + e0);
    const u32x4* o4 = reinterpret_cast<const u32x4*>(A.val_order + e0);
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int i = lane; 4 * i < Ep; i += 64) {
      const bool ok = 4 * i < E;
      reinterpret_cast<u32x4*>(sia)[i] = ok ? __builtin_nontemporal_load(la4 + i) : z;
      reinterpret_cast<u32x4*>(sib)[i] = ok ? __builtin_nontemporal_load(lb4 + i) : z;
      if constexpr (GATHER) {
        const u32x4 o = ok ? __builtin_nontemporal_load(o4 + i) : u32x4{~0u, ~0u, ~0u, ~0u};
        u32x4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = o[j] == ~0u ? 0u : __float_as_uint(A.val[o[j]]);
        reinterpret_cast<u32x4*>(sv)[i] = v;
      } else {
        reinterpret_cast<u32x4*>(sv)[i] = ok ? __builtin_nontemporal_load(v4 + i) : z;
      }
    }
  }
  load_segs(0);
  wave_lds_sync();
  const int k = lane >> 4, cix = lane & 15;
  const bool bok = cix < kb;
  floatx4_t C = {0.f, 0.f, 0.f, 0.f};
  int sg = 0;
  int seg_hi = __builtin_amdgcn_readlane(v_end, 0);
  auto flush = [&]() __attribute__((always_inline)) {
    if (bok) {
      float* dst = rows + sg * khat + 4 * k + ka * cix;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * k + r < ka) dst[r] = C[r];
    }
    C = floatx4_t{0.f, 0.f, 0.f, 0.f};
  };
  auto next_slice = [&]() __attribute__((always_inline)) {
    ++sg;
    if (sg - base == 64) {
      base = sg;
      load_segs(base);
    }
    seg_hi = __builtin_amdgcn_readlane(v_end, sg - base);
  };
  // Gather of block g: lane l takes element g + l/4, 16-byte quarter l%4 of
  // its F_a and F_b rows.  All lanes load: the factor copies are zero beyond
  // column K, so no predicate (a predicated load would make the in-flight
  // count path dependent).
  struct Blk { u32x4 x, y; float v; };
  auto fetch = [&](int g, Blk& r) __attribute__((always_inline)) {
    const int e = g + (lane >> 2);
    const int ia = sia[e], ib = sib[e];
    r.v = sv[e];
    r.x = *reinterpret_cast<const u32x4*>(A.F[0] + ((size_t)(uint32_t)ia * 16 + 4 * (lane & 3)));
    r.y = *reinterpret_cast<const u32x4*>(A.F[1] + ((size_t)(uint32_t)ib * 16 + 4 * (lane & 3)));
  };
  auto consume = [&](int g, const Blk& r) __attribute__((always_inline)) {
    // the rows of the block into the tile: F_a (times val) at 0, F_b at 256
    reinterpret_cast<float4*>(tile)[lane] =
        make_float4(__uint_as_float(r.x.x) * r.v, __uint_as_float(r.x.y) * r.v, __uint_as_float(r.x.z) * r.v,
                    __uint_as_float(r.x.w) * r.v);
    reinterpret_cast<float4*>(tile + 256)[lane] = make_float4(
        __uint_as_float(r.y.x), __uint_as_float(r.y.y), __uint_as_float(r.y.z), __uint_as_float(r.y.w));
    wave_lds_sync();
    if constexpr (!BFM) {
      // operand layout: step u, lane l reads element 4u + l/16, column l%16
      float xa[4], xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xa[u] = tile[(4 * u + k) * 16 + cix];
        xb[u] = tile[256 + (4 * u + k) * 16 + cix];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gu = g + 4 * u;
        if (gu >= E) break;
        if (gu >= seg_hi) {  // a new slice starts at this step
          flush();
          next_slice();
        }
        C = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u], xb[u], C, 0, 0, 0);
      }
    } else {
      // operand layout: lane l holds elements 4(l/16) .. +3 of the block, column l%16
      const float* ta = tile + (4 * k) * 16 + cix;
      const bf16x4_t xa = bf16x4_of(ta[0], ta[16], ta[32], ta[48]);
      const bf16x4_t xb = bf16x4_of(ta[256], ta[256 + 16], ta[256 + 32], ta[256 + 48]);
      const bf16x4_t zero = {0, 0, 0, 0};
      // runs of quads in one slice: quads [q0, q) belong to slice sg
      int q0 = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gq = g + 4 * q;
        if (gq >= E) break;
        if (gq >= seg_hi) {   // quad q starts a new slice: close the run before it
          if (q > q0) C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(k >= q0 && k < q ? xa : zero, xb, C, 0, 0, 0);
          flush();
          next_slice();
          q0 = q;
        }
      }
      const int qend = min(4, (E - g) >> 2);
      if (qend > q0) C = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(k >= q0 && k < qend ? xa : zero, xb, C, 0, 0, 0);
    }
    wave_lds_sync();   // the next block's write follows these reads
  };
  // Refills are unconditional (clamped to the last staged block): every path
  // then has the same loads in flight and the compiler waits only for the
  // oldest block instead of draining the ring.
  const int last = Ep - 16;
  Blk ring[TTM3_RING];
#pragma unroll
  for (int d = 0; d < TTM3_RING; ++d) {
    fetch(min(16 * d, last), ring[d]);
    __builtin_amdgcn_sched_barrier(0);  // issue order = consumption order
  }
  for (int g = 0; g < E; g += 16 * TTM3_RING) {
#pragma unroll
    for (int d = 0; d < TTM3_RING; ++d) {
      const int gg = g + 16 * d;
      if (gg < E) consume(gg, ring[d]);
      // keep the refill behind the consumption of its slot: hoisted above it,
      // the refill takes fresh registers and the wait at the loop head
      // drains every load in flight
      __builtin_amdgcn_sched_barrier(0);
      fetch(min(gg + 16 * TTM3_RING, last), ring[d]);
    }
  }
  flush();  // the bin's last slice
  wave_lds_sync();
  // The rows out: owned slices to Y, split slices to their partial slot.  The
  // destination is an offset from Y (a select of two pointers would become a
  // private-memory table).
  const uintptr_t ybase = reinterpret_cast<uintptr_t>(A.Y);
  const uintptr_t pdiff = reinterpret_cast<uintptr_t>(A.partial) - ybase;
  if ((khat & 3) == 0) {
    // 16-byte stores, two rows at a time when a row fits half a wave
    const int kq = khat >> 2;
    const bool two = kq <= 32;
    const int half = two ? lane >> 5 : 0, cl = two ? lane & 31 : lane;
    for (int g0 = 0; g0 < nseg; g0 += 64) {
      if (g0 != base) {
        base = g0;
        load_segs(base);
      }
      const int cnt = min(64, nseg - g0);
      for (int i = 0; i < cnt; i += two ? 2 : 1) {
        const int s0i = __builtin_amdgcn_readlane(v_slot, i), r0i = __builtin_amdgcn_readlane(v_row, i);
        const int i1 = min(i + 1, 63);
        const int s1i = __builtin_amdgcn_readlane(v_slot, i1), r1i = __builtin_amdgcn_readlane(v_row, i1);
        const int ii = i + half;
        if (ii >= cnt) continue;
        const int slot = half ? s1i : s0i;
        const int64_t r64 = slot < 0 ? (half ? r1i : r0i) : slot;
        auto* dst = reinterpret_cast<__attribute__((address_space(1))) floatx4_t*>(
            ybase + (slot < 0 ? 0 : pdiff) + (uintptr_t)(r64 * khat) * 4);
        const floatx4_t* src = reinterpret_cast<const floatx4_t*>(rows + (g0 + ii) * khat);
        for (int c4 = cl; c4 < kq; c4 += two ? 32 : 64) __builtin_nontemporal_store(src[c4], dst + c4);
      }
    }
  } else {
    for (int g0 = 0; g0 < nseg; g0 += 64) {
      if (g0 != base) {
        base = g0;
        load_segs(base);
      }
      const int cnt = min(64, nseg - g0);
      for (int i = 0; i < cnt; ++i) {
        const int slot = __builtin_amdgcn_readlane(v_slot, i);
        const int64_t r64 = slot < 0 ? __builtin_amdgcn_readlane(v_row, i) : slot;
        auto* dst = reinterpret_cast<__attribute__((address_space(1))) float*>(
            ybase + (slot < 0 ? 0 : pdiff) + (uintptr_t)(r64 * khat) * 4);
        for (int c = lane; c < khat; c += 64) __builtin_nontemporal_store(rows[(g0 + i) * khat + c], dst + c);
      }
    }
  }
}

// ---- four-mode TTM-chain on the matrix cores ------------------------------------------------
//
// With remaining modes a, b, c (ascending), Y[row] viewed as K_a x (K_b K_c) is
//   sum_e (val_e F_a[l_a(e)])^T (F_b[l_b(e)] (x) F_c[l_c(e)]),
// the three-mode MFMA step with B the Kronecker row of F_b and F_c: column
// j + K_b q of B is F_b[l_b(e)][j] F_c[l_c(e)][q], formed per lane from the LDS
// tile (two reads and a product), and the K_b K_c columns are covered by
// NT = ceil(K_b K_c / 16) output tiles, NT MFMAs per 4-element step (7 for
// ranks 10, against 10 with one tile per c-index).  Column of Y:
// i + K_a (j + K_b q).  The three rows of each element are gathered with
// 16-byte loads into a 3 KB LDS tile per wave, as in the three-mode kernel.
// A wave's slices that continue into a neighbouring wave keep their partial
// rows in registers and are added to the bin's LDS rows in wave order after
// the main loop (no atomics, deterministic).
//
// BFM (the precision form): the operands are rounded once to BF16 and each
// block of 16 elements takes NT v_mfma_f32_16x16x16_bf16 per slice present in
// it (lane group q supplies elements 4q .. 4q+3; other slices' lane groups get
// a zero A operand), FP32 accumulation, as in the three-mode kernel.
template <int NT, bool BFM>
// Up to eight output tiles, at most 170 registers per lane (three waves per
// SIMD): at ranks 10 the BF16 form would otherwise take 194 (166 + 28
// accumulation registers) and run at two waves, 26% slower, and the FP32 form
// drops from 154 to 119.  Wider tiles (a three-wave cap would spill) are held
// to two waves: left unbounded, 14 to 16 tiles take 250 to 284 registers and
// run at one wave (ranks 16, four modes: TTM-chain 53 ms against 31 at two).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 8 ? 3 : 2))) void k_ttm4_mfma(
    TtmArgs A, int Epad, int nseg_pad) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ka = A.Kj[0], kb = A.Kj[1], kbc = A.Kj[1] * A.Kj[2];
  const int64_t bin = xcd_bin(blockIdx.x, gridDim.x);
  const int64_t e0 = A.bin_ptr[bin];
  const int E = (int)(A.bin_ptr[bin + 1] - e0);   // multiple of 4
  const int s0 = A.seg_ptr[bin];
  const int nseg = A.seg_ptr[bin + 1] - s0;
  int* send = reinterpret_cast<int*>(smem);
  int* sslot = send + nseg_pad;
  int* srow = sslot + nseg_pad;
  int* sia = srow + nseg_pad;
  int* sib = sia + Epad;
  int* sic = sib + Epad;
  float* sv = reinterpret_cast<float*>(sic + Epad);
  float* tiles = sv + Epad;                                 // 4 waves x 768: F_a, F_b, F_c rows of one block
  float* rows = tiles + 4 * 768;                            // nseg x khat
  const int khat = A.khat;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uni(tid >> 6);
  for (int i = tid; i < nseg; i += 256) {
    send[i] = (int)(A.seg_begin[s0 + i + 1] - e0);
    sslot[i] = A.seg_slot[s0 + i];
    srow[i] = A.seg_row[s0 + i];
  }
  for (int i = tid; i < nseg * khat; i += 256) rows[i] = 0.f;   // shared rows are summed into
  const int Ep = (E + 15) & ~15;
  {
    const u32x4* la4 = reinterpret_cast<const u32x4*>(A.lay[0] + e0);
    const u32x4* lb4 = reinterpret_cast<const u32x4*>(A.lay[1] + e0);
    const u32x4* lc4 = reinterpret_cast<const u32x4*>(A.lay[2] + e0);
    const u32x4* v4 = reinterpret_cast<const u32x4*>(A.val + e0);
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int i = tid; 4 * i < Ep; i += 256) {
      const bool ok = 4 * i < E;
      reinterpret_cast<u32x4*>(sia)[i] = ok ? __builtin_nontemporal_load(la4 + i) : z;
      reinterpret_cast<u32x4*>(sib)[i] = ok ? __builtin_nontemporal_load(lb4 + i) : z;
      reinterpret_cast<u32x4*>(sic)[i] = ok ? __builtin_nontemporal_load(lc4 + i) : z;
      reinterpret_cast<u32x4*>(sv)[i] = ok ? __builtin_nontemporal_load(v4 + i) : z;
    }
  }
  __syncthreads();

  const int Q = (((E + 3) >> 2) + 15) & ~15;
  const int cs = min(wave * Q, E), ce = min(cs + Q, E);
  const int k = lane >> 4, cix = lane & 15;
  float* tile = tiles + wave * 768;
  floatx4_t C[NT];
  // column 16t + cix of the Kronecker row: tile offsets of its F_b and F_c
  // entries (j = col % K_b, q = col / K_b), packed; columns past K_b K_c read
  // entry 0 and are never written out
  uint32_t pk[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = 16 * t + cix, okc = col < kbc;
    pk[t] = (uint32_t)(256 + (okc ? col % kb : 0)) | ((uint32_t)(512 + (okc ? col / kb : 0)) << 16);
  }
  bool has_right = false;
  int right_sg = 0;
  // row += this lane's part of C, for the merge after the main loop.  Even
  // K_a: the lane's entries of a c-slab pair up into two 8-byte words, read
  // together and then written (one LDS round trip per slab instead of one per
  // entry).
  auto row_acc = [&](float* dst) __attribute__((always_inline)) {
    const bool h0 = 4 * k < ka, h1 = 4 * k + 2 < ka;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (16 * t + cix >= kbc) continue;
      float* p = dst + 4 * k + ka * (16 * t + cix);
      if ((ka & 1) == 0) {
        float2* w = reinterpret_cast<float2*>(p);
        const float2 o0 = h0 ? w[0] : float2{0.f, 0.f}, o1 = h1 ? w[1] : float2{0.f, 0.f};
        if (h0) w[0] = float2{o0.x + C[t][0], o0.y + C[t][1]};
        if (h1) w[1] = float2{o1.x + C[t][2], o1.y + C[t][3]};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * k + r < ka) p[r] += C[t][r];
      }
    }
  };
  if (cs < ce) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uni(send[mid]) > cs) hi = mid; else lo = mid + 1;
    }
    int sg = lo;
    int seg_lo = sg > 0 ? uni(send[sg - 1]) : 0;
    int seg_hi = uni(send[sg]);
#pragma unroll
    for (int t = 0; t < NT; ++t) C[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    auto flush = [&]() __attribute__((always_inline)) {
      const bool left = seg_lo < cs, right = seg_hi > ce;
      if (!left && !right) {
        float* dst = rows + sg * khat;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (16 * t + cix < kbc) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (4 * k + r < ka) dst[4 * k + r + ka * (16 * t + cix)] = C[t][r];
          }
      } else if (right) {   // the last slice of the quarter: stays in C
        has_right = true;
        right_sg = sg;
        return;
      } else {
        // the first slice of the quarter, begun by an earlier wave and ending
        // here: added to its (zeroed) row at once.  No other wave adds to this
        // row before the barrier (the earlier waves add theirs after it), so
        // the order of the sum is fixed.
        float* dst = rows + sg * khat;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (16 * t + cix < kbc) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (4 * k + r < ka) dst[4 * k + r + ka * (16 * t + cix)] += C[t][r];
          }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) C[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    };
    // gather of block g: lane l takes element g + l/4, 16-byte quarter l%4 of
    // its three rows (all lanes load: the copies are zero beyond column K)
    struct Blk { u32x4 x, y, z; float v; };
    auto fetch = [&](int g, Blk& r) __attribute__((always_inline)) {
      const int e = g + (lane >> 2);
      const int ia = sia[e], ib = sib[e], ic = sic[e];
      r.v = sv[e];
      const uint32_t o = 4 * (lane & 3);
      r.x = *reinterpret_cast<const u32x4*>(A.F[0] + ((size_t)(uint32_t)ia * 16 + o));
      r.y = *reinterpret_cast<const u32x4*>(A.F[1] + ((size_t)(uint32_t)ib * 16 + o));
      r.z = *reinterpret_cast<const u32x4*>(A.F[2] + ((size_t)(uint32_t)ic * 16 + o));
    };
    auto consume = [&](int g, const Blk& r) __attribute__((always_inline)) {
      reinterpret_cast<float4*>(tile)[lane] =
          make_float4(__uint_as_float(r.x.x) * r.v, __uint_as_float(r.x.y) * r.v, __uint_as_float(r.x.z) * r.v,
                      __uint_as_float(r.x.w) * r.v);
      reinterpret_cast<u32x4*>(tile + 256)[lane] = r.y;
      reinterpret_cast<u32x4*>(tile + 512)[lane] = r.z;
      wave_lds_sync();
      if constexpr (!BFM) {
        float xa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xa[u] = tile[(4 * u + k) * 16 + cix];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int gu = g + 4 * u;
          if (gu >= ce) break;
          if (gu >= seg_hi) {
            flush();
            ++sg;
            seg_lo = seg_hi;
            seg_hi = uni(send[sg]);
          }
          const float* te = tile + (4 * u + k) * 16;
#pragma unroll
          for (int t = 0; t < NT; ++t)
            C[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u], te[pk[t] & 0xffffu] * te[pk[t] >> 16], C[t], 0, 0, 0);
        }
      } else {
        // lane l holds elements 4(l/16) .. +3 of the block
        const float* tq = tile + (4 * k) * 16;
        const bf16x4_t xa = bf16x4_of(tq[cix], tq[16 + cix], tq[32 + cix], tq[48 + cix]);
        bf16x4_t xb[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const uint32_t ob = pk[t] & 0xffffu, oc = pk[t] >> 16;
          xb[t] = bf16x4_of(tq[ob] * tq[oc], tq[16 + ob] * tq[16 + oc], tq[32 + ob] * tq[32 + oc],
                            tq[48 + ob] * tq[48 + oc]);
        }
        const bf16x4_t zero = {0, 0, 0, 0};
        int q0 = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int gq = g + 4 * q;
          if (gq >= ce) break;
          if (gq >= seg_hi) {   // quad q starts a new slice: close the run before it
            if (q > q0) {
              const bf16x4_t a = k >= q0 && k < q ? xa : zero;
#pragma unroll
              for (int t = 0; t < NT; ++t) C[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb[t], C[t], 0, 0, 0);
            }
            flush();
            ++sg;
            seg_lo = seg_hi;
            seg_hi = uni(send[sg]);
            q0 = q;
          }
        }
        const int qend = min(4, (ce - g) >> 2);
        if (qend > q0) {
          const bf16x4_t a = k >= q0 && k < qend ? xa : zero;
#pragma unroll
          for (int t = 0; t < NT; ++t) C[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb[t], C[t], 0, 0, 0);
        }
      }
      wave_lds_sync();   // the next block's write follows these reads
    };
    // refills unconditional (clamped to the last staged block) and kept in
    // issue order, so the wait before each block is for its own loads only
    const int last = Ep - 16;
    Blk ring[TTM4_RING];
#pragma unroll
    for (int d = 0; d < TTM4_RING; ++d) {
      fetch(min(cs + 16 * d, last), ring[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
    static_assert(TTM4_RING == 3, "the ring steps below are written out for three blocks");
    auto step = [&](int gg, Blk& r) __attribute__((always_inline)) {
      consume(gg, r);
      __builtin_amdgcn_sched_barrier(0);
      fetch(min(gg + 16 * TTM4_RING, last), r);
    };
    for (int g = cs; g < ce; g += 16 * TTM4_RING) {
      step(g, ring[0]);
      step(g + 16, ring[1]);
      step(g + 32, ring[2]);
    }
    flush();
  }
  __syncthreads();
  // partial rows of slices continued by a later wave, added in wave order
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wave == w && has_right) row_acc(rows + right_sg * khat);
  }
  __syncthreads();
  // the bin's rows out, one row per wave at a time, 16-byte stores when the
  // row length allows; the destination is an offset from Y (a select of two
  // pointers would become a private-memory table)
  const uintptr_t ybase = reinterpret_cast<uintptr_t>(A.Y);
  const uintptr_t pdiff = reinterpret_cast<uintptr_t>(A.partial) - ybase;
  for (int sgi = wave; sgi < nseg; sgi += 4) {
    const int slot = uni(sslot[sgi]);
    const int64_t r64 = slot < 0 ? uni(srow[sgi]) : slot;
    const uintptr_t rowp = ybase + (slot < 0 ? 0 : pdiff) + (uintptr_t)(r64 * khat) * 4;
    if ((khat & 3) == 0) {
      const floatx4_t* src = reinterpret_cast<const floatx4_t*>(rows + sgi * khat);
      auto* dst = reinterpret_cast<__attribute__((address_space(1))) floatx4_t*>(rowp);
      for (int c4 = lane; c4 < (khat >> 2); c4 += 64) __builtin_nontemporal_store(src[c4], dst + c4);
    } else {
      auto* dst = reinterpret_cast<__attribute__((address_space(1))) float*>(rowp);
      for (int c = lane; c < khat; c += 64) __builtin_nontemporal_store(rows[sgi * khat + c], dst + c);
    }
  }
}

// Sum the partial rows of every split slice in bin order, along a tree of
// fixed shape: each level adds runs of at most FIX_CHUNK consecutive rows of
// one slice into new rows, then each slice's last rows go to Y (deterministic,
// and parallel however many bins a slice is split over).
// Sum of the at most FIX_CHUNK partial rows [a, b) of buf, column c, in row
// order: the loads of each batch of 32 rows are issued before its first add
// (the rows are independent), then the adds run in the fixed order.
__device__ __forceinline__ float fix_sum(const float* __restrict__ buf, int a, int b, int khat, int c) {
  float s = 0.f;
  for (int a0 = a; a0 < b; a0 += 32) {
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = a0 + i < b ? buf[(int64_t)(a0 + i) * khat + c] : 0.f;
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (a0 + i < b) s += v[i];
  }
  return s;
}
// One wave per run of rows (four runs per workgroup): lane l sums columns
// l, l + 64, ... of rows [a, b) of buf in row order into out; with khat a
// multiple of 4, four columns per lane through 16-byte loads.  Each column's
// adds keep fix_sum's order, so the result does not depend on the form.
__device__ __forceinline__ void fix_sum_wave(const float* __restrict__ buf, int a, int b, int khat,
                                             float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  if ((khat & 3) == 0) {
    const int kq = khat >> 2;
    for (int c4 = lane; c4 < kq; c4 += 64) {
      floatx4_t s = {0.f, 0.f, 0.f, 0.f};
      for (int a0 = a; a0 < b; a0 += 8) {
        floatx4_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          v[i] = a0 + i < b ? reinterpret_cast<const floatx4_t*>(buf + (int64_t)(a0 + i) * khat)[c4]
                            : floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (a0 + i < b) s += v[i];
      }
      reinterpret_cast<floatx4_t*>(out)[c4] = s;
    }
  } else {
    for (int c = lane; c < khat; c += 64) out[c] = fix_sum(buf, a, b, khat, c);
  }
}
constexpr int FIX_WAVES = 4;   // runs per workgroup
__global__ __launch_bounds__(64 * FIX_WAVES) void k_fixup_level(const int32_t* __restrict__ lo,
                                                                const int32_t* __restrict__ hi, int64_t first,
                                                                int64_t nl, float* __restrict__ buf, int khat) {
  const int64_t t = (int64_t)blockIdx.x * FIX_WAVES + (threadIdx.x >> 6);
  if (t >= nl) return;
  fix_sum_wave(buf, lo[t], hi[t], khat, buf + (first + t) * khat);
}
__global__ __launch_bounds__(64 * FIX_WAVES) void k_fixup(const int32_t* __restrict__ bad_row,
                                                          const int32_t* __restrict__ fin, int64_t nbad,
                                                          const float* __restrict__ buf, int khat,
                                                          float* __restrict__ Y) {
  const int64_t k = (int64_t)blockIdx.x * FIX_WAVES + (threadIdx.x >> 6);
  if (k >= nbad) return;
  fix_sum_wave(buf, fin[k], fin[nbad + k], khat, Y + (int64_t)bad_row[k] * khat);
}

// ---- dispatch -----------------------------------------------------------------------------------

// Three-mode tensors with both remaining ranks <= 16 and 16-float factor rows
// take the matrix-core kernel.
bool ttm_uses_mfma(int N, const int32_t* K, int n, const int* kp) {
  if (N != 3) return false;
  for (int j = 0; j < 3; ++j)
    if (j != n && (K[j] > 16 || kp[j] != 16)) return false;
  return true;
}

// The three-mode matrix-core kernel is the one ttm_run launches for mode n.
bool ttm_takes_mfma3(const Ctx* c, const ModePlan& pl, int N, int n, const int32_t* K, const int* kp) {
  if (pl.whole_slices || c->opt.ttm_kernel == TK_TTM_VECTOR) return false;
  if (c->opt.ttm_kernel == TK_TTM_FIBER && ttm_uses_fiber(N, K, n, kp)) return false;
  return ttm_uses_mfma(N, K, n, kp);
}

// Four-mode tensors with all remaining ranks <= 16 and 16-float factor rows
// take the four-mode matrix-core kernel.
bool ttm_uses_mfma4(int N, const int32_t* K, int n, const int* kp) {
  if (N != 4) return false;
  for (int j = 0; j < 4; ++j)
    if (j != n && (K[j] > 16 || kp[j] != 16)) return false;
  return true;
}

// Columns of Y a bin keeps in LDS per launch: whole rows for the matrix-core
// kernels, one tile of TTMV_TILE columns for the vector-ALU kernel.
int ttm_tile_width(int N, const int32_t* K, int n) {
  int kp16[8];
  for (int j = 0; j < N; ++j) kp16[j] = K[j] <= 16 ? 16 : 0;
  int kh = 1;
  for (int j = 0; j < N; ++j)
    if (j != n) kh *= K[j];
  if (ttm_uses_mfma(N, K, n, kp16) || ttm_uses_mfma4(N, K, n, kp16)) return kh;
  return TTMV_TILE;
}

// Default elements per Lite bin for the kernel mode n takes: the one-wave
// three-mode kernel wants small bins (one bin's start-up latency is covered by
// the others on the CU; 384-512 elements measured best, 448 by a little), the
// four-mode kernel's four waves share 1024, the one-wave fiber-factored
// kernel takes 512, and the vector-ALU kernel amortises its row tiles over 4096.
int64_t ttm_default_bin_nnz(int N, const int32_t* K, int n, int kernel) {
  int kp16[8];
  for (int j = 0; j < N; ++j) kp16[j] = K[j] <= 16 ? 16 : 0;
  if (kernel == TK_TTM_FIBER && ttm_uses_fiber(N, K, n, kp16)) return 512;   // one wave per bin
  if (ttm_uses_mfma(N, K, n, kp16)) return 448;
  if (ttm_uses_mfma4(N, K, n, kp16)) return 1024;
  return 4096;
}

int ttm_rows_cap(Ctx* c, int64_t tile_w) {
  // LDS budget for a bin's rows: about 40 KB so three bins share a CU, never
  // past the hardware limit.  Wide rows (the four-mode matrix-core kernel,
  // Khat >= 512) leave room for that kernel's staging (16 bytes per element)
  // and tiles (12 KB): 24 KB of rows keep three of its bins on a CU.
  int64_t budget = tile_w >= 512 ? 24576 : 40960;
  if ((int64_t)c->lds_per_block < budget) budget = (int64_t)c->lds_per_block;
  int64_t cap = budget / (4 * tile_w + 4);
  if (cap > 512) cap = 512;
  if (cap < 3) cap = 3;
  return (int)cap;
}

// TTM-chain of the elements of plan `pl` along mode n with FP32 factor copies
// F32[j] (row stride kp[j]) of every mode j != n; values are the plan's layout values.
void ttm_run(Ctx* c, const ModePlan& pl, int N, int n, const int32_t* K, const float* const* F32, const int* kp,
             const float* lay_val, int64_t m, float* Y, bool bf16, float* partial, const uint32_t* val_order) {
  TtmArgs a{};
  a.bin_ptr = pl.bin_pptr.as<int64_t>();
  a.seg_ptr = pl.seg_ptr.as<int32_t>();
  a.seg_row = pl.seg_row.as<int32_t>();
  a.seg_begin = pl.seg_pbegin.as<int64_t>();
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
  a.KA = a.Kj[0];
  a.KW = prod;
  a.khat = (int)pl.khat;
  a.val = lay_val;
  a.val_order = val_order;
  a.Y = Y;
  if (!partial) {
    ensure(c, c->partial, sizeof(float) * (size_t)std::max<int64_t>(pl.fix_rows, 1) * (size_t)pl.khat);
    partial = c->partial.as<float>();
  }
  a.partial = partial;
  a.P = pl.P;
  if (m == 0) {
    // a fill kernel, not a memset node, so the call can be captured into a graph
    const int64_t ny = pl.L_nz * pl.khat;
    if (ny > 0) {
      hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(ny, 256, 4096)), dim3(256), 0, c->stream, Y, ny);
      TK_CHECK_LAUNCH();
    }
    return;
  }
  if (c->ev_ttm[0]) TK_HIP(hipEventRecord(c->ev_ttm[0], c->stream));
  const bool vector_only = pl.whole_slices || c->opt.ttm_kernel == TK_TTM_VECTOR;
  TK_REQUIRE(!val_order || ttm_takes_mfma3(c, pl, N, n, K, kp), TK_ERR_UNSUPPORTED,
             "TTM-chain: gathered values need the three-mode matrix-core kernel");
  if (!pl.whole_slices && c->opt.ttm_kernel == TK_TTM_FIBER && ttm_uses_fiber(N, K, n, kp)) {
    ttm_fiber_launch(c, pl, a, N);
  } else if (!vector_only && ttm_uses_mfma(N, K, n, kp)) {
    const int Epad = (int)((pl.E_pad_max + 15) & ~(int64_t)15);
    const size_t lds = 12 * (size_t)Epad + sizeof(float) * 512 + sizeof(float) * (size_t)pl.R_max * (size_t)pl.khat;
    TK_REQUIRE(lds <= c->lds_per_block, TK_ERR_UNSUPPORTED, "TTM-chain: bin too large for LDS");
    if (val_order) {
      TK_REQUIRE(!bf16, TK_ERR_UNSUPPORTED, "TTM-chain: gathered values take the FP32 tiles");
      hipLaunchKernelGGL((k_ttm3_mfma<false, true>), dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
    } else if (bf16) {
      hipLaunchKernelGGL(k_ttm3_mfma<true>, dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
    } else {
      hipLaunchKernelGGL(k_ttm3_mfma<false>, dim3((unsigned)pl.P), dim3(64), lds, c->stream, a, Epad);
    }
    TK_CHECK_LAUNCH();
  } else if (!vector_only && ttm_uses_mfma4(N, K, n, kp)) {
    const int Epad = (int)((pl.E_pad_max + 15) & ~(int64_t)15);
    const int nseg_pad = (int)((pl.R_max + 3) & ~(int64_t)3);
    const size_t lds = 3 * sizeof(int) * (size_t)nseg_pad + 16 * (size_t)Epad + sizeof(float) * 4 * 768 +
                       sizeof(float) * (size_t)pl.R_max * (size_t)pl.khat;
    TK_REQUIRE(lds <= c->lds_per_block, TK_ERR_UNSUPPORTED, "TTM-chain: bin too large for LDS");
    const dim3 g((unsigned)pl.P), b(256);
    switch ((a.Kj[1] * a.Kj[2] + 15) / 16) {
#define TK_TTM4_CASE(NT)                                                                         \
      case NT:                                                                                   \
        if (bf16)                                                                                \
          hipLaunchKernelGGL((k_ttm4_mfma<NT, true>), g, b, lds, c->stream, a, Epad, nseg_pad);  \
        else                                                                                     \
          hipLaunchKernelGGL((k_ttm4_mfma<NT, false>), g, b, lds, c->stream, a, Epad, nseg_pad); \
        break;
      TK_TTM4_CASE(1) TK_TTM4_CASE(2) TK_TTM4_CASE(3) TK_TTM4_CASE(4) TK_TTM4_CASE(5) TK_TTM4_CASE(6)
      TK_TTM4_CASE(7) TK_TTM4_CASE(8) TK_TTM4_CASE(9) TK_TTM4_CASE(10) TK_TTM4_CASE(11) TK_TTM4_CASE(12)
      TK_TTM4_CASE(13) TK_TTM4_CASE(14) TK_TTM4_CASE(15) TK_TTM4_CASE(16)
#undef TK_TTM4_CASE
      default: fail(TK_ERR_UNSUPPORTED, "four-mode TTM: rank above 16");
    }
    TK_CHECK_LAUNCH();
  } else {
    const size_t lds = (size_t)pl.R_max * (sizeof(float) * TTMV_TILE + sizeof(int)) + 4;
    TK_REQUIRE(lds <= c->lds_per_block, TK_ERR_UNSUPPORTED, "TTM-chain: bin too large for LDS");
    const dim3 g((unsigned)pl.P, (unsigned)ceil_div(pl.khat, TTMV_TILE)), b(256);
    switch (no) {
      case 1: hipLaunchKernelGGL(k_ttm_cols<1>, g, b, lds, c->stream, a); break;
      case 2: hipLaunchKernelGGL(k_ttm_cols<2>, g, b, lds, c->stream, a); break;
      case 3: hipLaunchKernelGGL(k_ttm_cols<3>, g, b, lds, c->stream, a); break;
      default: hipLaunchKernelGGL(k_ttm_cols<0>, g, b, lds, c->stream, a); break;
    }
    TK_CHECK_LAUNCH();
  }
  if (c->ev_ttm[1]) TK_HIP(hipEventRecord(c->ev_ttm[1], c->stream));
  if (pl.n_bad > 0) {
    float* buf = partial;
    int64_t first = pl.n_slots, off = 0;
    for (int64_t nl : pl.fix_n) {
      const int32_t* lohi = pl.fix_lohi.as<int32_t>() + off;
      hipLaunchKernelGGL(k_fixup_level, dim3((unsigned)ceil_div(nl, FIX_WAVES)), dim3(64 * FIX_WAVES), 0, c->stream,
                         lohi, lohi + nl, first, nl, buf, (int)pl.khat);
      TK_CHECK_LAUNCH();
      first += nl;
      off += 2 * nl;
    }
    hipLaunchKernelGGL(k_fixup, dim3((unsigned)ceil_div(pl.n_bad, FIX_WAVES)), dim3(64 * FIX_WAVES), 0, c->stream,
                       pl.bad_row.as<int32_t>(),
                       pl.fix_fin.as<int32_t>(), pl.n_bad, buf, (int)pl.khat, Y);
    TK_CHECK_LAUNCH();
  }
}

// bf16: the precision form's BF16 Kronecker tiles on the matrix cores (where a
// matrix-core kernel runs, the FP32 factor rows rounded in registers; other
// shapes stay FP32).
void ttm_chain(Ctx* c, int n, float* Y, bool bf16, float* partial) {
  if (c->opt.ttm_kernel == TK_TTM_ATOMIC) {
    ttm_atomic(c, n, Y);
    return;
  }
  const float* F[8];
  for (int j = 0; j < c->N; ++j) F[j] = c->F32[j].as<float>();
  ttm_run(c, c->plan[n], c->N, n, c->K, F, c->kp32, c->plan[n].lay_val.as<float>(), c->m, Y, bf16, partial);
}

// ---- the allocation-free TTM-chain -------------------------------------------------------------
//
// tk_ttm_chain_noalloc keeps the partial rows of split slices in this array
// instead of a context buffer.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in symbol): its device address is
// taken once per device, at context creation, and kept below.
static __device__ __align__(256) float scratch[TK_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};
}  // namespace

void noalloc_scratch_init(int device) {
  TK_REQUIRE(device >= 0 && device < 64, TK_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  // the caller has made `device` current
  TK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  TK_REQUIRE(ptr != nullptr, TK_ERR_DEVICE, "no device address for the TTM-chain scratch array");
  g_scratch_ptr[device] = ptr;
}

void ttm_chain_noalloc(Ctx* c, int n, float* Y) {
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ptr = g_scratch_ptr[c->device];
  }
  TK_REQUIRE(ptr != nullptr, TK_ERR_STATE, "scratch array not set up on this device");
  const ModePlan& pl = c->plan[n];
  const int64_t need = std::max<int64_t>(pl.fix_rows, 1) * pl.khat * (int64_t)sizeof(float);
  TK_REQUIRE(need <= (int64_t)TK_NOALLOC_SCRATCH_BYTES, TK_ERR_UNSUPPORTED,
             "tk_ttm_chain_noalloc: mode " + std::to_string(n) + " needs " + std::to_string(need) +
                 " bytes of partial rows for its split slices, above the " +
                 std::to_string((long long)TK_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
  ttm_chain(c, n, Y, c->opt.prec == TK_BF16, static_cast<float*>(ptr));
}

}  // namespace tk
