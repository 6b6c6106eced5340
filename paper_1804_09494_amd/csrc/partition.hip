// The Lite scheme (Section 6, Lite figure) as a partition of one mode's
// elements over GPU workgroups ("bins"), plus the mode-sorted copy of the
// tensor the TTM-chain streams.
//
// The sequential two-stage procedure is evaluated with parallel prefix
// operations that give the same assignment element for element:
//
//  * slices are the nonempty mode-n index values; they are sorted by
//    (cardinality, id) ascending; t = 0, 1, ... is the sorted position;
//  * stage 1 gives slice t to bin t mod P while every bin stays within
//    limit = ceil(m/P).  With H(t) = sum of sizes of the earlier slices of the
//    same residue class, stage 1 ends at the first t where H(t) + s_t > limit.
//    One thread per residue class walks its class to find its first such t;
//    the minimum over classes is that first t (every earlier slice was placed,
//    so each class's running sum is exactly its bin's load);
//  * stage 2 fills each bin to the limit in bin order, splitting slices over
//    consecutive bins: this is a pour of the remaining slices (in order, each
//    slice's elements in canonical order) into the concatenation of the bins'
//    gaps g_p = limit - load_p.  The element at pour offset x lands in the bin
//    b = min{p : G_p > x}, G the inclusive prefix sum of the gaps (a bin with
//    gap 0 receives nothing, as in the procedure);
//  * layout: bins in order; inside a bin its stage-1 slices in sorted order,
//    then its stage-2 pieces in pour order; inside a piece, canonical order.
//
// Every quantity is an integer, so the result is bit-identical to the
// sequential procedure.
#include "common.hpp"

namespace tk {

__global__ void k_iota_u32b(uint32_t* __restrict__ out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)i;
}

__global__ void k_copy_key(const int32_t* __restrict__ idx, uint32_t* __restrict__ key, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = (uint32_t)idx[i];
}

// Slice boundaries in the slice-sorted element order: start/count per slice id.
__global__ void k_slice_bounds(const uint32_t* __restrict__ skey, int64_t m, int64_t* __restrict__ start,
                               int64_t* __restrict__ count) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    uint32_t k = skey[s];
    if (s == 0 || skey[s - 1] != k) start[k] = s;
    if (s == m - 1 || skey[s + 1] != k) count[k] = s + 1;  // end for now; converted below
  }
}

__global__ void k_finish_counts(const int64_t* __restrict__ start, int64_t* __restrict__ count,
                                int32_t* __restrict__ nonempty, int64_t L) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < L; l += (int64_t)gridDim.x * blockDim.x) {
    int64_t end = count[l];
    int64_t c = end > 0 ? end - start[l] : 0;
    count[l] = c;
    nonempty[l] = c > 0;
  }
}

// Compact nonempty slices (ascending id): row_slice[row] = l, key = count, val = l.
__global__ void k_compact_slices(const int64_t* __restrict__ count, const int32_t* __restrict__ row_of, int64_t L,
                                 int32_t* __restrict__ row_slice, uint32_t* __restrict__ ckey,
                                 uint32_t* __restrict__ cval) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < L; l += (int64_t)gridDim.x * blockDim.x) {
    int64_t c = count[l];
    if (c > 0) {
      int32_t r = row_of[l];
      row_slice[r] = (int32_t)l;
      ckey[r] = (uint32_t)c;
      cval[r] = (uint32_t)l;
    }
  }
}

// rank_of[slice id] = sorted position t; size_t[t] as int64.
__global__ void k_rank_of(const uint32_t* __restrict__ osize, const uint32_t* __restrict__ oslice, int64_t Lnz,
                          int32_t* __restrict__ rank_of, int64_t* __restrict__ size64) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < Lnz; t += (int64_t)gridDim.x * blockDim.x) {
    rank_of[oslice[t]] = (int32_t)t;
    size64[t] = (int64_t)osize[t];
  }
}

// Storage label of every index of this mode: nonempty slices by descending
// size (rank from the (size, id) sort read backwards), empty slices after them.
__global__ void k_labels(const int32_t* __restrict__ rank_of, const int32_t* __restrict__ row_of,
                         const int64_t* __restrict__ count, int64_t L, int64_t Lnz, int32_t* __restrict__ label) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < L; l += (int64_t)gridDim.x * blockDim.x)
    label[l] = count[l] > 0 ? (int32_t)(Lnz - 1 - rank_of[l]) : (int32_t)(Lnz + l - row_of[l]);
}

__global__ void k_apply_labels(int32_t* __restrict__ lay, int64_t m, const int32_t* __restrict__ label) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    lay[i] = label[lay[i]];
}

// Stage 1, pass A: first t of residue class p where the class's running load + s_t > limit.
__global__ void k_stage1_first_fail(const int64_t* __restrict__ size, int64_t Lnz, int64_t P, int64_t limit,
                                    int64_t* __restrict__ cand) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t h = 0, first = Lnz;
    for (int64_t t = p; t < Lnz; t += P) {
      int64_t s = size[t];
      if (h + s > limit) { first = t; break; }
      h += s;
    }
    cand[p] = first;
  }
}

// Stage 1, pass B: offsets of stage-1 slices inside their bin, loads, counts, gaps.
__global__ void k_stage1_place(const int64_t* __restrict__ size, int64_t t_hat, int64_t P, int64_t limit,
                               int64_t* __restrict__ off1, int64_t* __restrict__ load1, int64_t* __restrict__ cnt1,
                               int64_t* __restrict__ gap) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t h = 0, k = 0;
    for (int64_t t = p; t < t_hat; t += P) {
      off1[t] = h;
      h += size[t];
      ++k;
    }
    load1[p] = h;
    cnt1[p] = k;
    gap[p] = limit - h;
  }
}

// first index i in [0, n) with a[i] > x (n if none)
__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* __restrict__ a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Final loads and segment counts per bin.
//   Gin = inclusive prefix of gaps; X = exclusive prefix of stage-2 sizes (n2+1 entries, X[n2] = M2).
__global__ void k_bin_loads(const int64_t* __restrict__ load1, const int64_t* __restrict__ cnt1,
                            const int64_t* __restrict__ gap, const int64_t* __restrict__ Gin,
                            const int64_t* __restrict__ X, int64_t n2, int64_t M2, int64_t P,
                            int64_t* __restrict__ load, int64_t* __restrict__ nseg) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = Gin[p] - gap[p], hi = Gin[p];
    if (lo > M2) lo = M2;
    if (hi > M2) hi = M2;
    int64_t poured = hi - lo;
    int64_t k = cnt1[p];
    if (poured > 0) {
      int64_t u0 = upper_bound_i64(X + 1, n2, lo);        // slice containing offset lo
      int64_t u1 = upper_bound_i64(X + 1, n2, hi - 1);    // slice containing offset hi-1
      k += u1 - u0 + 1;
    }
    load[p] = load1[p] + poured;
    nseg[p] = k;
  }
}

// Fill the segment table, one thread per bin.
__global__ void k_fill_segments(const int64_t* __restrict__ bin_ptr, const int64_t* __restrict__ seg_first,
                                const int64_t* __restrict__ load1, const int64_t* __restrict__ gap,
                                const int64_t* __restrict__ Gin, const int64_t* __restrict__ X,
                                const int64_t* __restrict__ off1, const uint32_t* __restrict__ oslice,
                                const int32_t* __restrict__ row_of, int64_t t_hat, int64_t n2, int64_t M2, int64_t P,
                                int32_t* __restrict__ seg_ptr, int32_t* __restrict__ seg_row,
                                int64_t* __restrict__ seg_begin, int32_t* __restrict__ seg_u,
                                int64_t* __restrict__ first_seg, int64_t* __restrict__ last_seg) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = seg_first[p];
    seg_ptr[p] = (int32_t)k;
    const int64_t base = bin_ptr[p];
    for (int64_t t = p; t < t_hat; t += P) {
      seg_row[k] = row_of[oslice[t]];
      seg_begin[k] = base + off1[t];
      seg_u[k] = -1;
      ++k;
    }
    int64_t lo = Gin[p] - gap[p], hi = Gin[p];
    if (lo > M2) lo = M2;
    if (hi > M2) hi = M2;
    if (hi > lo) {
      int64_t u0 = upper_bound_i64(X + 1, n2, lo);
      int64_t u1 = upper_bound_i64(X + 1, n2, hi - 1);
      for (int64_t u = u0; u <= u1; ++u) {
        int64_t xs = X[u] > lo ? X[u] : lo;
        seg_row[k] = row_of[oslice[t_hat + u]];
        seg_begin[k] = base + load1[p] + (xs - lo);
        seg_u[k] = (int32_t)u;
        if (X[u] >= lo) first_seg[u] = k;          // slice starts in this bin
        if (X[u + 1] <= hi) last_seg[u] = k;       // slice ends in this bin
        ++k;
      }
    }
  }
}

__global__ void k_seg_bad(const int32_t* __restrict__ seg_u, const int64_t* __restrict__ first_seg,
                          const int64_t* __restrict__ last_seg, int64_t S, int32_t* __restrict__ bad) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < S; k += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = seg_u[k];
    bad[k] = (u >= 0 && first_seg[u] != last_seg[u]) ? 1 : 0;
  }
}

__global__ void k_seg_slot(const int32_t* __restrict__ bad, const int32_t* __restrict__ slot_scan, int64_t S,
                           int32_t* __restrict__ seg_slot) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < S; k += (int64_t)gridDim.x * blockDim.x)
    seg_slot[k] = bad[k] ? slot_scan[k] : -1;
}

// Bad-slice table for the fixup: row and slot range of every split stage-2 slice.
__global__ void k_bad_table(const int64_t* __restrict__ first_seg, const int64_t* __restrict__ last_seg,
                            const int32_t* __restrict__ seg_slot, const int32_t* __restrict__ seg_row,
                            const int32_t* __restrict__ badslice_scan, int64_t n2, int32_t* __restrict__ bad_row,
                            int32_t* __restrict__ bad_slot) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n2; u += (int64_t)gridDim.x * blockDim.x) {
    int64_t f = first_seg[u], l = last_seg[u];
    if (f != l) {
      int32_t k = badslice_scan[u];
      bad_row[k] = seg_row[f];
      bad_slot[k] = seg_slot[f];
      bad_slot[k + 1] = seg_slot[l] + 1;  // consecutive slots; the last entry closes the table
    }
  }
}

__global__ void k_is_bad_slice(const int64_t* __restrict__ first_seg, const int64_t* __restrict__ last_seg,
                               int64_t n2, int32_t* __restrict__ flag) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n2; u += (int64_t)gridDim.x * blockDim.x)
    flag[u] = first_seg[u] != last_seg[u];
}

struct IdxIn {
  const int32_t* p[8];
};
struct IdxOut {
  int32_t* p[8];
};

// Layout scatter: destination of every element, and its other-mode
// coordinates and value.  `dest` is the (exported, unpadded) layout position;
// the TTM-chain copy uses the padded position of the same element inside its
// segment.
__device__ __forceinline__ int64_t padded_pos(int64_t dest, int64_t bin, const int32_t* __restrict__ seg_ptr,
                                              const int64_t* __restrict__ seg_begin,
                                              const int64_t* __restrict__ seg_pbegin) {
  int lo = seg_ptr[bin], hi = seg_ptr[bin + 1] - 1;  // last segment with seg_begin <= dest
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_begin[mid] <= dest) lo = mid; else hi = mid - 1;
  }
  return seg_pbegin[lo] + (dest - seg_begin[lo]);
}

__global__ void k_layout(const uint32_t* __restrict__ skey, const uint32_t* __restrict__ sperm, int64_t m,
                         const int64_t* __restrict__ sstart, const int32_t* __restrict__ rank_of,
                         const int64_t* __restrict__ off1, const int64_t* __restrict__ X,
                         const int64_t* __restrict__ Gin, const int64_t* __restrict__ gap,
                         const int64_t* __restrict__ load1, const int64_t* __restrict__ bin_ptr, int64_t t_hat,
                         int64_t P, const int32_t* __restrict__ seg_ptr, const int64_t* __restrict__ seg_begin,
                         const int64_t* __restrict__ seg_pbegin, IdxIn in_idx, int n_other,
                         const float* __restrict__ vals, IdxOut out_idx, float* __restrict__ out_val,
                         uint32_t* __restrict__ elem_order, uint32_t* __restrict__ order_pad) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    uint32_t l = skey[s];
    uint32_t e = sperm[s];
    int64_t r = s - sstart[l];
    int64_t t = rank_of[l];
    int64_t dest, bin;
    if (t < t_hat) {
      bin = t % P;
      dest = bin_ptr[bin] + off1[t] + r;
    } else {
      int64_t x = X[t - t_hat] + r;
      bin = upper_bound_i64(Gin, P, x);
      dest = bin_ptr[bin] + load1[bin] + (x - (Gin[bin] - gap[bin]));
    }
    const int64_t pd = padded_pos(dest, bin, seg_ptr, seg_begin, seg_pbegin);
    for (int j = 0; j < n_other; ++j) out_idx.p[j][pd] = in_idx.p[j][e];
    if (out_val) out_val[pd] = vals[e];
    if (elem_order) elem_order[dest] = e;
    if (order_pad) order_pad[pd] = e;
  }
}

__global__ void k_seg_padlen(const int64_t* __restrict__ seg_begin, int64_t S, int64_t* __restrict__ plen) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < S; k += (int64_t)gridDim.x * blockDim.x)
    plen[k] = (seg_begin[k + 1] - seg_begin[k] + 3) & ~(int64_t)3;
}

__global__ void k_bin_pptr(const int32_t* __restrict__ seg_ptr, const int64_t* __restrict__ seg_pbegin, int64_t P,
                           int64_t* __restrict__ bin_pptr, int64_t* __restrict__ bsize) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= P; p += (int64_t)gridDim.x * blockDim.x) {
    bin_pptr[p] = seg_pbegin[seg_ptr[p]];
    if (p < P) bsize[p] = seg_pbegin[seg_ptr[p + 1]] - seg_pbegin[seg_ptr[p]];
  }
}

// ---- CoarseG (Section 5, coarse grained schemes): whole slices in a given
// random order, cut into contiguous blocks; the slice at position t (element
// prefix x_t in that order) goes to bin min(P-1, floor(x_t P / m)).

__global__ void k_coarse_sizes(const int32_t* __restrict__ order, const int64_t* __restrict__ count, int64_t L,
                               int64_t* __restrict__ csize, int32_t* __restrict__ nz) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = count[order[t]];
    csize[t] = c;
    nz[t] = c > 0;
  }
}

// One segment per nonempty slice, in the given order.
__global__ void k_coarse_segments(const int32_t* __restrict__ order, const int64_t* __restrict__ count,
                                  const int64_t* __restrict__ cpre, const int32_t* __restrict__ sidx,
                                  const int32_t* __restrict__ row_of, int64_t L, int64_t m, int64_t P,
                                  int32_t* __restrict__ seg_row, int64_t* __restrict__ seg_begin,
                                  int32_t* __restrict__ seg_slot, int64_t* __restrict__ seg_bin,
                                  int32_t* __restrict__ seg_of_slice) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t l = order[t];
    if (count[l] == 0) continue;
    const int32_t k = sidx[t];
    seg_row[k] = row_of[l];
    seg_begin[k] = cpre[t];
    seg_slot[k] = -1;
    const int64_t b = cpre[t] * P / m;
    seg_bin[k] = b < P - 1 ? b : P - 1;
    seg_of_slice[l] = k;
  }
}

// seg_ptr[p] = number of segments in bins below p (segment bins never
// decrease); bin_ptr[p] = the layout offset of its first segment.
__global__ void k_coarse_bins(const int64_t* __restrict__ seg_bin, const int64_t* __restrict__ seg_begin, int64_t S,
                              int64_t P, int64_t m, int32_t* __restrict__ seg_ptr, int64_t* __restrict__ bin_ptr,
                              int64_t* __restrict__ load, int64_t* __restrict__ nseg) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= P; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = S;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (seg_bin[mid] < p) lo = mid + 1; else hi = mid;
    }
    seg_ptr[p] = (int32_t)lo;
    bin_ptr[p] = lo < S ? seg_begin[lo] : m;
    if (p < P) {
      int64_t lo2 = lo, hi2 = S;   // first segment in a bin above p
      while (lo2 < hi2) {
        const int64_t mid = lo2 + ((hi2 - lo2) >> 1);
        if (seg_bin[mid] <= p) lo2 = mid + 1; else hi2 = mid;
      }
      nseg[p] = lo2 - lo;
      load[p] = (lo2 < S ? seg_begin[lo2] : m) - bin_ptr[p];
    }
  }
}

static int bits_for_len(int64_t L) {
  int b = 0;
  while (b < 32 && ((int64_t)1 << b) < L) ++b;
  return b < 1 ? 1 : b;
}

template <class T>
static T fetch(Ctx* c, const T* d) {
  T h{};
  d2h(c, &h, d, 1);
  c->sync();
  return h;
}

static void build_plan_coarse(Ctx* c, ModePlan& pl, int N, int n, int64_t L, int64_t m, Buf* idx, const float* vals,
                              bool keep_order, const int32_t* order, Buf& skey, Buf& sperm, Buf& sstart, Buf& count,
                              Buf& row_of);

void build_plan(Ctx* c, ModePlan& pl, int N, int n, const int64_t* dims, int64_t m, Buf* idx, const float* vals,
                int64_t khat, int tile_w, int64_t wg_default, bool keep_order, SortScratch& ss, bool last,
                const int32_t* coarse_order) {
  const int B = 256;
  const int64_t L = dims[n];
  pl = ModePlan();
  pl.L = L;
  pl.khat = khat;
  TK_REQUIRE(m < ((int64_t)1 << 32), TK_ERR_UNSUPPORTED, "this build handles fewer than 2^32 elements");

  // 1. slice-sorted order of the elements (stable => canonical order inside a slice)
  const size_t eb = 4 * (size_t)(m ? m : 1);
  ensure(c, ss.key, eb);
  ensure(c, ss.skey, eb);
  ensure(c, ss.perm, eb);
  ensure(c, ss.sperm, eb);
  Buf &key = ss.key, &skey = ss.skey, &perm = ss.perm, &sperm = ss.sperm;
  hipLaunchKernelGGL(k_copy_key, dim3(grid_for(m, B)), dim3(B), 0, c->stream, idx[n].as<int32_t>(),
                     key.as<uint32_t>(), m);
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_iota_u32b, dim3(grid_for(m, B)), dim3(B), 0, c->stream, perm.as<uint32_t>(), m);
  TK_CHECK_LAUNCH();
  sort_pairs_u32(c, key.as<uint32_t>(), skey.as<uint32_t>(), perm.as<uint32_t>(), sperm.as<uint32_t>(), m,
                 bits_for_len(L), &ss.tmp);
  if (last) {   // the sorted pair stays until the layout; the rest is done with
    key.release();
    perm.release();
    ss.tmp.release();
  }

  // 2. slice sizes, nonempty slices, sort by (size, id)
  Buf sstart(c, 8 * (size_t)L), count(c, 8 * (size_t)L), nonempty(c, 4 * (size_t)L), row_of(c, 4 * (size_t)L);
  TK_HIP(hipMemsetAsync(sstart.get(), 0, 8 * (size_t)L, c->stream));
  TK_HIP(hipMemsetAsync(count.get(), 0, 8 * (size_t)L, c->stream));
  hipLaunchKernelGGL(k_slice_bounds, dim3(grid_for(m, B)), dim3(B), 0, c->stream, skey.as<uint32_t>(), m,
                     sstart.as<int64_t>(), count.as<int64_t>());
  TK_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_finish_counts, dim3(grid_for(L, B)), dim3(B), 0, c->stream, sstart.as<int64_t>(),
                     count.as<int64_t>(), nonempty.as<int32_t>(), L);
  TK_CHECK_LAUNCH();
  exclusive_scan_i32(c, nonempty.as<int32_t>(), row_of.as<int32_t>(), L);
  const int64_t Lnz = (int64_t)fetch(c, row_of.as<int32_t>() + L - 1) + fetch(c, nonempty.as<int32_t>() + L - 1);
  pl.L_nz = Lnz;
  nonempty.release();
  const int64_t Lnz1 = Lnz > 0 ? Lnz : 1;
  pl.row_slice.alloc(c, 4 * (size_t)Lnz1);
  Buf ckey(c, 4 * (size_t)Lnz1), cval(c, 4 * (size_t)Lnz1), osize(c, 4 * (size_t)Lnz1), oslice(c, 4 * (size_t)Lnz1);
  hipLaunchKernelGGL(k_compact_slices, dim3(grid_for(L, B)), dim3(B), 0, c->stream, count.as<int64_t>(),
                     row_of.as<int32_t>(), L, pl.row_slice.as<int32_t>(), ckey.as<uint32_t>(), cval.as<uint32_t>());
  TK_CHECK_LAUNCH();
  int max_bits = bits_for_len(m + 1);
  sort_pairs_u32(c, ckey.as<uint32_t>(), osize.as<uint32_t>(), cval.as<uint32_t>(), oslice.as<uint32_t>(), Lnz,
                 max_bits);
  ckey.release();
  cval.release();
  Buf rank_of(c, 4 * (size_t)L), size64(c, 8 * (size_t)Lnz1);
  hipLaunchKernelGGL(k_rank_of, dim3(grid_for(Lnz, B)), dim3(B), 0, c->stream, osize.as<uint32_t>(),
                     oslice.as<uint32_t>(), Lnz, rank_of.as<int32_t>(), size64.as<int64_t>());
  TK_CHECK_LAUNCH();
  pl.label.alloc(c, 4 * (size_t)L);
  hipLaunchKernelGGL(k_labels, dim3(grid_for(L, B)), dim3(B), 0, c->stream, rank_of.as<int32_t>(),
                     row_of.as<int32_t>(), count.as<int64_t>(), L, Lnz, pl.label.as<int32_t>());
  TK_CHECK_LAUNCH();

  // 3. number of bins and the limit
  const int cap = c->opt.lds_rows_cap >= 3 ? std::min(c->opt.lds_rows_cap, ttm_rows_cap(c, tile_w))
                                            : ttm_rows_cap(c, tile_w);
  const int64_t wg = c->opt.wg_nnz_target > 0 ? c->opt.wg_nnz_target : wg_default;
  int64_t P = std::max<int64_t>(1, std::max(ceil_div(m, wg), ceil_div(Lnz, cap - 2)));
  const int64_t limit = m > 0 ? ceil_div(m, P) : 0;
  pl.P = P;
  pl.limit = limit;
  pl.rows_cap = cap;
  if (coarse_order) {
    build_plan_coarse(c, pl, N, n, L, m, idx, vals, keep_order, coarse_order, skey, sperm, sstart, count, row_of);
    pl.row_of = std::move(row_of);
    return;
  }
  count.release();

  // 4. stage 1
  Buf cand(c, 8 * (size_t)P), tmin(c, 8);
  hipLaunchKernelGGL(k_stage1_first_fail, dim3(grid_for(P, B)), dim3(B), 0, c->stream, size64.as<int64_t>(), Lnz, P,
                     limit, cand.as<int64_t>());
  TK_CHECK_LAUNCH();
  reduce_min_i64(c, cand.as<int64_t>(), tmin.as<int64_t>(), P);
  const int64_t t_hat = Lnz > 0 ? fetch(c, tmin.as<int64_t>()) : 0;
  cand.release();
  pl.n_stage1 = t_hat;
  Buf off1(c, 8 * (size_t)Lnz1), load1(c, 8 * (size_t)P), cnt1(c, 8 * (size_t)P), gap(c, 8 * (size_t)P);
  hipLaunchKernelGGL(k_stage1_place, dim3(grid_for(P, B)), dim3(B), 0, c->stream, size64.as<int64_t>(), t_hat, P,
                     limit, off1.as<int64_t>(), load1.as<int64_t>(), cnt1.as<int64_t>(), gap.as<int64_t>());
  TK_CHECK_LAUNCH();

  // 5. stage 2 as a pour into the gaps
  const int64_t n2 = Lnz - t_hat;
  Buf Gin(c, 8 * (size_t)P), X(c, 8 * (size_t)(n2 + 1));
  inclusive_scan_i64(c, gap.as<int64_t>(), Gin.as<int64_t>(), P);
  int64_t M2 = 0;
  if (n2 > 0) {
    // X = exclusive scan of sizes[t_hat..], with X[n2] = M2
    exclusive_scan_i64(c, size64.as<int64_t>() + t_hat, X.as<int64_t>(), n2);
    M2 = fetch(c, X.as<int64_t>() + n2 - 1) + fetch(c, size64.as<int64_t>() + Lnz - 1);
  }
  h2d(c, X.as<int64_t>() + n2, &M2, 1);
  c->sync();
  pl.M2 = M2;
  if (n2 > 0) {
    int64_t gtot = fetch(c, Gin.as<int64_t>() + P - 1);
    TK_REQUIRE(M2 <= gtot, TK_ERR_DEVICE, "Lite stage 2: gaps smaller than the remaining elements");
  }

  Buf load(c, 8 * (size_t)P), nseg(c, 8 * (size_t)P);
  hipLaunchKernelGGL(k_bin_loads, dim3(grid_for(P, B)), dim3(B), 0, c->stream, load1.as<int64_t>(),
                     cnt1.as<int64_t>(), gap.as<int64_t>(), Gin.as<int64_t>(), X.as<int64_t>(), n2, M2, P,
                     load.as<int64_t>(), nseg.as<int64_t>());
  TK_CHECK_LAUNCH();
  pl.bin_ptr.alloc(c, 8 * (size_t)(P + 1));
  exclusive_scan_i64(c, load.as<int64_t>(), pl.bin_ptr.as<int64_t>(), P);
  h2d(c, pl.bin_ptr.as<int64_t>() + P, &m, 1);
  Buf seg_first(c, 8 * (size_t)(P + 1)), mx(c, 8);
  exclusive_scan_i64(c, nseg.as<int64_t>(), seg_first.as<int64_t>(), P);
  const int64_t S = fetch(c, seg_first.as<int64_t>() + P - 1) + fetch(c, nseg.as<int64_t>() + P - 1);
  pl.S = S;
  reduce_max_i64(c, nseg.as<int64_t>(), mx.as<int64_t>(), P);
  pl.R_max = fetch(c, mx.as<int64_t>());
  reduce_max_i64(c, load.as<int64_t>(), mx.as<int64_t>(), P);
  pl.E_max = fetch(c, mx.as<int64_t>());
  TK_REQUIRE(pl.R_max <= cap, TK_ERR_DEVICE, "Lite partition: a bin holds more slices than the LDS row budget");
  TK_REQUIRE(S < ((int64_t)1 << 31), TK_ERR_UNSUPPORTED, "too many segments");

  // 6. segments
  const int64_t S1 = S > 0 ? S : 1;
  pl.seg_ptr.alloc(c, 4 * (size_t)(P + 1));
  pl.seg_row.alloc(c, 4 * (size_t)S1);
  pl.seg_begin.alloc(c, 8 * (size_t)(S + 1));
  pl.seg_slot.alloc(c, 4 * (size_t)S1);
  Buf seg_u(c, 4 * (size_t)S1), first_seg(c, 8 * (size_t)(n2 + 1)), last_seg(c, 8 * (size_t)(n2 + 1));
  hipLaunchKernelGGL(k_fill_segments, dim3(grid_for(P, B)), dim3(B), 0, c->stream, pl.bin_ptr.as<int64_t>(),
                     seg_first.as<int64_t>(), load1.as<int64_t>(), gap.as<int64_t>(), Gin.as<int64_t>(),
                     X.as<int64_t>(), off1.as<int64_t>(), oslice.as<uint32_t>(), row_of.as<int32_t>(), t_hat, n2, M2,
                     P, pl.seg_ptr.as<int32_t>(), pl.seg_row.as<int32_t>(), pl.seg_begin.as<int64_t>(),
                     seg_u.as<int32_t>(), first_seg.as<int64_t>(), last_seg.as<int64_t>());
  TK_CHECK_LAUNCH();
  {
    int32_t Si = (int32_t)S;
    h2d(c, pl.seg_ptr.as<int32_t>() + P, &Si, 1);
    h2d(c, pl.seg_begin.as<int64_t>() + S, &m, 1);
    c->sync();
  }
  Buf bad(c, 4 * (size_t)S1), slot_scan(c, 4 * (size_t)S1);
  hipLaunchKernelGGL(k_seg_bad, dim3(grid_for(S, B)), dim3(B), 0, c->stream, seg_u.as<int32_t>(),
                     first_seg.as<int64_t>(), last_seg.as<int64_t>(), S, bad.as<int32_t>());
  TK_CHECK_LAUNCH();
  exclusive_scan_i32(c, bad.as<int32_t>(), slot_scan.as<int32_t>(), S);
  hipLaunchKernelGGL(k_seg_slot, dim3(grid_for(S, B)), dim3(B), 0, c->stream, bad.as<int32_t>(),
                     slot_scan.as<int32_t>(), S, pl.seg_slot.as<int32_t>());
  TK_CHECK_LAUNCH();
  pl.n_slots = S > 0 ? (int64_t)fetch(c, slot_scan.as<int32_t>() + S - 1) + fetch(c, bad.as<int32_t>() + S - 1) : 0;
  // bad slices
  int64_t nbad = 0;
  pl.fix_n.clear();
  pl.fix_rows = pl.n_slots;
  if (n2 > 0) {
    Buf bflag(c, 4 * (size_t)n2), bscan(c, 4 * (size_t)n2);
    hipLaunchKernelGGL(k_is_bad_slice, dim3(grid_for(n2, B)), dim3(B), 0, c->stream, first_seg.as<int64_t>(),
                       last_seg.as<int64_t>(), n2, bflag.as<int32_t>());
    TK_CHECK_LAUNCH();
    exclusive_scan_i32(c, bflag.as<int32_t>(), bscan.as<int32_t>(), n2);
    nbad = (int64_t)fetch(c, bscan.as<int32_t>() + n2 - 1) + fetch(c, bflag.as<int32_t>() + n2 - 1);
    pl.bad_row.alloc(c, 4 * (size_t)(nbad > 0 ? nbad : 1));
    pl.bad_slot.alloc(c, 4 * (size_t)(nbad + 1));
    int32_t zero = 0;
    h2d(c, pl.bad_slot.as<int32_t>(), &zero, 1);
    hipLaunchKernelGGL(k_bad_table, dim3(grid_for(n2, B)), dim3(B), 0, c->stream, first_seg.as<int64_t>(),
                       last_seg.as<int64_t>(), pl.seg_slot.as<int32_t>(), pl.seg_row.as<int32_t>(),
                       bscan.as<int32_t>(), n2, pl.bad_row.as<int32_t>(), pl.bad_slot.as<int32_t>());
    TK_CHECK_LAUNCH();
    c->sync();
    // fixup tree: each level sums runs of at most FIX_CHUNK consecutive rows
    // of one slice (fixed shape, so the order of every sum is fixed)
    std::vector<int32_t> bs((size_t)nbad + 1);
    d2h(c, bs.data(), pl.bad_slot.as<int32_t>(), (size_t)nbad + 1);
    c->sync();
    std::vector<int64_t> lo(bs.begin(), bs.end() - 1), hi(bs.begin() + 1, bs.end());
    std::vector<int32_t> lohi;
    int64_t rows = pl.n_slots;
    for (;;) {
      std::vector<int32_t> l0, h0;
      int64_t next = rows;
      for (int64_t k = 0; k < nbad; ++k) {
        if (hi[k] - lo[k] <= FIX_CHUNK) continue;
        const int64_t first = next;
        for (int64_t a = lo[k]; a < hi[k]; a += FIX_CHUNK) {
          l0.push_back((int32_t)a);
          h0.push_back((int32_t)std::min<int64_t>(a + FIX_CHUNK, hi[k]));
          ++next;
        }
        lo[k] = first;
        hi[k] = next;
      }
      if (l0.empty()) break;
      TK_REQUIRE(next < ((int64_t)1 << 31), TK_ERR_UNSUPPORTED, "fixup tree too large");
      pl.fix_n.push_back((int64_t)l0.size());
      lohi.insert(lohi.end(), l0.begin(), l0.end());
      lohi.insert(lohi.end(), h0.begin(), h0.end());
      rows = next;
    }
    pl.fix_rows = rows;
    std::vector<int32_t> fin((size_t)2 * nbad);
    for (int64_t k = 0; k < nbad; ++k) {
      fin[k] = (int32_t)lo[k];
      fin[nbad + k] = (int32_t)hi[k];
    }
    pl.fix_fin.alloc(c, 4 * fin.size());
    h2d(c, pl.fix_fin.as<int32_t>(), fin.data(), fin.size());
    if (!lohi.empty()) {
      pl.fix_lohi.alloc(c, 4 * lohi.size());
      h2d(c, pl.fix_lohi.as<int32_t>(), lohi.data(), lohi.size());
    }
    c->sync();
  }
  pl.n_bad = nbad;

  // 7. padded segment offsets, then the layout
  {
    Buf plen(c, 8 * (size_t)S1), bsize(c, 8 * (size_t)P);
    pl.seg_pbegin.alloc(c, 8 * (size_t)(S + 1));
    hipLaunchKernelGGL(k_seg_padlen, dim3(grid_for(S, B)), dim3(B), 0, c->stream, pl.seg_begin.as<int64_t>(), S,
                       plen.as<int64_t>());
    TK_CHECK_LAUNCH();
    exclusive_scan_i64(c, plen.as<int64_t>(), pl.seg_pbegin.as<int64_t>(), S);
    pl.m_pad = S > 0 ? fetch(c, pl.seg_pbegin.as<int64_t>() + S - 1) + fetch(c, plen.as<int64_t>() + S - 1) : 0;
    h2d(c, pl.seg_pbegin.as<int64_t>() + S, &pl.m_pad, 1);
    c->sync();
    pl.bin_pptr.alloc(c, 8 * (size_t)(P + 1));
    hipLaunchKernelGGL(k_bin_pptr, dim3(grid_for(P + 1, B)), dim3(B), 0, c->stream, pl.seg_ptr.as<int32_t>(),
                       pl.seg_pbegin.as<int64_t>(), P, pl.bin_pptr.as<int64_t>(), bsize.as<int64_t>());
    TK_CHECK_LAUNCH();
    reduce_max_i64(c, bsize.as<int64_t>(), mx.as<int64_t>(), P);
    pl.E_pad_max = fetch(c, mx.as<int64_t>());
  }
  const int64_t m1 = pl.m_pad > 0 ? pl.m_pad : 1;
  IdxIn ii{};
  IdxOut oo{};
  int no = 0;
  for (int j = 0; j < N; ++j) {
    if (j == n) continue;
    pl.lay_idx[no].alloc(c, 4 * (size_t)m1);
    ii.p[no] = idx[j].as<int32_t>();
    oo.p[no] = pl.lay_idx[no].as<int32_t>();
    ++no;
  }
  for (int j = 0; j < no; ++j) TK_HIP(hipMemsetAsync(oo.p[j], 0, 4 * (size_t)m1, c->stream));
  if (vals) {
    pl.lay_val.alloc(c, 4 * (size_t)m1);
    TK_HIP(hipMemsetAsync(pl.lay_val.get(), 0, 4 * (size_t)m1, c->stream));
  } else {
    pl.order_pad.alloc(c, 4 * (size_t)m1);
    TK_HIP(hipMemsetAsync(pl.order_pad.get(), 0xff, 4 * (size_t)m1, c->stream));
  }
  if (keep_order) pl.elem_order.alloc(c, 4 * (size_t)(m > 0 ? m : 1));
  hipLaunchKernelGGL(k_layout, dim3(grid_for(m, B)), dim3(B), 0, c->stream, skey.as<uint32_t>(),
                     sperm.as<uint32_t>(), m, sstart.as<int64_t>(), rank_of.as<int32_t>(), off1.as<int64_t>(),
                     X.as<int64_t>(), Gin.as<int64_t>(), gap.as<int64_t>(), load1.as<int64_t>(),
                     pl.bin_ptr.as<int64_t>(), t_hat, P, pl.seg_ptr.as<int32_t>(), pl.seg_begin.as<int64_t>(),
                     pl.seg_pbegin.as<int64_t>(), ii, no, vals, oo, vals ? pl.lay_val.as<float>() : nullptr,
                     keep_order ? pl.elem_order.as<uint32_t>() : nullptr,
                     vals ? nullptr : pl.order_pad.as<uint32_t>());
  TK_CHECK_LAUNCH();
  c->sync();
  pl.row_of = std::move(row_of);
}

__global__ void k_coarse_layout(const uint32_t* __restrict__ skey, const uint32_t* __restrict__ sperm, int64_t m,
                                const int64_t* __restrict__ sstart, const int32_t* __restrict__ seg_of_slice,
                                const int64_t* __restrict__ seg_begin, const int64_t* __restrict__ seg_pbegin,
                                IdxIn in_idx, int n_other, const float* __restrict__ vals, IdxOut out_idx,
                                float* __restrict__ out_val, uint32_t* __restrict__ elem_order,
                                uint32_t* __restrict__ order_pad) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < m; s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t l = skey[s];
    const uint32_t e = sperm[s];
    const int64_t r = s - sstart[l];
    const int32_t k = seg_of_slice[l];
    const int64_t pd = seg_pbegin[k] + r;
    for (int j = 0; j < n_other; ++j) out_idx.p[j][pd] = in_idx.p[j][e];
    if (out_val) out_val[pd] = vals[e];
    if (elem_order) elem_order[seg_begin[k] + r] = e;
    if (order_pad) order_pad[pd] = e;
  }
}

static void build_plan_coarse(Ctx* c, ModePlan& pl, int N, int n, int64_t L, int64_t m, Buf* idx, const float* vals,
                              bool keep_order, const int32_t* order, Buf& skey, Buf& sperm, Buf& sstart, Buf& count,
                              Buf& row_of) {
  const int B = 256;
  const int64_t P = pl.P;
  const int64_t S = pl.L_nz;              // one segment per nonempty slice
  const int64_t S1 = S > 0 ? S : 1;
  pl.whole_slices = true;
  pl.n_stage1 = S;
  pl.n_bad = 0;
  pl.n_slots = 0;
  pl.fix_rows = 0;
  pl.S = S;
  Buf csize(c, 8 * (size_t)L), cpre(c, 8 * (size_t)L), nz(c, 4 * (size_t)L), sidx(c, 4 * (size_t)L);
  hipLaunchKernelGGL(k_coarse_sizes, dim3(grid_for(L, B)), dim3(B), 0, c->stream, order, count.as<int64_t>(), L,
                     csize.as<int64_t>(), nz.as<int32_t>());
  TK_CHECK_LAUNCH();
  exclusive_scan_i64(c, csize.as<int64_t>(), cpre.as<int64_t>(), L);
  exclusive_scan_i32(c, nz.as<int32_t>(), sidx.as<int32_t>(), L);
  pl.seg_row.alloc(c, 4 * (size_t)S1);
  pl.seg_begin.alloc(c, 8 * (size_t)(S + 1));
  pl.seg_slot.alloc(c, 4 * (size_t)S1);
  pl.seg_ptr.alloc(c, 4 * (size_t)(P + 1));
  pl.bin_ptr.alloc(c, 8 * (size_t)(P + 1));
  Buf seg_bin(c, 8 * (size_t)S1), seg_of_slice(c, 4 * (size_t)L), load(c, 8 * (size_t)P), nseg(c, 8 * (size_t)P),
      mx(c, 8);
  hipLaunchKernelGGL(k_coarse_segments, dim3(grid_for(L, B)), dim3(B), 0, c->stream, order, count.as<int64_t>(),
                     cpre.as<int64_t>(), sidx.as<int32_t>(), row_of.as<int32_t>(), L, m > 0 ? m : 1, P,
                     pl.seg_row.as<int32_t>(), pl.seg_begin.as<int64_t>(), pl.seg_slot.as<int32_t>(),
                     seg_bin.as<int64_t>(), seg_of_slice.as<int32_t>());
  TK_CHECK_LAUNCH();
  h2d(c, pl.seg_begin.as<int64_t>() + S, &m, 1);
  hipLaunchKernelGGL(k_coarse_bins, dim3(grid_for(P + 1, B)), dim3(B), 0, c->stream, seg_bin.as<int64_t>(),
                     pl.seg_begin.as<int64_t>(), S, P, m, pl.seg_ptr.as<int32_t>(), pl.bin_ptr.as<int64_t>(),
                     load.as<int64_t>(), nseg.as<int64_t>());
  TK_CHECK_LAUNCH();
  reduce_max_i64(c, nseg.as<int64_t>(), mx.as<int64_t>(), P);
  pl.R_max = fetch(c, mx.as<int64_t>());
  reduce_max_i64(c, load.as<int64_t>(), mx.as<int64_t>(), P);
  pl.E_max = fetch(c, mx.as<int64_t>());
  csize.release();
  cpre.release();
  nz.release();
  sidx.release();
  count.release();

  // padded segment offsets, then the layout
  {
    Buf plen(c, 8 * (size_t)S1), bsize(c, 8 * (size_t)P);
    pl.seg_pbegin.alloc(c, 8 * (size_t)(S + 1));
    hipLaunchKernelGGL(k_seg_padlen, dim3(grid_for(S, B)), dim3(B), 0, c->stream, pl.seg_begin.as<int64_t>(), S,
                       plen.as<int64_t>());
    TK_CHECK_LAUNCH();
    exclusive_scan_i64(c, plen.as<int64_t>(), pl.seg_pbegin.as<int64_t>(), S);
    pl.m_pad = S > 0 ? fetch(c, pl.seg_pbegin.as<int64_t>() + S - 1) + fetch(c, plen.as<int64_t>() + S - 1) : 0;
    h2d(c, pl.seg_pbegin.as<int64_t>() + S, &pl.m_pad, 1);
    c->sync();
    pl.bin_pptr.alloc(c, 8 * (size_t)(P + 1));
    hipLaunchKernelGGL(k_bin_pptr, dim3(grid_for(P + 1, B)), dim3(B), 0, c->stream, pl.seg_ptr.as<int32_t>(),
                       pl.seg_pbegin.as<int64_t>(), P, pl.bin_pptr.as<int64_t>(), bsize.as<int64_t>());
    TK_CHECK_LAUNCH();
    reduce_max_i64(c, bsize.as<int64_t>(), mx.as<int64_t>(), P);
    pl.E_pad_max = fetch(c, mx.as<int64_t>());
  }
  const int64_t m1 = pl.m_pad > 0 ? pl.m_pad : 1;
  IdxIn ii{};
  IdxOut oo{};
  int no = 0;
  for (int j = 0; j < N; ++j) {
    if (j == n) continue;
    pl.lay_idx[no].alloc(c, 4 * (size_t)m1);
    ii.p[no] = idx[j].as<int32_t>();
    oo.p[no] = pl.lay_idx[no].as<int32_t>();
    ++no;
  }
  for (int j = 0; j < no; ++j) TK_HIP(hipMemsetAsync(oo.p[j], 0, 4 * (size_t)m1, c->stream));
  if (vals) {
    pl.lay_val.alloc(c, 4 * (size_t)m1);
    TK_HIP(hipMemsetAsync(pl.lay_val.get(), 0, 4 * (size_t)m1, c->stream));
  } else {
    pl.order_pad.alloc(c, 4 * (size_t)m1);
    TK_HIP(hipMemsetAsync(pl.order_pad.get(), 0xff, 4 * (size_t)m1, c->stream));
  }
  if (keep_order) pl.elem_order.alloc(c, 4 * (size_t)(m > 0 ? m : 1));
  hipLaunchKernelGGL(k_coarse_layout, dim3(grid_for(m, B)), dim3(B), 0, c->stream, skey.as<uint32_t>(),
                     sperm.as<uint32_t>(), m, sstart.as<int64_t>(), seg_of_slice.as<int32_t>(),
                     pl.seg_begin.as<int64_t>(), pl.seg_pbegin.as<int64_t>(), ii, no, vals, oo,
                     vals ? pl.lay_val.as<float>() : nullptr, keep_order ? pl.elem_order.as<uint32_t>() : nullptr,
                     vals ? nullptr : pl.order_pad.as<uint32_t>());
  TK_CHECK_LAUNCH();
  c->sync();
}

// Rewrite the other modes' coordinates of plan n into storage labels.
void relabel_layout(Ctx* c, ModePlan& pl, int N, int n, const ModePlan* plans, int64_t m) {
  (void)m;
  int no = 0;
  for (int j = 0; j < N; ++j) {
    if (j == n) continue;
    hipLaunchKernelGGL(k_apply_labels, dim3(grid_for(pl.m_pad, 256)), dim3(256), 0, c->stream,
                       pl.lay_idx[no].as<int32_t>(), pl.m_pad, plans[j].label.as<int32_t>());
    TK_CHECK_LAUNCH();
    ++no;
  }
}

// ---- export -------------------------------------------------------------------------------------

__global__ void k_export_segments(const int32_t* __restrict__ seg_ptr, int64_t P, const int32_t* __restrict__ seg_row,
                                  const int32_t* __restrict__ row_slice, const int32_t* __restrict__ seg_slot,
                                  int32_t* __restrict__ seg_bin, int32_t* __restrict__ seg_slice,
                                  uint8_t* __restrict__ seg_bad) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    for (int32_t k = seg_ptr[p]; k < seg_ptr[p + 1]; ++k) {
      if (seg_bin) seg_bin[k] = (int32_t)p;
      if (seg_slice) seg_slice[k] = row_slice[seg_row[k]];
      if (seg_bad) seg_bad[k] = seg_slot[k] >= 0 ? 1 : 0;
    }
  }
}

__global__ void k_u32_to_i64(const uint32_t* __restrict__ in, int64_t* __restrict__ out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int64_t)in[i];
}

void export_partition(Ctx* c, ModePlan& pl, int64_t m, int64_t* bin_ptr, int64_t* elem_order, int32_t* seg_bin,
                      int32_t* seg_slice, int64_t* seg_begin, uint8_t* seg_bad, tk_mem mem) {
  const int B = 256;
  const int64_t S1 = pl.S > 0 ? pl.S : 1;
  if (bin_ptr) copy_out(c, bin_ptr, pl.bin_ptr.as<int64_t>(), (size_t)(pl.P + 1), mem);
  if (seg_begin) copy_out(c, seg_begin, pl.seg_begin.as<int64_t>(), (size_t)(pl.S + 1), mem);
  if (seg_bin || seg_slice || seg_bad) {
    Buf b(c, 4 * (size_t)S1), s(c, 4 * (size_t)S1), f(c, (size_t)S1);
    hipLaunchKernelGGL(k_export_segments, dim3(grid_for(pl.P, B)), dim3(B), 0, c->stream, pl.seg_ptr.as<int32_t>(),
                       pl.P, pl.seg_row.as<int32_t>(), pl.row_slice.as<int32_t>(), pl.seg_slot.as<int32_t>(),
                       seg_bin ? b.as<int32_t>() : nullptr, seg_slice ? s.as<int32_t>() : nullptr,
                       seg_bad ? f.as<uint8_t>() : nullptr);
    TK_CHECK_LAUNCH();
    if (seg_bin) copy_out(c, seg_bin, b.as<int32_t>(), (size_t)pl.S, mem);
    if (seg_slice) copy_out(c, seg_slice, s.as<int32_t>(), (size_t)pl.S, mem);
    if (seg_bad) copy_out(c, seg_bad, f.as<uint8_t>(), (size_t)pl.S, mem);
    c->sync();
  }
  if (elem_order) {
    TK_REQUIRE(pl.elem_order, TK_ERR_STATE, "element order was not kept (keep_elem_order = 0)");
    Buf t(c, 8 * (size_t)(m > 0 ? m : 1));
    hipLaunchKernelGGL(k_u32_to_i64, dim3(grid_for(m, B)), dim3(B), 0, c->stream, pl.elem_order.as<uint32_t>(),
                       t.as<int64_t>(), m);
    TK_CHECK_LAUNCH();
    copy_out(c, elem_order, t.as<int64_t>(), (size_t)m, mem);
    c->sync();
  }
}

}  // namespace tk
