// FP64 TTM-chain through the Kronecker reformulation, multi-threaded (oracle;
// TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
// benchmark's CPU baseline call it; the library never does, and this file
// shares nothing with it).
//
// Section 3, "Reformulation" (eq. 1) and Appendix A: the mode-n penultimate
// matrix has one row per mode-n index l, and
//     Z_(n)[l, :] = sum over the elements e of slice l of val(e) * Kron_n(e),
// where Kron_n(e) is the Kronecker product of the factor rows F_j[l_j(e), :]
// for j != n, first remaining mode fastest: entry sum_j c_j prod_{i<j} K_i
// (j, i over the remaining modes) is prod_j F_j[l_j(e)][c_j].
//
// The same definition as oracle/ttm.py, written for inputs too large for
// NumPy's temporaries: every contribution is formed and added in FP64.
//   oracle_ttm_rows_add  adds the contributions of a batch of elements to the
//                        rows of selected slices (batches can be streamed);
//   oracle_ttm_chain     the whole Z_(n): elements grouped by mode-n index
//                        with a counting sort, slices split over the threads,
//                        so each row is summed by one thread in element order.
#include <omp.h>

#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// Kron_n(e) * val into kr (length prod_{j != n} K_j), first remaining mode fastest.
inline void kron_row(int N, int n, const int64_t* K, const int32_t* const* idx, const double* const* F, int64_t e,
                     double val, double* kr) {
  int64_t len = 1;
  kr[0] = val;
  for (int j = 0; j < N; ++j) {
    if (j == n) continue;
    const double* row = F[j] + (int64_t)idx[j][e] * K[j];
    // new[a + len * b] = old[a] * row[b], written from the back so old stays readable
    for (int64_t b = K[j] - 1; b >= 0; --b)
      for (int64_t a = len - 1; a >= 0; --a) kr[a + len * b] = kr[a] * row[b];
    len *= K[j];
  }
}

int64_t khat_of(int N, int n, const int64_t* K) {
  int64_t k = 1;
  for (int j = 0; j < N; ++j)
    if (j != n) k *= K[j];
  return k;
}

}  // namespace

extern "C" {

int oracle_threads(void) { return omp_get_max_threads(); }

// out[sel[l] * khat + c] += val(e) * Kron_n(e)[c] for every element e of the
// batch whose mode-n index l has sel[l] >= 0 (sel has L_n entries).  Each
// thread sums its contiguous part of the batch into its own rows; the threads'
// rows are then added to out in thread order.
void oracle_ttm_rows_add(int N, int n, const int64_t* K, int64_t nnz, const int32_t* const* idx, const float* vals,
                         const double* const* F, const int32_t* sel, int64_t nrows, double* out) {
  const int64_t khat = khat_of(N, n, K);
  const int T = omp_get_max_threads();
  std::vector<std::vector<double>> part(T);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    std::vector<double>& acc = part[t];
    acc.assign((size_t)(nrows * khat), 0.0);
    std::vector<double> kr((size_t)khat);
    const int64_t a = nnz * t / nt, b = nnz * (t + 1) / nt;
    for (int64_t e = a; e < b; ++e) {
      const int32_t r = sel[idx[n][e]];
      if (r < 0) continue;
      kron_row(N, n, K, idx, F, e, (double)vals[e], kr.data());
      double* dst = acc.data() + (int64_t)r * khat;
      for (int64_t c = 0; c < khat; ++c) dst[c] += kr[c];
    }
  }
  for (int t = 0; t < T; ++t) {
    if (part[t].empty()) continue;
    for (int64_t i = 0; i < nrows * khat; ++i) out[i] += part[t][(size_t)i];
  }
}

// The whole Z_(n) (dims[n] x khat, row-major, zero rows for empty slices).
void oracle_ttm_chain(int N, int n, const int64_t* dims, const int64_t* K, int64_t nnz, const int32_t* const* idx,
                      const float* vals, const double* const* F, double* out) {
  const int64_t L = dims[n];
  const int64_t khat = khat_of(N, n, K);
  // elements grouped by mode-n index (counting sort, stable)
  std::vector<int64_t> start((size_t)L + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) ++start[(size_t)idx[n][e] + 1];
  for (int64_t l = 0; l < L; ++l) start[(size_t)l + 1] += start[(size_t)l];
  std::vector<int64_t> order((size_t)nnz);
  {
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (int64_t e = 0; e < nnz; ++e) order[(size_t)pos[(size_t)idx[n][e]]++] = e;
  }
#pragma omp parallel
  {
    std::vector<double> kr((size_t)khat);
#pragma omp for schedule(dynamic, 256)
    for (int64_t l = 0; l < L; ++l) {
      double* dst = out + l * khat;
      for (int64_t c = 0; c < khat; ++c) dst[c] = 0.0;
      for (int64_t p = start[(size_t)l]; p < start[(size_t)l + 1]; ++p) {
        const int64_t e = order[(size_t)p];
        kron_row(N, n, K, idx, F, e, (double)vals[e], kr.data());
        for (int64_t c = 0; c < khat; ++c) dst[c] += kr[c];
      }
    }
  }
}

}  // extern "C"
