// The Lite distribution scheme, sequential, for large inputs (oracle; TEST
// INFRASTRUCTURE ONLY: the test-suite calls it, the library never does, and
// this file shares nothing with it).
//
// Section 6 ("Distribution Scheme Lite") and its pseudocode figure, with the
// readings of oracle/lite.py: empty slices left out; slices sorted by
// (cardinality, id) ascending; limit = ceil(m / P); stage 1 gives whole slices
// to bins 0, 1, ..., P-1, 0, ... until a slice would push its bin above the
// limit; stage 2 walks the remaining slices and the bins together, a slice
// that fits the current bin's gap going there whole, otherwise the bin being
// filled to the limit (a bin with gap 0 receives nothing) and the walk moving
// to the next bin.  The same steps as lite.py, in C++ for millions of slices
// and bins; the segments come out in layout order (bins in order; inside a
// bin its stage-1 slices, then its stage-2 pieces in the order assigned).
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

extern "C" {

// sizes[L]: cardinality of every slice (0 = empty).  Outputs: stats[7] =
// {limit, m, L_nonempty, n_stage1, E_max, R_max, n_bad}; seg_* arrays of the
// segments (at most L + P entries) in layout order; returns the segment
// count (R_sum), or -1 when stage 2 runs out of bins (impossible for limit =
// ceil(m/P)).
int64_t oracle_lite(int64_t L, const int64_t* sizes, int64_t P, int64_t* stats, int64_t* seg_bin, int64_t* seg_slice,
                    int64_t* seg_count, uint8_t* seg_bad) {
  int64_t m = 0;
  std::vector<int64_t> order;
  for (int64_t l = 0; l < L; ++l) {
    m += sizes[l];
    if (sizes[l] > 0) order.push_back(l);
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return sizes[a] < sizes[b]; });
  const int64_t limit = m > 0 ? (m + P - 1) / P : 0;
  const int64_t T = (int64_t)order.size();
  std::vector<int64_t> load((size_t)P, 0);
  // per bin: its stage-1 slices, then its stage-2 pieces (slice, count)
  std::vector<std::vector<std::pair<int64_t, int64_t>>> in_bin((size_t)P);
  std::vector<int32_t> n_pieces((size_t)L, 0);

  // stage 1
  int64_t t = 0, p = 0;
  while (t < T) {
    const int64_t S = order[(size_t)t];
    if (load[(size_t)p] + sizes[S] > limit) break;
    load[(size_t)p] += sizes[S];
    in_bin[(size_t)p].push_back({S, sizes[S]});
    n_pieces[(size_t)S] = 1;
    p = (p + 1) % P;
    ++t;
  }
  const int64_t n_stage1 = t;
  // stage 2
  p = 0;
  int64_t remaining = t < T ? sizes[order[(size_t)t]] : 0;
  while (p < P && t < T) {
    const int64_t S = order[(size_t)t];
    const int64_t g = limit - load[(size_t)p];
    if (remaining <= g) {
      load[(size_t)p] += remaining;
      in_bin[(size_t)p].push_back({S, remaining});
      ++n_pieces[(size_t)S];
      ++t;
      remaining = t < T ? sizes[order[(size_t)t]] : 0;
    } else {
      if (g > 0) {
        load[(size_t)p] += g;
        in_bin[(size_t)p].push_back({S, g});
        ++n_pieces[(size_t)S];
        remaining -= g;
      }
      ++p;
    }
  }
  if (t < T) return -1;

  int64_t k = 0, E_max = 0, R_max = 0, n_bad = 0;
  for (int64_t b = 0; b < P; ++b) {
    E_max = std::max(E_max, load[(size_t)b]);
    R_max = std::max(R_max, (int64_t)in_bin[(size_t)b].size());
    for (const auto& sc : in_bin[(size_t)b]) {
      seg_bin[k] = b;
      seg_slice[k] = sc.first;
      seg_count[k] = sc.second;
      seg_bad[k] = n_pieces[(size_t)sc.first] > 1 ? 1 : 0;
      ++k;
    }
  }
  for (int64_t l = 0; l < L; ++l) n_bad += n_pieces[(size_t)l] > 1;
  stats[0] = limit;
  stats[1] = m;
  stats[2] = T;
  stats[3] = n_stage1;
  stats[4] = E_max;
  stats[5] = R_max;
  stats[6] = n_bad;
  return k;
}

}  // extern "C"
