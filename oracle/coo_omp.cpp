// Coalescing of a drawn element list for lists too large for NumPy (oracle;
// TEST INFRASTRUCTURE ONLY: the test-suite calls it, the library never does,
// and this file shares nothing with it).
//
// Section 3 keeps the tensor as a set of elements: repeated coordinates are
// one element, whose value is the FP64 sum of the repeated values in input
// order, rounded once to FP32 (oracle/coo.py states the same for small
// lists).  For billions of draws this file computes two things:
//   * the distinct coordinates and, from them, the merged cardinality of every
//     slice of every mode (the input of the Lite partition, Section 6):
//     coordinates are packed into 64-bit keys, split into 2^b parts by the top
//     bits of the first coordinate when they need more than 64 bits, and each
//     part is sorted and deduplicated;
//   * the merged values of chosen coordinates: the values of all draws of each
//     chosen coordinate, kept in input order and summed in that order.
#include <omp.h>
#include <parallel/algorithm>

#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace {

int bits_for(int64_t L) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < L) ++b;
  return b;
}

struct Distinct {
  int N = 0;
  int64_t dims[8] = {0};
  int bits[8] = {0};
  int shift[8] = {0};      // position of each coordinate's field in the key
  int part_bits = 0;       // top bits of coordinate 0 that pick the part
  std::vector<std::vector<uint64_t>> parts;
  std::mutex mu;
};

struct KeySums {
  int N = 0;
  std::vector<std::vector<int32_t>> coords;        // chosen coordinates, one vector per mode
  std::unordered_map<uint64_t, int64_t> slot;      // hash of a chosen coordinate -> its index
  std::vector<uint8_t> first_mode_hit;             // coordinate 0 values that occur among the chosen
  std::vector<std::vector<double>> vals;           // per chosen coordinate: values in input order
};

uint64_t hash_coord(int N, const int32_t* c) {
  uint64_t h = 1469598103934665603ULL;
  for (int j = 0; j < N; ++j) h = (h ^ (uint64_t)(uint32_t)c[j]) * 1099511628211ULL;
  return h;
}

}  // namespace

extern "C" {

void* oracle_distinct_new(int N, const int64_t* dims) {
  Distinct* d = new Distinct();
  d->N = N;
  int total = 0;
  for (int j = 0; j < N; ++j) {
    d->dims[j] = dims[j];
    d->bits[j] = bits_for(dims[j]);
    total += d->bits[j];
  }
  d->part_bits = total > 64 ? total - 64 : 0;
  if (d->part_bits > d->bits[0] || d->part_bits > 16) {
    delete d;
    return nullptr;   // the key would not fit: not needed for the workloads checked
  }
  int sh = 0;
  for (int j = N - 1; j >= 1; --j) {
    d->shift[j] = sh;
    sh += d->bits[j];
  }
  d->shift[0] = sh;   // the low (bits[0] - part_bits) bits of coordinate 0
  d->parts.resize((size_t)1 << d->part_bits);
  return d;
}

// Add the keys of a batch of drawn coordinates.
void oracle_distinct_add(void* h, int64_t n, const int32_t* const* idx) {
  Distinct* d = static_cast<Distinct*>(h);
  const int np = 1 << d->part_bits;
  const int low0 = d->bits[0] - d->part_bits;
#pragma omp parallel
  {
    std::vector<std::vector<uint64_t>> local((size_t)np);
#pragma omp for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
      const uint64_t c0 = (uint32_t)idx[0][e];
      uint64_t key = (c0 & (((uint64_t)1 << low0) - 1)) << d->shift[0];
      for (int j = 1; j < d->N; ++j) key |= (uint64_t)(uint32_t)idx[j][e] << d->shift[j];
      local[(size_t)(c0 >> low0)].push_back(key);
    }
    std::lock_guard<std::mutex> lock(d->mu);
    for (int p = 0; p < np; ++p)
      d->parts[(size_t)p].insert(d->parts[(size_t)p].end(), local[(size_t)p].begin(), local[(size_t)p].end());
  }
}

// Deduplicate every part; counts[j][l] += number of distinct coordinates with
// l_j = l.  Returns the number of distinct coordinates.  Frees the keys.
int64_t oracle_distinct_finish(void* h, int64_t* const* counts) {
  Distinct* d = static_cast<Distinct*>(h);
  const int low0 = d->bits[0] - d->part_bits;
  int64_t total = 0;
  for (size_t p = 0; p < d->parts.size(); ++p) {
    std::vector<uint64_t>& k = d->parts[p];
    __gnu_parallel::sort(k.begin(), k.end());
    k.erase(std::unique(k.begin(), k.end()), k.end());
    total += (int64_t)k.size();
    for (int j = 0; j < d->N; ++j) {
      const int T = omp_get_max_threads();
      std::vector<std::vector<int64_t>> c((size_t)T);
#pragma omp parallel num_threads(T)
      {
        std::vector<int64_t>& cj = c[(size_t)omp_get_thread_num()];
        cj.assign((size_t)d->dims[j], 0);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < (int64_t)k.size(); ++i) {
          const uint64_t key = k[(size_t)i];
          const uint64_t mask = j == 0 ? (((uint64_t)1 << low0) - 1) : (((uint64_t)1 << d->bits[j]) - 1);
          uint64_t l = (key >> d->shift[j]) & mask;
          if (j == 0) l |= (uint64_t)p << low0;
          ++cj[(size_t)l];
        }
      }
      for (int t = 0; t < T; ++t)
        if (!c[(size_t)t].empty())
          for (int64_t l = 0; l < d->dims[j]; ++l) counts[j][l] += c[(size_t)t][(size_t)l];
    }
    std::vector<uint64_t>().swap(k);
  }
  return total;
}

void oracle_distinct_free(void* h) { delete static_cast<Distinct*>(h); }

// ---- merged values of chosen coordinates ----------------------------------------------------------

// coords: N arrays of n chosen coordinates (distinct); L0 = dims[0].
void* oracle_keysums_new(int N, int64_t n, const int32_t* const* coords, int64_t L0) {
  KeySums* s = new KeySums();
  s->N = N;
  s->coords.assign((size_t)N, std::vector<int32_t>((size_t)n));
  s->first_mode_hit.assign((size_t)L0, 0);
  s->vals.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int32_t c[8];
    for (int j = 0; j < N; ++j) {
      c[j] = coords[j][i];
      s->coords[(size_t)j][(size_t)i] = c[j];
    }
    s->slot[hash_coord(N, c)] = i;
    s->first_mode_hit[(size_t)c[0]] = 1;
  }
  return s;
}

// Values of the draws of a batch (in input order) at the chosen coordinates.
// Each thread scans a contiguous part of the batch; the threads' matches are
// appended in thread order, so every coordinate's values stay in input order.
void oracle_keysums_add(void* h, int64_t n, const int32_t* const* idx, const float* vals) {
  KeySums* s = static_cast<KeySums*>(h);
  const int N = s->N;
  const int T = omp_get_max_threads();
  std::vector<std::vector<std::pair<int64_t, double>>> found((size_t)T);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    const int64_t a = n * t / nt, b = n * (t + 1) / nt;
    for (int64_t e = a; e < b; ++e) {
      if (!s->first_mode_hit[(size_t)idx[0][e]]) continue;
      int32_t c[8];
      for (int j = 0; j < N; ++j) c[j] = idx[j][e];
      const auto it = s->slot.find(hash_coord(N, c));
      if (it == s->slot.end()) continue;
      bool same = true;
      for (int j = 0; j < N; ++j) same = same && s->coords[(size_t)j][(size_t)it->second] == c[j];
      if (same) found[(size_t)t].push_back({it->second, (double)vals[e]});
    }
  }
  for (int t = 0; t < T; ++t)
    for (const auto& f : found[(size_t)t]) s->vals[(size_t)f.first].push_back(f.second);
}

// out[i] = the FP64 sum, in input order, of the values at chosen coordinate i,
// rounded once to FP32; cnt[i] = how many draws it had.
void oracle_keysums_finish(void* h, float* out, int64_t* cnt) {
  KeySums* s = static_cast<KeySums*>(h);
  for (size_t i = 0; i < s->vals.size(); ++i) {
    double acc = 0.0;
    for (double v : s->vals[i]) acc += v;
    out[i] = (float)acc;
    cnt[i] = (int64_t)s->vals[i].size();
  }
}

void oracle_keysums_free(void* h) { delete static_cast<KeySums*>(h); }

}  // extern "C"
