// Device-wide sort / scan / reduce primitives (rocPRIM), wrapped with the
// context's allocator for their temporary storage.  Used by the set-up
// stages (coalescing and the Lite partition), never by the TTM-chain.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.hpp"

namespace tk {

#define TK_PRIM(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) fail(TK_ERR_DEVICE, std::string("rocprim: ") + hipGetErrorString(e_)); \
  } while (0)

void sort_pairs_u32(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, int64_t n,
                    int end_bit, Buf* keep) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::radix_sort_pairs(nullptr, tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  Buf t;
  Buf& st = keep ? *keep : t;
  ensure(c, st, tmp);
  TK_PRIM(rocprim::radix_sort_pairs(st.get(), tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  c->sync();  // a local temporary storage is released on return
}

void sort_pairs_u64_u32(Ctx* c, const uint64_t* kin, uint64_t* kout, const uint32_t* vin, uint32_t* vout, int64_t n,
                        int end_bit) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::radix_sort_pairs(nullptr, tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::radix_sort_pairs(t.get(), tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  c->sync();
}

// Key sort carrying element positions of either width.
template <class V>
static void sort_pairs_u32_impl(Ctx* c, const uint32_t* kin, uint32_t* kout, const V* vin, V* vout, int64_t n,
                                int end_bit) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::radix_sort_pairs(nullptr, tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::radix_sort_pairs(t.get(), tmp, kin, kout, vin, vout, (size_t)n, 0, end_bit, c->stream));
  c->sync();
}
void sort_pairs_u32_key(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, int64_t n,
                        int end_bit) {
  sort_pairs_u32_impl(c, kin, kout, vin, vout, n, end_bit);
}
void sort_pairs_u32_key(Ctx* c, const uint32_t* kin, uint32_t* kout, const uint64_t* vin, uint64_t* vout, int64_t n,
                        int end_bit) {
  sort_pairs_u32_impl(c, kin, kout, vin, vout, n, end_bit);
}

template <class T>
static void exclusive_scan_impl(Ctx* c, const T* in, T* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::exclusive_scan(nullptr, tmp, in, out, (T)0, (size_t)n, rocprim::plus<T>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::exclusive_scan(t.get(), tmp, in, out, (T)0, (size_t)n, rocprim::plus<T>(), c->stream));
  c->sync();
}
void exclusive_scan_pos(Ctx* c, const uint32_t* in, uint32_t* out, int64_t n) { exclusive_scan_impl(c, in, out, n); }
void exclusive_scan_pos(Ctx* c, const uint64_t* in, uint64_t* out, int64_t n) { exclusive_scan_impl(c, in, out, n); }

void exclusive_scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::exclusive_scan(nullptr, tmp, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::exclusive_scan(t.get(), tmp, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), c->stream));
  c->sync();
}

void inclusive_scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::inclusive_scan(nullptr, tmp, in, out, (size_t)n, rocprim::plus<int64_t>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::inclusive_scan(t.get(), tmp, in, out, (size_t)n, rocprim::plus<int64_t>(), c->stream));
  c->sync();
}

void exclusive_scan_i32(Ctx* c, const int32_t* in, int32_t* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  TK_PRIM(rocprim::exclusive_scan(nullptr, tmp, in, out, (int32_t)0, (size_t)n, rocprim::plus<int32_t>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::exclusive_scan(t.get(), tmp, in, out, (int32_t)0, (size_t)n, rocprim::plus<int32_t>(), c->stream));
  c->sync();
}

void reduce_max_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n) {
  size_t tmp = 0;
  TK_PRIM(rocprim::reduce(nullptr, tmp, in, out, (int64_t)INT64_MIN, (size_t)n, rocprim::maximum<int64_t>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::reduce(t.get(), tmp, in, out, (int64_t)INT64_MIN, (size_t)n, rocprim::maximum<int64_t>(), c->stream));
  c->sync();
}

void reduce_min_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n) {
  size_t tmp = 0;
  TK_PRIM(rocprim::reduce(nullptr, tmp, in, out, (int64_t)INT64_MAX, (size_t)n, rocprim::minimum<int64_t>(), c->stream));
  Buf t(c, tmp);
  TK_PRIM(rocprim::reduce(t.get(), tmp, in, out, (int64_t)INT64_MAX, (size_t)n, rocprim::minimum<int64_t>(), c->stream));
  c->sync();
}

}  // namespace tk
