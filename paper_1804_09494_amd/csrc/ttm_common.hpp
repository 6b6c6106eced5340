// Device helpers and the argument block shared by the TTM-chain kernels
// (csrc/ttm.hip: the Lite-bin kernels; csrc/ttm_ablation.hip: the ablation
// kernels).
#pragma once

#include "common.hpp"

namespace tk {

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct TtmArgs {
  const int64_t* bin_ptr;
  const int32_t* seg_ptr;
  const int32_t* seg_row;
  const int64_t* seg_begin;
  const int32_t* seg_slot;
  const int32_t* lay[7];    // other modes' coordinates in layout order (ascending mode)
  const float* val;
  const uint32_t* val_order;  // non-null: the value of layout position p is val[val_order[p]] (0xffffffff: zero)
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

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// s_waitcnt immediate that waits for vector memory only (vmcnt 0; expcnt and
// lgkmcnt at their maxima, gfx9 encoding)
constexpr int kVmcnt0 = 0x0F70;

// Order LDS writes of some lanes before reads of others in the same wave.  The
// hardware keeps a wave's LDS operations in order; this stops the compiler
// from treating the lanes as independent threads (it could otherwise forward
// a lane's own earlier read past another lane's write).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef short bf16x4_t __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x4_h __attribute__((ext_vector_type(4)));
typedef float floatx4_c __attribute__((ext_vector_type(4)));
// four FP32 values as the four BF16 halves of an MFMA operand, in order,
// rounded to nearest even (two v_cvt_pk_bf16_f32)
__device__ __forceinline__ bf16x4_t bf16x4_of(float a, float b, float c, float d) {
  const floatx4_c f = {a, b, c, d};
  return __builtin_bit_cast(bf16x4_t, __builtin_convertvector(f, bf16x4_h));
}

constexpr int TTMV_CPL = 2;                  // vector-ALU kernels: columns per lane
constexpr int TTMV_TILE = 64 * TTMV_CPL;     // columns per tile

// Y = 0 with a kernel (not a memset node, so the calls can be captured into a graph)
static __global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// the ablation kernels (csrc/ttm_ablation.hip)
void ttm_atomic(Ctx* c, int n, float* Y);
bool ttm_uses_fiber(int N, const int32_t* K, int n, const int* kp);
void ttm_fiber_launch(Ctx* c, const ModePlan& pl, const TtmArgs& a, int N);

}  // namespace tk
