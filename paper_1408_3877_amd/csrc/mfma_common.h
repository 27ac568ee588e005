// Matrix-core (MFMA) helpers shared by the block assembly and the matrix-free
// apply on gfx950.  For the 16x16 instructions a lane holds A[row = lane % 16]
// [k = lane / 16] (16x16x32 BF16: k = 8 (lane / 16) .. + 7) and B[k][col =
// lane % 16]; result lanes: FP64 holds rows 4r + lane/16, FP32 and BF16 hold
// rows 4(lane/16) + r, column lane % 16 (r = 0..3), as measured on gfx950.
#pragma once
#include "device_common.h"

namespace ldg {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));

template <int PREC> struct Mfma;
template <> struct Mfma<0> {   // V_MFMA_F64_16X16X4_F64
  using A = double; using B = double; using Acc = d4_t; using Out = double;
  static constexpr int KS = 4;   // k per instruction
  __device__ static inline Acc run(A a, B b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int r, int q) { return 4 * r + q; }
};
template <> struct Mfma<1> {   // V_MFMA_F32_16X16X4_F32
  using A = float; using B = float; using Acc = f4_t; using Out = float;
  static constexpr int KS = 4;
  __device__ static inline Acc run(A a, B b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int r, int q) { return 4 * q + r; }
};
template <> struct Mfma<2> {   // V_MFMA_F32_16X16X32_BF16
  using A = s8_t; using B = s8_t; using Acc = f4_t; using Out = bf16;
  static constexpr int KS = 32;
  __device__ static inline Acc run(A a, B b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int r, int q) { return 4 * q + r; }
};

template <class T> __device__ inline T zero_acc();
template <> __device__ inline d4_t zero_acc<d4_t>() { return d4_t{0.0, 0.0, 0.0, 0.0}; }
template <> __device__ inline f4_t zero_acc<f4_t>() { return f4_t{0.f, 0.f, 0.f, 0.f}; }

__device__ inline int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace ldg
