// Device helpers shared by the kernels: tiled layouts, block storage types,
// BF16 rounding.  Included by .hip sources only.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ldg_internal.h"

namespace ldg {

// Kernel instances per N = (p+1)(p+2)/2.  The stored-block path (projection,
// assembly, block-Jacobi, operator apply, Krylov) runs up to p = 6; the
// learned preconditioner's network and factor kernels and the matrix-free
// apply up to p = 4 (the library rejects higher orders for those options).
// An N outside the list launches nothing.
#define LDG_SWITCH_N(N, CALL)                                   \
  switch (N) {                                                  \
    case 1: { constexpr int NT = 1; CALL; } break;              \
    case 3: { constexpr int NT = 3; CALL; } break;              \
    case 6: { constexpr int NT = 6; CALL; } break;              \
    case 10: { constexpr int NT = 10; CALL; } break;            \
    case 15: { constexpr int NT = 15; CALL; } break;            \
    default: break;                                             \
  }
#define LDG_SWITCH_N_P6(N, CALL)                                \
  switch (N) {                                                  \
    case 1: { constexpr int NT = 1; CALL; } break;              \
    case 3: { constexpr int NT = 3; CALL; } break;              \
    case 6: { constexpr int NT = 6; CALL; } break;              \
    case 10: { constexpr int NT = 10; CALL; } break;            \
    case 15: { constexpr int NT = 15; CALL; } break;            \
    case 21: { constexpr int NT = 21; CALL; } break;            \
    case 28: { constexpr int NT = 28; CALL; } break;            \
    default: break;                                             \
  }

// ---- stored N x N blocks: 16 bytes per lane and load ----------------------
// Block entry f = i*N + j of (triangle k, slot s) lives in group g = f / W at
//   [k/64][s][g][k%64][f%W],  W = 16 bytes / sizeof(storage type).
using bf16 = uint16_t;
using fp8 = uint8_t;   // OCP E4M3 (gfx950 conversions), factor blocks only

// Stored blocks are read once per apply: load them non-temporally so that the
// stream does not evict the coefficient vectors neighbouring tiles gather.
typedef double nt_f64x2 __attribute__((ext_vector_type(2)));
typedef float nt_f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u32x4 __attribute__((ext_vector_type(4)));

template <class BT> struct Blk;
template <> struct Blk<double> {
  static constexpr int W = 2;
  template <class T>
  __device__ static inline void load(const double* p, T* v) {
    const nt_f64x2 x = __builtin_nontemporal_load(reinterpret_cast<const nt_f64x2*>(p));
    v[0] = (T)x.x;
    v[1] = (T)x.y;
  }
};
template <> struct Blk<float> {
  static constexpr int W = 4;
  template <class T>
  __device__ static inline void load(const float* p, T* v) {
    const nt_f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const nt_f32x4*>(p));
    v[0] = (T)x.x;
    v[1] = (T)x.y;
    v[2] = (T)x.z;
    v[3] = (T)x.w;
  }
};
template <> struct Blk<bf16> {
  static constexpr int W = 8;
  template <class T>
  __device__ static inline void load(const bf16* p, T* v) {
    const nt_u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const nt_u32x4*>(p));
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = (T)__uint_as_float(w[q] << 16);
      v[2 * q + 1] = (T)__uint_as_float(w[q] & 0xffff0000u);
    }
  }
};

template <> struct Blk<fp8> {
  static constexpr int W = 16;
  template <class T>
  __device__ static inline void load(const fp8* p, T* v) {
    const nt_u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const nt_u32x4*>(p));
    const int w[4] = {(int)x.x, (int)x.y, (int)x.z, (int)x.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[4 * q + 0] = (T)__builtin_amdgcn_cvt_f32_fp8(w[q], 0);
      v[4 * q + 1] = (T)__builtin_amdgcn_cvt_f32_fp8(w[q], 1);
      v[4 * q + 2] = (T)__builtin_amdgcn_cvt_f32_fp8(w[q], 2);
      v[4 * q + 3] = (T)__builtin_amdgcn_cvt_f32_fp8(w[q], 3);
    }
  }
};

__host__ __device__ constexpr int ngroups(int N, int W) { return (N * N + W - 1) / W; }

// Packed block layout (BF16 operator blocks, and the factor's O blocks in
// every storage): with W entries per 16-byte group, the first W floor(N^2 / W)
// entries of each slot in whole groups, [k/64][s][g][k%64][W], then the other
// N^2 mod W entries of every slot together in tail groups after the slots
// (BF16, N = 15: 28 groups per slot and one tail group holding entry 224 of all
// five slots, 141 groups per triangle instead of 145).  bp_idx is the storage
// index of entry f of block s of triangle k.
__host__ __device__ constexpr int bp_full(int N, int W = 8) { return N * N / W; }
__host__ __device__ constexpr int bp_rem(int N, int W = 8) { return N * N % W; }
__host__ __device__ constexpr int bp_tail(int N, int ns, int W = 8) {
  return (ns * bp_rem(N, W) + W - 1) / W;
}
__host__ __device__ constexpr int bp_groups(int N, int ns, int W = 8) {
  return ns * bp_full(N, W) + bp_tail(N, ns, W);
}
__host__ __device__ inline int64_t bp_gidx(int64_t k, int g, int N, int ns, int W = 8) {
  return (((k >> 6) * bp_groups(N, ns, W) + g) * TILE + (k & 63)) * W;
}
__host__ __device__ inline int64_t bp_idx(int64_t k, int s, int f, int N, int ns, int W = 8) {
  const int nf = bp_full(N, W);
  if (f < W * nf) return bp_gidx(k, s * nf + f / W, N, ns, W) + f % W;
  const int t = s * bp_rem(N, W) + (f - W * nf);
  return bp_gidx(k, ns * nf + t / W, N, ns, W) + t % W;
}

__host__ __device__ inline int64_t bgidx(int64_t k, int s, int g, int ns, int ng, int W) {
  return ((((k >> 6) * ns + s) * (int64_t)ng + g) * TILE + (k & 63)) * W;
}

// round-to-nearest-even FP32 -> BF16 (finite inputs; NaN kept quiet)
// Tile of workgroup b out of nb.  Consecutive workgroups go to the 8 XCDs in
// turn, each with its own L2; giving each XCD a contiguous range of tiles keeps
// the neighbours a tile gathers in the L2 that read them as its own.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ inline bf16 to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (bf16)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}

template <class BT> __device__ inline BT from_double(double x);
template <> __device__ inline double from_double<double>(double x) { return x; }
template <> __device__ inline float from_double<float>(double x) { return (float)x; }
template <> __device__ inline bf16 from_double<bf16>(double x) { return to_bf16((float)x); }
// round to nearest even E4M3; the conversion does not saturate (448 is the
// largest finite value), so magnitudes are clamped first
template <> __device__ inline fp8 from_double<fp8>(double x) {
  const float f = (float)fmin(fmax(x, -448.0), 448.0);
  return (fp8)(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.f, 0, false) & 0xff);
}
__device__ inline float fp8_to_float(fp8 v) { return __builtin_amdgcn_cvt_f32_fp8((int)v, 0); }

// acc += Blk(k, s) z, one lane per triangle, fully unrolled over the block
template <int N, class BT, class T>
__device__ inline void block_mv(const BT* __restrict__ blocks, int64_t k, int s, int ns,
                                const T* z, T* acc) {
  constexpr int W = Blk<BT>::W;
  constexpr int NN = N * N;
  constexpr int NG = ngroups(N, W);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    T v[W];
    Blk<BT>::load(blocks + bgidx(k, s, g, ns, NG, W), v);
#pragma unroll
    for (int h = 0; h < W; ++h) {
      const int f = g * W + h;
      if (f < NN) acc[f / N] += v[h] * z[f % N];
    }
  }
}

// packed blocks: the tail entries of all ns slots of triangle k, loaded once
// per triangle (TAILN values), and acc += Blk(k, s) z from the slot's whole
// groups and its tail entries
template <int N, class BT>
__host__ __device__ constexpr int bp_tailn(int ns) {
  return bp_tail(N, ns, Blk<BT>::W) > 0 ? Blk<BT>::W * bp_tail(N, ns, Blk<BT>::W) : 1;
}

template <int N, class BT, class T>
__device__ inline void bp_tail_load(const BT* __restrict__ blocks, int64_t k, int ns, T* tail) {
  constexpr int W = Blk<BT>::W;
#pragma unroll
  for (int g = 0; g < bp_tail(N, ns, W); ++g)
    Blk<BT>::load(blocks + bp_gidx(k, ns * bp_full(N, W) + g, N, ns, W), tail + W * g);
}

template <int N, class BT, class T>
__device__ inline void block_mv_bp(const BT* __restrict__ blocks, int64_t k, int s, int ns,
                                   const T* tail, const T* z, T* acc) {
  constexpr int W = Blk<BT>::W;
  constexpr int NF = bp_full(N, W), R = bp_rem(N, W);
#pragma unroll
  for (int g = 0; g < NF; ++g) {
    T v[W];
    Blk<BT>::load(blocks + bp_gidx(k, s * NF + g, N, ns, W), v);
#pragma unroll
    for (int h = 0; h < W; ++h) {
      const int f = g * W + h;
      acc[f / N] += v[h] * z[f % N];
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int f = W * NF + j;
    acc[f / N] += tail[s * R + j] * z[f % N];
  }
}

// acc += Blk(k, s)^T z
template <int N, class BT, class T>
__device__ inline void block_mtv(const BT* __restrict__ blocks, int64_t k, int s, int ns,
                                 const T* z, T* acc) {
  constexpr int W = Blk<BT>::W;
  constexpr int NN = N * N;
  constexpr int NG = ngroups(N, W);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    T v[W];
    Blk<BT>::load(blocks + bgidx(k, s, g, ns, NG, W), v);
#pragma unroll
    for (int h = 0; h < W; ++h) {
      const int f = g * W + h;
      if (f < NN) acc[f % N] += v[h] * z[f / N];
    }
  }
}

template <int N, class T>
__device__ inline void load_vec(const T* __restrict__ v, int64_t k, T* x) {
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = v[vidx(k, i, N)];
}

template <int N, class T>
__device__ inline void store_vec(T* __restrict__ v, int64_t k, const T* x) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[vidx(k, i, N)] = x[i];
}

}  // namespace ldg
