// Block assembly on the matrix cores (Sec. 3.6.3, 3.6.6, 3.6.7).
//
// Per triangle k the D-dependent blocks are contractions of its projected
// coefficient D_k (or a neighbour's) with reference tensors:
//   P_t = sum_l D_kl T_t(l, :, :),  T_t = G_hat(:,:,l,1), G_hat(:,:,l,2), R_hat_diag(:,:,l,n)
//   B^m_kk = sum_t w^m_t(k) P_t      (w: geometry, normals, edge lengths, edge kinds)
//   U_kn   = 1/2 |E_kn| sum_l D_{k+ l} R_hat_off(:,:,l,n,n+)
// Written transposed, block^T(f, k) = sum_l T(f, l) D(l, k) with f = i*N + j,
// this is a GEMM whose A operand (the tensor, 16 entries f x 4 or 32 l) is
// shared by the 16 triangles of a wave and whose B operand holds their
// coefficients.  One wave owns 16 triangles (4 waves = one 64-triangle
// storage tile) and sweeps the N*N entries in 16-row tiles; each output
// column is one triangle, so the per-triangle weights are per-lane scalars.
//
//   PREC 0: V_MFMA_F64_16X16X4_F64, FP64 blocks
//   PREC 1: V_MFMA_F32_16X16X4_F32, FP32 blocks (FP32 operands and accumulation)
//   PREC 2: V_MFMA_F32_16X16X32_BF16, BF16 operands, FP32 accumulation, BF16 blocks
//
// Result lanes: FP64 holds rows 4r + lane/16, FP32 and BF16 hold rows
// 4(lane/16) + r, column lane%16 (r = 0..3), as measured on gfx950.
// The neighbour's edge n+ selects the R_hat_off tensor; when the 16 triangles
// of a wave disagree on it (only on irregular meshes) all three candidates
// are computed and each lane keeps its own.
#include "device_common.h"
#include "kernels.h"
#include "mfma_common.h"

namespace ldg {

namespace {

constexpr int NT_ELEM = 5;   // G1, G2, Rd0, Rd1, Rd2

// B operand of k-step ks for coefficient vector of triangle kk (or zeros)
template <int N, int PREC>
__device__ inline typename Mfma<PREC>::B b_operand(const double* __restrict__ D, int64_t kk, int ks,
                                                   int q) {
  if constexpr (PREC == 2) {
    s8_t v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int l = 8 * q + j;
      const float x = (kk >= 0 && l < N) ? (float)D[vidx(kk, l, N)] : 0.f;
      v[j] = (short)to_bf16(x);
    }
    return v;
  } else {
    const int l = 4 * ks + q;
    const double x = (kk >= 0 && l < N) ? D[vidx(kk, l, N)] : 0.0;
    return (typename Mfma<PREC>::B)x;
  }
}

// A operand: tensor t, k-step ks, 16-row tile ft; layouts
//   PREC 0, 1: [t][mfma_lrows(N)][NFP] (l-major), PREC 2: [t][NFP][32] (f-major, l contiguous)
template <int N, int PREC>
__device__ inline typename Mfma<PREC>::A a_operand(const void* __restrict__ T, int t, int ks,
                                                   int ft, int lane) {
  constexpr int NN = N * N;
  constexpr int NFP = (NN + 15) / 16 * 16;
  const int col = lane & 15, q = lane >> 4;
  const int f = 16 * ft + col;
  if constexpr (PREC == 2) {
    const bf16* p = static_cast<const bf16*>(T) + ((int64_t)t * NFP + f) * 32 + 8 * q;
    return *reinterpret_cast<const s8_t*>(p);
  } else {
    using A = typename Mfma<PREC>::A;
    const A* p = static_cast<const A*>(T);
    return p[((int64_t)t * mfma_lrows(N) + 4 * ks + q) * NFP + f];
  }
}

template <int N, int PREC>
__device__ inline void store_col(typename Mfma<PREC>::Out* __restrict__ blocks, int64_t k, int s,
                                 int ft, int q, const float* vf, const double* vd) {
  constexpr int NN = N * N;
  if constexpr (PREC == 0) {
    constexpr int NG = ngroups(N, 2);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * ft + Mfma<0>::row(r, q);
      if (f < NG * 2) blocks[bgidx(k, s, f >> 1, NSLOT, NG, 2) + (f & 1)] = vd[r];
    }
  } else if constexpr (PREC == 1) {
    constexpr int NG = ngroups(N, 4);
    const int gi = 4 * ft + q;   // rows 16 ft + 4q .. +3 form one group of four
    if (gi < NG)
      *reinterpret_cast<float4*>(blocks + bgidx(k, s, gi, NSLOT, NG, 4)) =
          make_float4(vf[0], vf[1], vf[2], vf[3]);
  } else {
    // packed BF16 layout: rows 16 ft + 4q .. +3 are half a group, or tail entries
    const int f0 = 16 * ft + 4 * q;
    if (f0 < 8 * bp_full(N, 8)) {
      uint2 w;
      w.x = (uint32_t)to_bf16(vf[0]) | ((uint32_t)to_bf16(vf[1]) << 16);
      w.y = (uint32_t)to_bf16(vf[2]) | ((uint32_t)to_bf16(vf[3]) << 16);
      *reinterpret_cast<uint2*>(blocks + bp_idx(k, s, f0, N, NSLOT, 8)) = w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (f0 + j < NN) blocks[bp_idx(k, s, f0 + j, N, NSLOT, 8)] = to_bf16(vf[j]);
    }
  }
  (void)NN;
}

}  // namespace

template <int N, int PREC>
__global__ void __launch_bounds__(256) k_assemble_mfma(Geo g, const double* __restrict__ D,
                                                       const void* __restrict__ T,
                                                       typename Mfma<PREC>::Out* __restrict__ blocks) {
  using M = Mfma<PREC>;
  using Acc = typename M::Acc;
  constexpr int NN = N * N;
  constexpr int NFT = (NN + 15) / 16;
  constexpr int NKS = PREC == 2 ? 1 : (N + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, q = lane >> 4;
  const int64_t k = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + col;
  const bool valid = k < g.K;
  const int64_t Kp = g.Kpad;
  // per-column (per-triangle) weights
  double wgt[2][NT_ELEM], uo[3];
  int npl[3];
  int64_t kp[3];
  if (valid) {
    const double B11 = g.B[k], B12 = g.B[Kp + k], B21 = g.B[2 * Kp + k], B22 = g.B[3 * Kp + k];
    wgt[0][0] = -B22; wgt[0][1] = B21;      // -G^1 = -(B22 G1 - B21 G2)
    wgt[1][0] = B12;  wgt[1][1] = -B11;     // -G^2 = -(-B12 G1 + B11 G2)
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int kind = g.kind[n * Kp + k];
      const double L = g.elen[n * Kp + k];
      const double c = kind == LDG_EDGE_INTERIOR ? 0.5 : (kind == LDG_EDGE_DIRICHLET ? 1.0 : 0.0);
      wgt[0][2 + n] = c * g.nu[(2 * n) * Kp + k] * L;
      wgt[1][2 + n] = c * g.nu[(2 * n + 1) * Kp + k] * L;
      kp[n] = g.nbr[n * Kp + k];
      npl[n] = kp[n] >= 0 ? g.nbrn[n * Kp + k] : 0;
      uo[n] = kp[n] >= 0 ? 0.5 * L : 0.0;
    }
  } else {
#pragma unroll
    for (int t = 0; t < NT_ELEM; ++t) wgt[0][t] = wgt[1][t] = 0.0;
#pragma unroll
    for (int n = 0; n < 3; ++n) { kp[n] = -1; npl[n] = 0; uo[n] = 0.0; }
  }
  // B operands: own coefficients and the three neighbours'
  typename M::B bD[NKS], bN[3][NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    bD[ks] = b_operand<N, PREC>(D, valid ? k : -1, ks, q);
#pragma unroll
    for (int n = 0; n < 3; ++n) bN[n][ks] = b_operand<N, PREC>(D, kp[n], ks, q);
  }
  // n+ shared by the wave's triangles for each local edge? (-2: no neighbours)
  int unif[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const int mn = wave_min(kp[n] >= 0 ? npl[n] : 3);
    const int mx = wave_max(kp[n] >= 0 ? npl[n] : -1);
    unif[n] = mx < 0 ? -2 : (mn == mx ? mn : -1);
  }
  for (int ft = 0; ft < NFT; ++ft) {
    // element blocks
    Acc acc[NT_ELEM];
#pragma unroll
    for (int t = 0; t < NT_ELEM; ++t) acc[t] = zero_acc<Acc>();
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int t = 0; t < NT_ELEM; ++t)
        acc[t] = M::run(a_operand<N, PREC>(T, t, ks, ft, lane), bD[ks], acc[t]);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double vd[4];
      float vf[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NT_ELEM; ++t) s += wgt[m][t] * (double)acc[t][r];
        vd[r] = s;
        vf[r] = (float)s;
      }
      store_col<N, PREC>(blocks, k, m, ft, q, vf, vd);
    }
    // edge blocks
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      double vd[4] = {0.0, 0.0, 0.0, 0.0};
      float vf[4] = {0.f, 0.f, 0.f, 0.f};
      if (unif[n] >= 0) {
        Acc a = zero_acc<Acc>();
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks)
          a = M::run(a_operand<N, PREC>(T, NT_ELEM + 3 * n + unif[n], ks, ft, lane), bN[n][ks], a);
#pragma unroll
        for (int r = 0; r < 4; ++r) vd[r] = uo[n] * (double)a[r];
      } else if (unif[n] == -1) {
        Acc a[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          a[b] = zero_acc<Acc>();
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            a[b] = M::run(a_operand<N, PREC>(T, NT_ELEM + 3 * n + b, ks, ft, lane), bN[n][ks], a[b]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          vd[r] = uo[n] * (double)(npl[n] == 0 ? a[0][r] : (npl[n] == 1 ? a[1][r] : a[2][r]));
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) vf[r] = (float)vd[r];
      store_col<N, PREC>(blocks, k, 2 + n, ft, q, vf, vd);
    }
  }
}

namespace {
inline unsigned nblk64(int64_t Kpad) { return (unsigned)(Kpad / 64); }
}

void launch_assemble_mfma(int N, int bt, const Geo& g, const double* D, const void* T, void* blocks,
                          hipStream_t st) {
  const unsigned nb = nblk64(g.Kpad);
  if (bt == BT_F64) {
    LDG_SWITCH_N_P6(N, (k_assemble_mfma<NT, 0><<<nb, 256, 0, st>>>(g, D, T, (double*)blocks)));
  } else if (bt == BT_F32) {
    LDG_SWITCH_N_P6(N, (k_assemble_mfma<NT, 1><<<nb, 256, 0, st>>>(g, D, T, (float*)blocks)));
  } else {
    LDG_SWITCH_N_P6(N, (k_assemble_mfma<NT, 2><<<nb, 256, 0, st>>>(g, D, T, (bf16*)blocks)));
  }
}

}  // namespace ldg
