// Matrix-free block terms of the divergence half on the matrix cores.
//
// The D-dependent part of the eliminated operator (Sec. 3.6.3, 3.6.6, 3.6.7),
//   sum_m B^m_kk Z^m_k + sum_n U_kn (nu^1_kn Z^1_k+ + nu^2_kn Z^2_k+),
// is applied without the stored blocks: with P_t = sum_l D_kl T_t(l) for the
// element tensors T_t = G_hat(.,.,l,1), G_hat(.,.,l,2), R_hat_diag(.,.,l,n)
// and B^m = sum_t w^m_t P_t (geometry weights w), the element part is
//   y_i = sum_t sum_{l,j} T_t(l)_ij D_kl u_tj,  u_t = w^1_t Z^1_k + w^2_t Z^2_k,
// a contraction over the pair (l, j): a GEMM whose A operand is the tensor
// (rows i, the pair as the reduction index) shared by the 16 triangles of a
// wave, and whose B operand is the per-triangle outer product D_kl u_tj.
// The edge part is the same with the neighbour's coefficient, the tensor
// R_hat_off(.,.,l,n,n+) and w = 1/2 |E_kn| (nu^1 Z^1_k+ + nu^2 Z^2_k+).  All
// tensors accumulate into one 16 x 16 tile per wave (rows i, columns the
// triangles), so each lane ends with four entries of y.
//
// Pair order: l outer, j inner, j padded to NJ = 4 ceil(N / 4); one k-step
// takes the four pairs (l, 4 jb + q), q = lane / 16, so a lane needs u only at
// j = q, q + 4, ... and D at every l (kept in registers).
//   PREC 0: V_MFMA_F64_16X16X4_F64 on FP64 vectors
//   PREC 1: V_MFMA_F32_16X16X4_F32 on FP32 vectors (FP32 operands and sums)
#include "device_common.h"
#include "kernels.h"
#include "mfma_common.h"

namespace ldg {

namespace {

constexpr int NT_ELEM = 5;   // G1, G2, Rd0, Rd1, Rd2; then Ro(n, n+) at 5 + 3 n + n+

template <int N>
__host__ __device__ constexpr int mf_steps() {   // k-steps per tensor
  return N * ((N + 3) / 4);
}

}  // namespace

int mf_table_size(int N) { return 14 * N * ((N + 3) / 4) * 64; }

// A operands: table[t][s][lane], s = l * NJB + jb, lane = 16 q + i:
// T_t(l)_{i, 4 jb + q}, zero for i >= N or 4 jb + q >= N
void mf_build_table(int N, const double* const* tens, double* out) {
  const int NJB = (N + 3) / 4, NS = N * NJB, NN = N * N;
  for (int t = 0; t < 14; ++t)
    for (int l = 0; l < N; ++l)
      for (int jb = 0; jb < NJB; ++jb)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, j = 4 * jb + (lane >> 4);
          const double v = (i < N && j < N) ? tens[t][(size_t)l * NN + i * N + j] : 0.0;
          out[((size_t)t * NS + l * NJB + jb) * 64 + lane] = v;
        }
}

// A operands come straight from the tables (L1/L2-resident, coalesced 64-lane
// loads); staging them in LDS per block or reusing them over several triangle
// groups per wave measured slower on the 2M-triangle p = 4 workload.
template <int N, int PREC, class T>
__global__ void __launch_bounds__(256) k_mf_blocks(Geo g, const double* __restrict__ D,
                                                   const typename Mfma<PREC>::A* __restrict__ A,
                                                   const T* __restrict__ C,
                                                   const T* __restrict__ Z1,
                                                   const T* __restrict__ Z2, double tau,
                                                   T* __restrict__ y,
                                                   double* __restrict__ partials) {
  using M = Mfma<PREC>;
  using Acc = typename M::Acc;
  using V = typename M::B;   // operand type: double or float
  using AT = typename M::A;
  constexpr int NJB = (N + 3) / 4;
  constexpr int NS = mf_steps<N>();
  __shared__ int sb[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, q = lane >> 4;
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * 64 + wave * 16 + col;
  const bool valid = k < g.K;
  const int64_t Kp = g.Kpad;
  Acc acc = zero_acc<Acc>();
  // element tensors: u_t = w^1_t Z^1 + w^2_t Z^2 at j = 4 jb + q, D at every l
  {
    double wgt[2][NT_ELEM];
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
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT_ELEM; ++t) wgt[0][t] = wgt[1][t] = 0.0;
    }
    V dl[N], u[NT_ELEM][NJB];
#pragma unroll
    for (int l = 0; l < N; ++l) dl[l] = valid ? (V)D[vidx(k, l, N)] : (V)0;
#pragma unroll
    for (int jb = 0; jb < NJB; ++jb) {
      const int j = 4 * jb + q;
      const double z1 = (valid && j < N) ? (double)Z1[vidx(k, j, N)] : 0.0;
      const double z2 = (valid && j < N) ? (double)Z2[vidx(k, j, N)] : 0.0;
#pragma unroll
      for (int t = 0; t < NT_ELEM; ++t) u[t][jb] = (V)(wgt[0][t] * z1 + wgt[1][t] * z2);
    }
#pragma unroll
    for (int t = 0; t < NT_ELEM; ++t) {
      const AT* At = A + (size_t)t * NS * 64 + lane;
#pragma unroll
      for (int l = 0; l < N; ++l)
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb) acc = M::run(At[(l * NJB + jb) * 64], dl[l] * u[t][jb], acc);
    }
  }
  // edge tensors: the neighbour's coefficient and w = 1/2 |E| (nu^1 Z^1_k+ + nu^2 Z^2_k+)
  for (int n = 0; n < 3; ++n) {
    const int64_t p = valid ? g.nbr[n * Kp + k] : -1;
    const int npl = p >= 0 ? g.nbrn[n * Kp + k] : 0;
    // the candidates n+ of the block's triangles (one on structured meshes),
    // block-uniform so that every wave runs the same tensors
    int mn = wave_min(p >= 0 ? npl : 3), mx = wave_max(p >= 0 ? npl : -1);
    __syncthreads();
    if (lane == 0) {
      sb[0][wave] = mn;
      sb[1][wave] = mx;
    }
    __syncthreads();
    mn = min(min(sb[0][0], sb[0][1]), min(sb[0][2], sb[0][3]));
    mx = max(max(sb[1][0], sb[1][1]), max(sb[1][2], sb[1][3]));
    if (mx < 0) continue;   // no interior edge n in this block (block-uniform)
    V dn[N], w[NJB];
#pragma unroll
    for (int l = 0; l < N; ++l) dn[l] = p >= 0 ? (V)D[vidx(p, l, N)] : (V)0;
    double s1 = 0.0, s2 = 0.0;
    if (p >= 0) {
      const double hl = 0.5 * g.elen[n * Kp + k];
      s1 = hl * g.nu[(2 * n) * Kp + k];
      s2 = hl * g.nu[(2 * n + 1) * Kp + k];
    }
#pragma unroll
    for (int jb = 0; jb < NJB; ++jb) {
      const int j = 4 * jb + q;
      double s = 0.0;
      if (p >= 0 && j < N) s = s1 * (double)Z1[vidx(p, j, N)] + s2 * (double)Z2[vidx(p, j, N)];
      w[jb] = (V)s;
    }
    for (int b = mn; b <= mx; ++b) {
      const V on = (p >= 0 && npl == b) ? (V)1 : (V)0;
      const AT* At = A + (size_t)(NT_ELEM + 3 * n + b) * NS * 64 + lane;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        const V dlb = on * dn[l];
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb) acc = M::run(At[(l * NJB + jb) * 64], dlb * w[jb], acc);
      }
    }
  }
  // y_i += tau * acc (rows i < N of this lane), and <C, y> for the fused dot
  double dot = 0.0;
  if (valid) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = M::row(r, q);
      if (i < N) {
        const int64_t id = vidx(k, i, N);
        const T v = y[id] + (T)(tau * (double)acc[r]);
        y[id] = v;
        dot += (double)C[id] * (double)v;
      }
    }
  }
  if (partials == nullptr) return;
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
  if (lane == 0) red[wave] = dot;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

void launch_mf_blocks(int N, int vt, const Geo& g, const double* D, const void* table,
                      const void* C, const void* Z1, const void* Z2, double tau, void* y,
                      const Reducer* red, hipStream_t st) {
  const unsigned nb = (unsigned)(g.Kpad / 64);   // 64 triangles (one tile) per block
  double* parts = red ? red->partials : nullptr;
  if (vt == VT_F64) {
    LDG_SWITCH_N(N, (k_mf_blocks<NT, 0, double><<<nb, 256, 0, st>>>(
                        g, D, (const double*)table, (const double*)C, (const double*)Z1,
                        (const double*)Z2, tau, (double*)y, parts)));
  } else {
    LDG_SWITCH_N(N, (k_mf_blocks<NT, 1, float><<<nb, 256, 0, st>>>(
                        g, D, (const float*)table, (const float*)C, (const float*)Z1,
                        (const float*)Z2, tau, (float*)y, parts)));
  }
  if (red) reduce_partials((int)nb, red->partials, red->result, st, red->cg, red->cg_mode);
}

}  // namespace ldg
