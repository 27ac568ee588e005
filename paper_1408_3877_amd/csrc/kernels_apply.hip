// Operator application and block-Jacobi application, templated on the
// vector type T (double, or float for the inner solves of the mixed modes)
// and the storage type BT of the stored blocks (double, float, bf16), with
// arithmetic and accumulation in T.  One lane per triangle.
//
// Gradient half:   Z^m = -M^{-1} (A^m C + J^m),  A^m = -H^m + Q^m + Q^m_N
// Divergence half: y = alpha M C + tau (eta (S + S_D) C + sum_m B^m Z^m),
//                  B^m = -G^m + R^m + R^m_D   (eq:timeDepSystem)
// H, Q, S enter through the reference matrices H_hat, S_hat_diag, S_hat_off
// (Sec. 3.6.2, 3.6.4, 3.6.5), kept in LDS or, in the FP32 gradient kernel, read
// through the scalar cache; G and R through the stored blocks.
#include "device_common.h"
#include "kernels.h"

namespace ldg {

namespace {

constexpr int NREF = 14;  // H1, H2, Sd[3], So[3][3]
__device__ inline int ref_h(int m) { return m; }
__device__ inline int ref_sd(int n) { return 2 + n; }
__device__ inline int ref_so(int a, int b) { return 5 + 3 * a + b; }

// FP32 reference matrices in LDS with rows padded to whole 16-byte vectors, so
// that a row is read with ceil(N / 4) LDS instructions instead of N (measured
// faster for the FP32 kernels); FP64 rows stay unpadded with scalar reads
// (the 16-byte form measured slower there)
template <class T> constexpr int lds_w() { return sizeof(T) == 4 ? 4 : 1; }
template <int N, class T> constexpr int row_stride() { return (N + lds_w<T>() - 1) / lds_w<T>() * lds_w<T>(); }
template <int N, class T> constexpr int ref_size() { return NREF * N * row_stride<N, T>(); }
// FP64 matrices of N = 28 (86 KiB) exceed 64 KiB of LDS: those kernels read
// them from global memory, where FP64 rows have the same unpadded layout
template <int N, class T> constexpr bool refs_in_lds() { return ref_size<N, T>() * sizeof(T) <= 65536; }

template <int N, class T>
__device__ inline void load_refs(T* sm, const double* __restrict__ g) {
  constexpr int RS = row_stride<N, T>();
  for (int t = threadIdx.x; t < ref_size<N, T>(); t += blockDim.x) {
    const int row = t / RS, j = t % RS;   // row = matrix * N + i
    sm[t] = j < N ? (T)g[row * N + j] : (T)0;
  }
  __syncthreads();
}

template <int N, class T>
__device__ inline void mv_add(const T* __restrict__ A, const T* x, T* acc, T scale) {
  constexpr int W = lds_w<T>(), RS = row_stride<N, T>();
  typedef T vec __attribute__((ext_vector_type(W)));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = 0;
#pragma unroll
    for (int jb = 0; jb < RS / W; ++jb) {
      const vec v = *reinterpret_cast<const vec*>(A + i * RS + jb * W);
#pragma unroll
      for (int e = 0; e < W; ++e)
        if (jb * W + e < N) s += v[e] * x[jb * W + e];
    }
    acc[i] += scale * s;
  }
}

// acc += scale * A x with A (N x N, row-major) in global memory at an address
// that is the same for every lane of the wave: each entry is one scalar-cache
// load and the SGPR operand of the vector FMA, so the products need no LDS
// traffic (broadcast LDS reads of the matrices bound the gradient kernel)
template <int N, class T>
__device__ inline void mv_add_s(const T* __restrict__ A, const T* x, T* acc, T scale) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) s += A[i * N + j] * x[j];
    acc[i] += scale * s;
  }
}

// acc += A x for A = H1 or H2: row i holds the integrals of d phi_i / d x_m
// against phi_j, which vanish unless phi_j has a lower degree than phi_i (the
// derivative has degree deg(i) - 1 and the basis is orthogonal and ordered by
// degree), so only the columns j < deg(i) (deg(i) + 1) / 2 are read
__host__ __device__ constexpr int h_cols(int i) {
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= i) ++d;
  return d * (d + 1) / 2;
}
template <int N, class T>
__device__ inline void mv_add_h(const T* __restrict__ A, const T* x, T* acc) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < h_cols(i); ++j) s += A[i * N + j] * x[j];
    acc[i] += s;
  }
}

// Gauss points per edge of the C traces of the FP32 gradient kernel: p + 1,
// exact for the degree-2p products of S_diag and S_off
__host__ __device__ constexpr int c_trace_points(int N) {
  int p = 0;
  while ((p + 1) * (p + 2) / 2 < N) ++p;
  return p + 1;
}

}  // namespace

// The 14 reference matrices (H1, H2, S_diag[3], S_off[3][3]), N x N each: the
// FP32 kernel reads them through the scalar cache (rT, FP32 copy); the FP64
// kernel keeps them in LDS (as SGPR operands its products spill registers).
// TR (FP32 only), for the quadrature form of the divergence half (k_div_q):
//   sig[k][n][q] = d_h(x_q) (nu_n . Z_h)(x_q)  at the Gauss points x_q of each
//     interior or Dirichlet edge n (its own parametrisation; trT[n][q][j] =
//     phi_j at point q of reference edge n, dE = d_h at the same points),
//   pen[k] = eta (S_diag + S_D) C - eta S_off C+, the penalty rows of the
//     divergence half, from the C traces the gradient's edge terms use.
template <int N, class T, bool TR>
__global__ void __launch_bounds__(256) k_grad(Geo g, const double* __restrict__ refs,
                                              const T* __restrict__ rT,
                                              const T* __restrict__ C, const T* __restrict__ J1,
                                              const T* __restrict__ J2, T* __restrict__ Z1,
                                              T* __restrict__ Z2, const float* __restrict__ dE,
                                              const float* __restrict__ trT,
                                              float* __restrict__ sig, float* __restrict__ pen,
                                              float eta) {
  static_assert(!TR || sizeof(T) == 4, "edge traces are an FP32 form");
  constexpr int NN = N * N;
  constexpr bool SC = sizeof(T) == 4;
  constexpr bool LDSR = !SC && refs_in_lds<N, T>();
  __shared__ __align__(16) T smem[LDSR ? ref_size<N, T>() : 1];
  const T* sm = rT;
  if constexpr (LDSR) {
    load_refs<N, T>(smem, refs);
    sm = smem;
  }
  auto mv = [&](int ref, const T* x, T* acc, T scale) {
    mv_add<N, T>(sm + ref * N * row_stride<N, T>(), x, acc, scale);
  };
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  T a1[N], a2[N];
#pragma unroll
  for (int i = 0; i < N; ++i) a1[i] = a2[i] = 0;
  if (k >= g.K) {
    store_vec<N, T>(Z1, k, a1);
    store_vec<N, T>(Z2, k, a2);
    if constexpr (TR) store_vec<N, T>(pen, k, a1);
    return;
  }
  const int64_t Kp = g.Kpad;
  T c[N];
  load_vec<N, T>(C, k, c);
  // FP32: the geometry from its FP32 copies (the same values in half the bytes)
  auto geoB = [&](int q) { if constexpr (SC) return g.B32[q * Kp + k]; else return (T)g.B[q * Kp + k]; };
  const T B11 = geoB(0), B12 = geoB(1), B21 = geoB(2), B22 = geoB(3);
  {
    // -H^1 = -(B22 H1 - B21 H2), -H^2 = -(-B12 H1 + B11 H2)   (Sec. 3.6.2)
    T u1[N], u2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) u1[i] = u2[i] = 0;
    if constexpr (SC) {
      mv_add_h<N, T>(rT + ref_h(0) * NN, c, u1);
      mv_add_h<N, T>(rT + ref_h(1) * NN, c, u2);
    } else {
      mv(ref_h(0), c, u1, (T)1);
      mv(ref_h(1), c, u2, (T)1);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      a1[i] -= B22 * u1[i] - B21 * u2[i];
      a2[i] -= -B12 * u1[i] + B11 * u2[i];
    }
  }
  T pv[TR ? N : 1];
#pragma unroll
  for (int i = 0; i < (TR ? N : 1); ++i) pv[i] = 0;
  for (int n = 0; n < 3; ++n) {
    const int kind = g.kind[n * Kp + k];
    if (kind == LDG_EDGE_DIRICHLET && !TR) continue;
    T L, nu1, nu2;
    if constexpr (SC) {
      L = g.elen32[n * Kp + k];
      nu1 = g.nu32[(2 * n) * Kp + k];
      nu2 = g.nu32[(2 * n + 1) * Kp + k];
    } else {
      L = (T)g.elen[n * Kp + k];
      nu1 = (T)g.nu[(2 * n) * Kp + k];
      nu2 = (T)g.nu[(2 * n + 1) * Kp + k];
    }
    const T cq = (kind == LDG_EDGE_INTERIOR ? (T)0.5 : (T)1) * L;
    T s[N];
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = 0;
    if constexpr (SC) {
      // S_diag(n) c and S_off(n, n+) c+ through the traces at the p + 1 Gauss
      // points of the edge, own_q = c(x_q) and nb_q = c+(x_q); x_q is point
      // Q-1-q of the neighbour's edge n+.  Gradient (interior and Neumann
      // edges): s_i = sum_q w_q phi_i(x_q) (cq own_q + L/2 nb_q).  Penalty (TR;
      // interior and Dirichlet edges): eta sum_q w_q phi_i(x_q) (own_q - nb_q).
      // rT holds after the 14 matrices tc[3][Q][N] (phi_j at point q of
      // reference edge n) and lc[3][Q][N] (w_q phi_i at the same points).
      constexpr int Q = c_trace_points(N);
      const T* tc = rT + NREF * NN;
      const T* lc = tc + 3 * Q * N;
      T own[Q], nb[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        T v = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) v += tc[(n * Q + q) * N + j] * c[j];
        own[q] = v;
        nb[q] = 0;
      }
      if (kind == LDG_EDGE_INTERIOR) {
        const int64_t kp = g.nbr[n * Kp + k];
        const int np = g.nbrn[n * Kp + k];
        T cp[N];
        load_vec<N, T>(C, kp, cp);
        // n+ per lane: one wave-uniform trace matrix per candidate (a single
        // candidate on structured meshes; the others are skipped)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (np == b) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              T v = 0;
#pragma unroll
              for (int j = 0; j < N; ++j) v += tc[(b * Q + Q - 1 - q) * N + j] * cp[j];
              nb[q] = v;
                  }
          }
      }
      // both lifts in one pass over the table: the gradient's (interior and
      // Neumann edges) into s, the penalty's (TR; interior and Dirichlet
      // edges) into pv
      const T gw = kind != LDG_EDGE_DIRICHLET ? (T)1 : (T)0;
      const T pw = TR && kind != LDG_EDGE_NEUMANN ? (T)eta : (T)0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const T u = gw * (cq * own[q] + (T)0.5 * L * nb[q]);
        const T up = pw * (own[q] - nb[q]);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const T l = lc[(n * Q + q) * N + i];
          s[i] += l * u;
          if constexpr (TR) pv[i] += l * up;
        }
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        a1[i] += nu1 * s[i];
        a2[i] += nu2 * s[i];
      }
    } else {
      mv(ref_sd(n), c, s, cq);
      if (kind == LDG_EDGE_INTERIOR) {
        const int64_t kp = g.nbr[n * Kp + k];
        const int np = g.nbrn[n * Kp + k];
        T cp[N];
        load_vec<N, T>(C, kp, cp);
        mv(ref_so(n, np), cp, s, (T)0.5 * L);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        a1[i] += nu1 * s[i];
        a2[i] += nu2 * s[i];
      }
    }
  }
  if (J1 != nullptr) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      a1[i] += J1[vidx(k, i, N)];
      a2[i] += J2[vidx(k, i, N)];
    }
  }
  T inv;
  if constexpr (SC) inv = g.ainv32[k];
  else inv = (T)(-1.0 / g.area2[k]);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    a1[i] *= inv;
    a2[i] *= inv;
  }
  store_vec<N, T>(Z1, k, a1);
  store_vec<N, T>(Z2, k, a2);
  if constexpr (TR) {
    store_vec<N, T>(pen, k, pv);
    constexpr int Q = edge_trace_points(N), NQ = 3 * Q;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      if (g.kind[n * Kp + k] == LDG_EDGE_NEUMANN) continue;   // no flux term there
      const float nu1 = g.nu32[(2 * n) * Kp + k], nu2 = g.nu32[(2 * n + 1) * Kp + k];
      float zn[N];
#pragma unroll
      for (int j = 0; j < N; ++j) zn[j] = nu1 * a1[j] + nu2 * a2[j];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float v = 0.0f;
#pragma unroll
        for (int j = 0; j < N; ++j) v += trT[(n * Q + q) * N + j] * zn[j];
        sig[vidx(k, n * Q + q, NQ)] = dE[vidx(k, n * Q + q, NQ)] * v;
      }
    }
  }
}

// The divergence half in the quadrature form of the FP32 apply (no stored
// blocks): y = alpha M C + tau (pen + sum_m B^m Z^m) with
//   -G^m Z^m  (eq:hatG): sum over the exact volume rule of w_q d_h(x_q)
//       dphi_i/dx_m(x_q) Z^m(x_q), with dvol[k][q] = w_q d_h(x_q) and
//       vt[q][0..2][.] = phi, dphi/dx1_hat, dphi/dx2_hat at x_q;
//   R^m, R^m_D (eq:hatRdiag, eq:hatRoffdiag): per interior edge |E| sum_q
//       w_q phi_i(x_q) (sig_k(x_q) - sig_k+(x_q)) / 2, per Dirichlet edge
//       |E| sum_q w_q phi_i(x_q) sig_k(x_q), from the flux traces sig that
//       k_grad wrote (the neighbour's at its point Q-1-q, its normal -nu);
//   pen: the penalty rows k_grad wrote.
// partials (optional): per-block sums of <C, y>.
template <int N>
__global__ void __launch_bounds__(256) k_div_q(Geo g, const float* __restrict__ C,
                                               const float* __restrict__ Z1,
                                               const float* __restrict__ Z2,
                                               const float* __restrict__ pen, double alpha,
                                               double tau, float* __restrict__ y,
                                               double* __restrict__ partials,
                                               const float* __restrict__ sig,
                                               const float* __restrict__ dvol,
                                               const float* __restrict__ vt,
                                               const float* __restrict__ lift) {
  constexpr int Q = edge_trace_points(N), NQ = 3 * Q, RV = vol_points(N);
  __shared__ double red[4];
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t Kp = g.Kpad;
  double dot = 0.0;
  if (k < Kp) {
    float t[N];
    if (k >= g.K) {
#pragma unroll
      for (int i = 0; i < N; ++i) t[i] = 0.0f;
      store_vec<N, float>(y, k, t);
    } else {
      load_vec<N, float>(pen, k, t);
      if constexpr (RV > 0) {
        float z1[N], z2[N];
        load_vec<N, float>(Z1, k, z1);
        load_vec<N, float>(Z2, k, z2);
        const float B11 = g.B32[k], B12 = g.B32[Kp + k], B21 = g.B32[2 * Kp + k],
                    B22 = g.B32[3 * Kp + k];
#pragma unroll 2
        for (int q = 0; q < RV; ++q) {
          const float* ph = vt + q * 3 * N;
          float zq1 = 0.0f, zq2 = 0.0f;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            zq1 += ph[j] * z1[j];
            zq2 += ph[j] * z2[j];
          }
          const float dw = dvol[vidx(k, q, RV)];
          const float g1 = dw * (B22 * zq1 - B12 * zq2), g2 = dw * (B11 * zq2 - B21 * zq1);
#pragma unroll
          for (int i = 0; i < N; ++i) t[i] -= ph[N + i] * g1 + ph[2 * N + i] * g2;
        }
      }
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        const int kind = g.kind[n * Kp + k];
        if (kind == LDG_EDGE_NEUMANN) continue;
        const float L = g.elen32[n * Kp + k];
        float w[Q];
        if (kind == LDG_EDGE_INTERIOR) {
          const int64_t kp = g.nbr[n * Kp + k];
          const int np = g.nbrn[n * Kp + k];
#pragma unroll
          for (int q = 0; q < Q; ++q)
            w[q] = 0.5f * L * (sig[vidx(k, n * Q + q, NQ)] - sig[vidx(kp, np * Q + (Q - 1 - q), NQ)]);
        } else {
#pragma unroll
          for (int q = 0; q < Q; ++q) w[q] = L * sig[vidx(k, n * Q + q, NQ)];
        }
        // one point at a time: each step reads N table entries through the
        // scalar cache, and the barrier keeps the compiler from hoisting the
        // loads of all points at once (more SGPRs than a wave has)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
#pragma unroll
          for (int i = 0; i < N; ++i) t[i] += lift[(n * Q + q) * N + i] * w[q];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      float c[N];
      load_vec<N, float>(C, k, c);
      const float a2 = (float)(alpha * g.area2[k]);
      const float tt = (float)tau;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        t[i] = a2 * c[i] + tt * t[i];
        dot += (double)c[i] * (double)t[i];
      }
      store_vec<N, float>(y, k, t);
    }
  }
  if (partials == nullptr) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one triangle of the divergence half; returns <C_k, y_k> for the fused dot.
// BLOCKS = false leaves out the block terms (the matrix-free kernel adds them).
template <int N, class T, class BT, bool BLOCKS>
__device__ inline double div_row(const Geo& g, const T* __restrict__ sm,
                                 const BT* __restrict__ blocks, const T* __restrict__ C,
                                 const T* __restrict__ Z1, const T* __restrict__ Z2, double alpha,
                                 double tau, double eta, T* __restrict__ y, int64_t k) {
  T t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = 0;
  if (k >= g.K) {
    store_vec<N, T>(y, k, t);
    return 0.0;
  }
  const int64_t Kp = g.Kpad;
  T c[N], z[N];
  load_vec<N, T>(C, k, c);
  for (int n = 0; n < 3; ++n) {
    const int kind = g.kind[n * Kp + k];
    if (kind == LDG_EDGE_NEUMANN) continue;
    mv_add<N, T>(sm + ref_sd(n) * N * row_stride<N, T>(), c, t, (T)eta);   // (1/|E|) |E| S_hat_diag
    if (kind == LDG_EDGE_INTERIOR) {
      const int64_t kp = g.nbr[n * Kp + k];
      const int np = g.nbrn[n * Kp + k];
      T cp[N];
      load_vec<N, T>(C, kp, cp);
      mv_add<N, T>(sm + ref_so(n, np) * N * row_stride<N, T>(), cp, t, (T)(-eta));
    }
  }
  if constexpr (BLOCKS) {
    constexpr bool PACKED = sizeof(BT) == 2;   // BF16: packed layout with tail groups
    T tail[PACKED ? bp_tailn<N, BT>(NSLOT) : 1];
    if constexpr (PACKED) bp_tail_load<N, BT, T>(blocks, k, NSLOT, tail);
    load_vec<N, T>(Z1, k, z);
    if constexpr (PACKED) block_mv_bp<N, BT, T>(blocks, k, 0, NSLOT, tail, z, t);
    else block_mv<N, BT, T>(blocks, k, 0, NSLOT, z, t);
    load_vec<N, T>(Z2, k, z);
    if constexpr (PACKED) block_mv_bp<N, BT, T>(blocks, k, 1, NSLOT, tail, z, t);
    else block_mv<N, BT, T>(blocks, k, 1, NSLOT, z, t);
    for (int n = 0; n < 3; ++n) {
      const int64_t kp = g.nbr[n * Kp + k];
      if (kp < 0) continue;
      T nu1, nu2;
      if constexpr (sizeof(T) == 4) {   // the FP32 copies: the same values, half the bytes
        nu1 = g.nu32[(2 * n) * Kp + k];
        nu2 = g.nu32[(2 * n + 1) * Kp + k];
      } else {
        nu1 = (T)g.nu[(2 * n) * Kp + k];
        nu2 = (T)g.nu[(2 * n + 1) * Kp + k];
      }
#pragma unroll
      for (int j = 0; j < N; ++j) z[j] = nu1 * Z1[vidx(kp, j, N)] + nu2 * Z2[vidx(kp, j, N)];
      if constexpr (PACKED) block_mv_bp<N, BT, T>(blocks, k, 2 + n, NSLOT, tail, z, t);
      else block_mv<N, BT, T>(blocks, k, 2 + n, NSLOT, z, t);
    }
  }
  const T a2 = (T)(alpha * g.area2[k]);
  const T tt = (T)tau;
  double dot = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    t[i] = a2 * c[i] + tt * t[i];
    dot += (double)c[i] * (double)t[i];
  }
  store_vec<N, T>(y, k, t);
  return dot;
}

// y = alpha M C + tau (eta S' C + sum_m B^m Z^m); partials (optional): per-block
// sums of <C, y>, the CG curvature p^T A p fused into the apply
template <int N, class T, class BT, bool BLOCKS>
__global__ void __launch_bounds__(256) k_div(Geo g, const double* __restrict__ refs,
                                             const BT* __restrict__ blocks,
                                             const T* __restrict__ C, const T* __restrict__ Z1,
                                             const T* __restrict__ Z2, double alpha, double tau,
                                             double eta, T* __restrict__ y,
                                             double* __restrict__ partials) {
  constexpr bool LDSR = refs_in_lds<N, T>();
  static_assert(LDSR || sizeof(T) == 8, "FP32 reference matrices always fit in LDS");
  __shared__ __align__(16) T smem[LDSR ? ref_size<N, T>() : 1];
  __shared__ double red[4];
  const T* sm;
  if constexpr (LDSR) {
    load_refs<N, T>(smem, refs);
    sm = smem;
  } else {
    sm = reinterpret_cast<const T*>(refs);
  }
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (k < g.Kpad) s = div_row<N, T, BT, BLOCKS>(g, sm, blocks, C, Z1, Z2, alpha, tau, eta, y, k);
  if (partials == nullptr) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// z = P^{-1} r; with `partials`, also per-block sums of <r, z> in FP64
template <int N, class T, class BT>
__global__ void __launch_bounds__(256) k_bj_apply(Geo g, const BT* __restrict__ bj,
                                                  const T* __restrict__ r, T* __restrict__ z,
                                                  double* __restrict__ partials) {
  __shared__ double red[4];
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (k < g.Kpad) {
    T x[N], acc[N];
    load_vec<N, T>(r, k, x);
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0;
    block_mv<N, BT, T>(bj, k, 0, 1, x, acc);
    store_vec<N, T>(z, k, acc);
#pragma unroll
    for (int i = 0; i < N; ++i) s += (double)x[i] * (double)acc[i];
  }
  if (partials == nullptr) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// low-precision copies of stored blocks: dst (BT layout) <- src (double layout)
template <class BT>
__global__ void k_convert_blocks(int64_t Kpad, int N, int ns, const double* __restrict__ src,
                                 BT* __restrict__ dst) {
  const int NN = N * N;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int W = Blk<BT>::W;
  const int NG = ngroups(N, W);
  const int NGd = ngroups(N, 2);
  if (t >= Kpad * ns * NG * W) return;
  // t enumerates the destination in storage order
  const int h = (int)(t % W);
  const int64_t e = (t / W) % TILE;
  const int64_t rest = t / (W * TILE);
  const int gg = (int)(rest % NG);
  const int64_t rest2 = rest / NG;
  const int s = (int)(rest2 % ns);
  const int64_t tile = rest2 / ns;
  const int64_t k = tile * TILE + e;
  const int f = gg * W + h;
  const double v = f < NN ? src[bgidx(k, s, f / 2, ns, NGd, 2) + (f & 1)] : 0.0;
  dst[t] = from_double<BT>(v);
}

template <class BT>
__global__ void k_export_any(int64_t K, int N, int ns, const BT* __restrict__ src,
                             double* __restrict__ dst) {
  const int NN = N * N;
  const int W = Blk<BT>::W;
  const int NG = ngroups(N, W);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * ns * NN) return;
  const int64_t k = t / (ns * NN);
  const int rem = (int)(t % (ns * NN));
  const int s = rem / NN, f = rem % NN;
  BT v = sizeof(BT) == 2 ? src[bp_idx(k, s, f, N, ns, 8)] : src[bgidx(k, s, f / W, ns, NG, W) + f % W];
  if constexpr (sizeof(BT) == 2) {
    dst[t] = (double)__uint_as_float((uint32_t)v << 16);
  } else if constexpr (sizeof(BT) == 1) {
    dst[t] = (double)fp8_to_float(v);
  } else {
    dst[t] = (double)v;
  }
}

// rows of stored blocks for the listed triangles, FP64 [n][ns][N][N]
__global__ void k_export_rows(int64_t n, const int32_t* __restrict__ elems, int N, int ns,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int NN = N * N;
  const int NG = ngroups(N, 2);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ns * NN) return;
  const int64_t i = t / (ns * NN);
  const int rem = (int)(t % (ns * NN));
  const int s = rem / NN, f = rem % NN;
  dst[t] = src[bgidx(elems[i], s, f / 2, ns, NG, 2) + (f & 1)];
}

// d_h at the points of the quadrature form, once per step from the FP64 tiled
// coefficients D (FP64 sums, stored FP32; zero on padding triangles):
//   dE[k][n][q]  = sum_l D_kl phi_l(point q of reference edge n),
//   dvol[k][q]   = w_q sum_l D_kl phi_l(x_q)  (the exact volume rule)
template <int N>
__global__ void __launch_bounds__(256) k_edge_d(Geo g, const double* __restrict__ D,
                                                const double* __restrict__ trace64,
                                                const double* __restrict__ vol64,
                                                float* __restrict__ dE, float* __restrict__ dvol) {
  constexpr int Q = edge_trace_points(N), NQ = 3 * Q, RV = vol_points(N);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  double d[N];
#pragma unroll
  for (int l = 0; l < N; ++l) d[l] = k < g.K ? D[vidx(k, l, N)] : 0.0;
  for (int r = 0; r < NQ; ++r) {
    double v = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) v += trace64[r * N + l] * d[l];
    dE[vidx(k, r, NQ)] = (float)v;
  }
  for (int r = 0; r < RV; ++r) {
    double v = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) v += vol64[r * N + l] * d[l];
    dvol[vidx(k, r, RV)] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}

void launch_grad(int N, int vt, const Geo& g, const double* refs, const float* refs32,
                 const void* C, const void* J1, const void* J2, void* Z1, void* Z2,
                 hipStream_t st, const EdgeTraces* tr) {
  const unsigned nb = nblk(g.Kpad, 256);
  if (vt == VT_F64) {
    LDG_SWITCH_N_P6(N, (k_grad<NT, double, false><<<nb, 256, 0, st>>>(
                        g, refs, refs, (const double*)C, (const double*)J1, (const double*)J2,
                        (double*)Z1, (double*)Z2, nullptr, nullptr, nullptr, nullptr, 0.0f)));
  } else if (tr) {
    LDG_SWITCH_N_P6(N, (k_grad<NT, float, true><<<nb, 256, 0, st>>>(
                        g, refs, refs32, (const float*)C, (const float*)J1, (const float*)J2,
                        (float*)Z1, (float*)Z2, tr->dE, tr->trace, tr->sig, tr->pen, tr->eta)));
  } else {
    LDG_SWITCH_N_P6(N, (k_grad<NT, float, false><<<nb, 256, 0, st>>>(
                        g, refs, refs32, (const float*)C, (const float*)J1, (const float*)J2,
                        (float*)Z1, (float*)Z2, nullptr, nullptr, nullptr, nullptr, 0.0f)));
  }
}

void launch_div(int N, int vt, int bt, const Geo& g, const double* refs, const void* blocks,
                const void* C, const void* Z1, const void* Z2, double alpha, double tau,
                double eta, void* y, hipStream_t st, const Reducer* red, const EdgeTraces* tr) {
  const unsigned nb = nblk(g.Kpad, 256);
  double* parts = red ? red->partials : nullptr;
  if (tr) {   // FP32 quadrature form: no stored blocks, penalty from the gradient half
    LDG_SWITCH_N_P6(N, (k_div_q<NT><<<nb, 256, 0, st>>>(
                        g, (const float*)C, (const float*)Z1, (const float*)Z2, tr->pen, alpha, tau,
                        (float*)y, parts, tr->sig, tr->dvol, tr->vtab, tr->lift)));
  } else if (blocks == nullptr) {   // matrix-free: the terms without blocks
    if (vt == VT_F64) {
      LDG_SWITCH_N_P6(N, (k_div<NT, double, double, false><<<nb, 256, 0, st>>>(
                          g, refs, nullptr, (const double*)C, (const double*)Z1,
                          (const double*)Z2, alpha, tau, eta, (double*)y, parts)));
    } else {
      LDG_SWITCH_N_P6(N, (k_div<NT, float, float, false><<<nb, 256, 0, st>>>(
                          g, refs, nullptr, (const float*)C, (const float*)Z1, (const float*)Z2,
                          alpha, tau, eta, (float*)y, parts)));
    }
  } else if (vt == VT_F64) {
    LDG_SWITCH_N_P6(N, (k_div<NT, double, double, true><<<nb, 256, 0, st>>>(
                        g, refs, (const double*)blocks, (const double*)C, (const double*)Z1,
                        (const double*)Z2, alpha, tau, eta, (double*)y, parts)));
  } else if (bt == BT_F32) {
    LDG_SWITCH_N_P6(N, (k_div<NT, float, float, true><<<nb, 256, 0, st>>>(
                        g, refs, (const float*)blocks, (const float*)C, (const float*)Z1,
                        (const float*)Z2, alpha, tau, eta, (float*)y, parts)));
  } else {
    LDG_SWITCH_N_P6(N, (k_div<NT, float, bf16, true><<<nb, 256, 0, st>>>(
                        g, refs, (const bf16*)blocks, (const float*)C, (const float*)Z1,
                        (const float*)Z2, alpha, tau, eta, (float*)y, parts)));
  }
  if (red) reduce_partials((int)nb, red->partials, red->result, st, red->cg, red->cg_mode);
}

void launch_edge_d(int N, const Geo& g, const double* D, const EdgeTraces& tr, hipStream_t st) {
  LDG_SWITCH_N_P6(N, (k_edge_d<NT><<<nblk(g.Kpad, 256), 256, 0, st>>>(
                         g, D, tr.trace64, tr.vol64, tr.dE, tr.dvol)));
}

void launch_bj_apply(int N, int vt, int bt, const Geo& g, const void* bj, const void* r, void* z,
                     const Reducer* red, hipStream_t st) {
  const unsigned nb = nblk(g.Kpad, 256);
  double* parts = red ? red->partials : nullptr;
  if (vt == VT_F64) {
    LDG_SWITCH_N_P6(N, (k_bj_apply<NT, double, double><<<nb, 256, 0, st>>>(
                        g, (const double*)bj, (const double*)r, (double*)z, parts)));
  } else if (bt == BT_F32) {
    LDG_SWITCH_N_P6(N, (k_bj_apply<NT, float, float><<<nb, 256, 0, st>>>(
                        g, (const float*)bj, (const float*)r, (float*)z, parts)));
  } else {
    LDG_SWITCH_N_P6(N, (k_bj_apply<NT, float, bf16><<<nb, 256, 0, st>>>(
                        g, (const bf16*)bj, (const float*)r, (float*)z, parts)));
  }
  if (red) reduce_partials((int)nb, red->partials, red->result, st, red->cg, red->cg_mode);
}

void launch_convert_blocks(int bt, int64_t Kpad, int N, int ns, const double* src, void* dst,
                           hipStream_t st) {
  if (bt == BT_F32) {
    const int64_t n = Kpad * ns * ngroups(N, 4) * 4;
    k_convert_blocks<float><<<nblk(n, 256), 256, 0, st>>>(Kpad, N, ns, src, (float*)dst);
  }
}

void launch_export_blocks_any(int bt, int64_t K, int N, int ns, const void* src, double* dst,
                              hipStream_t st) {
  const unsigned nb = nblk(K * ns * N * N, 256);
  if (bt == BT_F64) k_export_any<double><<<nb, 256, 0, st>>>(K, N, ns, (const double*)src, dst);
  else if (bt == BT_F32) k_export_any<float><<<nb, 256, 0, st>>>(K, N, ns, (const float*)src, dst);
  else if (bt == BT_BF16) k_export_any<bf16><<<nb, 256, 0, st>>>(K, N, ns, (const bf16*)src, dst);
  else k_export_any<fp8><<<nb, 256, 0, st>>>(K, N, ns, (const fp8*)src, dst);
}

void launch_export_rows(int64_t n, const int32_t* elems, int N, int ns, const double* src,
                        double* dst, hipStream_t st) {
  if (n == 0) return;
  k_export_rows<<<nblk(n * ns * N * N, 256), 256, 0, st>>>(n, elems, N, ns, src, dst);
}

size_t block_bytes(int bt, int64_t Kpad, int N, int ns) {
  if (bt == BT_BF16) return (size_t)(Kpad / TILE) * bp_groups(N, ns, 8) * TILE * 8 * 2;
  const int W = bt == BT_F64 ? 2 : (bt == BT_F32 ? 4 : 8);
  const size_t es = bt == BT_F64 ? 8 : (bt == BT_F32 ? 4 : 2);
  return (size_t)Kpad * ns * ngroups(N, W) * W * es;
}

}  // namespace ldg
