// Learned factored preconditioner on the element graph (linear, SPD):
//
//   P = W^T (I + F)^T (I + F) W,   W = blockdiag(W_k),  W_k^T W_k = BJ_k^{-1},
//   F_kj = -omega_kn O_kn  for j = k+ across local edge n,
//   O_kn = W_k S_kj W_j^T  (the neighbour blocks of the scaled operator W S W^T).
//
// W_k = R_k^T with R_k the lower Cholesky factor of the block-Jacobi inverse;
// omega comes from the graph network (kernels_gnn.hip).  Setup once per
// system: Cholesky factors (16 lanes per triangle), then the explicit
// neighbour blocks of the eliminated operator, once per interior edge, with
// O written to both sides (O_{k+ n+} = O_kn^T exactly after rounding).
//
//   S_kj = tau [ -eta S_off(n, n+)
//                - (|E_kn| / (2 * 2|T_k|)) (sum_m nu^m_kn B^m_kk) S_off(n, n+)
//                - (1 / 2|T_j|) U_kn (sum_m nu^m_kn A^m_jj) ],
//   A^m_jj = -H^m_j + sum_n' q_n' nu^m_jn' |E_jn'| S_diag(n'),  q = 1/2 interior, 1 Neumann,
//
// the blocks of M + tau (eta (S + S_D) - sum_m B^m M^{-1} A^m) between two
// triangles sharing an edge (paths through a third triangle next to both
// exist only around interior vertices of degree three and are left out).
// Application: three one-lane-per-triangle passes, y = W x, a = (I + F) y,
// z = W^T (I + F)^T a, the transpose using the stored O_kn as O_{k+ n+}^T.
#include "device_common.h"
#include "kernels.h"

namespace ldg {

namespace {

constexpr int NREF = 14;  // H1, H2, Sd[3], So[3][3]
__device__ inline int ref_so(int a, int b) { return 5 + 3 * a + b; }
inline unsigned nbk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// the O blocks use the packed layout (whole groups per slot, shared tail groups)
template <class BT>
__device__ inline void put(BT* __restrict__ fb, int64_t k, int s, int ns, int f, int N, double v) {
  fb[bp_idx(k, s, f, N, ns, Blk<BT>::W)] = from_double<BT>(v);
}

template <class BT>
__device__ inline double get_any(const BT* __restrict__ fb, int64_t k, int s, int ns, int f, int N) {
  const BT v = fb[bp_idx(k, s, f, N, ns, Blk<BT>::W)];
  if constexpr (sizeof(BT) == 2) return (double)__uint_as_float((uint32_t)v << 16);
  else if constexpr (sizeof(BT) == 1) return (double)fp8_to_float(v);
  else return (double)v;
}

__device__ inline double get64(const double* __restrict__ b, int64_t k, int s, int ns, int f,
                               int NP) {
  return b[pidx(k, s, f >> 1, ns, NP) + (f & 1)];
}

// W_k is upper triangular: only its N(N+1)/2 entries W[r][i], i >= r, are
// stored, packed row by row (entry e = rN - r(r-1)/2 + i - r) in groups of the
// storage width in the element-fastest tile layout of one block slot.
template <int N>
__host__ __device__ constexpr int tri_size() { return N * (N + 1) / 2; }
template <int N>
__host__ __device__ constexpr int tri_index(int r, int i) { return r * N - r * (r - 1) / 2 + i - r; }

template <int N, class BW>
__device__ inline void putw(BW* __restrict__ fw, int64_t k, int r, int i, double v) {
  constexpr int Wv = Blk<BW>::W;
  constexpr int NG = (tri_size<N>() + Wv - 1) / Wv;
  const int e = tri_index<N>(r, i);
  fw[bgidx(k, 0, e / Wv, 1, NG, Wv) + e % Wv] = from_double<BW>(v);
}

// W[r][i] as stored (zero below the diagonal), for exports; N at run time
template <class BW>
__device__ inline double getw(const BW* __restrict__ fw, int64_t k, int N, int r, int i) {
  if (i < r) return 0.0;
  constexpr int Wv = Blk<BW>::W;
  const int NG = (N * (N + 1) / 2 + Wv - 1) / Wv;
  const int e = r * N - r * (r - 1) / 2 + i - r;
  const BW v = fw[bgidx(k, 0, e / Wv, 1, NG, Wv) + e % Wv];
  if constexpr (sizeof(BW) == 2) return (double)__uint_as_float((uint32_t)v << 16);
  else if constexpr (sizeof(BW) == 1) return (double)fp8_to_float(v);
  else return (double)v;
}

// acc += W_k z  (TRANS false) or acc += W_k^T z  (TRANS true) from the packed
// triangle, walking it in storage order: a group is loaded where e starts one
// (all indices are constants once the loops are unrolled)
template <int N, class BW, class T, bool TRANS>
__device__ inline void tri_mv(const BW* __restrict__ fw, int64_t k, const T* z, T* acc) {
  constexpr int Wv = Blk<BW>::W;
  constexpr int NG = (tri_size<N>() + Wv - 1) / Wv;
  T v[Wv];
#pragma unroll
  for (int r = 0; r < N; ++r) {
#pragma unroll
    for (int i = r; i < N; ++i) {
      const int e = tri_index<N>(r, i);
      if (e % Wv == 0) Blk<BW>::load(fw + bgidx(k, 0, e / Wv, 1, NG, Wv), v);
      if (TRANS) acc[i] += v[e % Wv] * z[r];
      else acc[r] += v[e % Wv] * z[i];
    }
  }
}

// W stored in FP8 carries a power-of-two scale per triangle (W = s W8); the
// other storages carry none
template <class BW>
__device__ inline float wscale(const float* __restrict__ ws, int64_t k) {
  if constexpr (sizeof(BW) == 1) return ws[k];
  else return 1.f;
}

}  // namespace

// W_k = R_k^T, BJ_k^{-1} = R_k R_k^T (lower Cholesky), 16 lanes per triangle,
// lane i owns row i; padding triangles get the identity.  sym: factor the
// symmetric part (BJ_k^{-1} + BJ_k^{-T}) / 2 instead (nonsymmetric steps; it is
// positive definite where the symmetric part of the diagonal block is).
template <int N, class BT>
__global__ void __launch_bounds__(256) k_fac_chol(Geo g, const double* __restrict__ bj,
                                                  double* __restrict__ w64, BT* __restrict__ fb,
                                                  float* __restrict__ ws,
                                                  int* __restrict__ status, bool sym) {
  constexpr int NP = npairs(N);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid >> 4;
  const int i = (int)(gid & 15);
  const bool elem_ok = k < g.K;
  const bool row_ok = elem_ok && i < N;
  double a[N];
#pragma unroll
  for (int c = 0; c < N; ++c)
    a[c] = row_ok ? (sym ? 0.5 * (get64(bj, k, 0, 1, i * N + c, NP) + get64(bj, k, 0, 1, c * N + i, NP))
                         : get64(bj, k, 0, 1, i * N + c, NP))
                  : (c == i ? 1.0 : 0.0);
  // right-looking, branch-free: after column c, lane i holds L[i][c] in a[c] and
  // the updated a[i][j] for j > c (entries with j > i are don't-cares)
  bool bad = false;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const double piv = __shfl(a[c], c, 16);
    bad |= !(piv > 0.0);
    const double inv = 1.0 / sqrt(piv);
    const double lic = (i >= c ? 1.0 : 0.0) * a[c] * inv;
    a[c] = lic;
#pragma unroll
    for (int j = c + 1; j < N; ++j) a[j] -= lic * __shfl(lic, j, 16);
  }
  if (row_ok && bad) atomicOr(status, 2);
  // FP8 storage: scale 2^round(log2(max |W_k| / 256)) puts the block's largest
  // entry in [181, 362], inside the E4M3 range (448)
  double inv_s = 1.0;
  if constexpr (sizeof(BT) == 1) {
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) m = fmax(m, (r <= i && i < N) ? fabs(a[r]) : 0.0);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 16));
    const double sc = m > 0.0 ? exp2(rint(log2(m / 256.0))) : 1.0;
    inv_s = 1.0 / sc;
    if (i == 0 && k < g.Kpad) ws[k] = (float)sc;
  }
  if (k < g.Kpad && i < N) {
#pragma unroll
    for (int r = 0; r < N; ++r) {   // lane i holds R[i][r] = W[r][i]
      const double v = r <= i ? a[r] : 0.0;
      const int f = r * N + i;
      w64[pidx(k, 0, f >> 1, 1, NP) + (f & 1)] = v;
      if (r <= i) putw<N, BT>(fb, k, r, i, v * inv_s);
    }
  }
}

// O_kn for every interior edge once (from the triangle with the smaller index),
// written to (k, n) and transposed to (k+, n+); lognorm = log ||O_kn||_F on both.
// 64 threads = 4 triangles x 16 lanes; lane i owns row i.  SYM (nonsymmetric
// steps): S_kj is replaced by the block of the symmetric part of the operator,
// (S_kj + S_jk^T) / 2, with S_jk from the same formula seen from triangle j
// (its edge n+, its blocks B^m_jj and U_jn+, the A^m_kk of triangle k).
template <int N, class BT, bool SYM>
__global__ void __launch_bounds__(64) k_fac_offdiag(Geo g, const double* __restrict__ refs,
                                                    const double* __restrict__ blocks,
                                                    const double* __restrict__ w64, double tau,
                                                    double eta, BT* __restrict__ fo,
                                                    float* __restrict__ lognorm) {
  // every intermediate N x N matrix lives in LDS (one set per triangle of the
  // block); registers hold scalars only
  constexpr int NN = N * N;
  constexpr int NP = npairs(N);
  __shared__ double sm[NREF * NN];
  __shared__ double t1[4][NN];
  __shared__ double t2[4][NN];
  __shared__ double t3[4][NN];
  // S_jk only for the symmetric part: the plain instance keeps 7 KB less LDS
  // (three workgroups per CU instead of two)
  __shared__ double t4[SYM ? 4 : 1][SYM ? NN : 1];
  for (int t = threadIdx.x; t < NREF * NN; t += blockDim.x) sm[t] = refs[t];
  __syncthreads();
  const int grp = threadIdx.x >> 4;
  const int i = threadIdx.x & 15;
  const bool row = i < N;
  const int ii = row ? i : 0;
  const int64_t k = (int64_t)blockIdx.x * 4 + grp;
  const bool elem_ok = k < g.K;
  const int64_t kk = elem_ok ? k : 0;
  const int64_t Kp = g.Kpad;
  const double area2k = g.area2[kk];
  double* T1 = t1[grp];
  double* T2 = t2[grp];
  double* T3 = t3[grp];
  double* T4 = SYM ? t4[grp] : nullptr;
#pragma unroll 1
  for (int n = 0; n < 3; ++n) {
    const int64_t jn = elem_ok ? g.nbr[n * Kp + kk] : -1;
    const bool act = jn > k;
    const int64_t j = act ? jn : kk;
    const int npl = act ? g.nbrn[n * Kp + kk] : 0;
    // each interior edge once, by the triangle with the lower index: the other
    // side and boundary edges skip the arithmetic (every lane still reaches the
    // barriers and the shuffles)
    const bool work = row && act;
    const double nu1 = g.nu[(2 * n) * Kp + kk], nu2 = g.nu[(2 * n + 1) * Kp + kk];
    // T1 <- sum_m nu^m_kn A^m_jj;  T2 <- sum_m nu^m_kn B^m_kk (row ii per lane)
    {
      const double B11 = g.B[j], B12 = g.B[Kp + j], B21 = g.B[2 * Kp + j], B22 = g.B[3 * Kp + j];
      const double c0 = -(nu1 * B22 - nu2 * B12);
      const double c1 = -(-nu1 * B21 + nu2 * B11);
      double cq[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int kd = g.kind[q * Kp + j];
        const double w = kd == LDG_EDGE_INTERIOR ? 0.5 : (kd == LDG_EDGE_NEUMANN ? 1.0 : 0.0);
        cq[q] = w * (nu1 * g.nu[(2 * q) * Kp + j] + nu2 * g.nu[(2 * q + 1) * Kp + j]) *
                g.elen[q * Kp + j];
      }
      if (work) {
#pragma unroll 1
        for (int c = 0; c < N; ++c) {
          const int e = ii * N + c;
          T1[e] = c0 * sm[e] + c1 * sm[NN + e] + cq[0] * sm[2 * NN + e] +
                  cq[1] * sm[3 * NN + e] + cq[2] * sm[4 * NN + e];
          T2[e] = nu1 * get64(blocks, kk, 0, NSLOT, e, NP) + nu2 * get64(blocks, kk, 1, NSLOT, e, NP);
        }
      }
    }
    __syncthreads();
    // T3 <- S_kj (row ii per lane)
    if (work) {
      const double* So = sm + ref_so(n, npl) * NN;
      const double s1 = 0.5 * g.elen[n * Kp + kk] / area2k;
      const double s2 = 1.0 / g.area2[j];
#pragma unroll 1
      for (int c = 0; c < N; ++c) {
        double acc = -eta * So[ii * N + c];
#pragma unroll
        for (int l = 0; l < N; ++l)
          acc -= s1 * T2[ii * N + l] * So[l * N + c] +
                 s2 * get64(blocks, kk, 2 + n, NSLOT, ii * N + l, NP) * T1[l * N + c];
        T3[ii * N + c] = tau * acc;
      }
    }
    __syncthreads();
    if constexpr (SYM) {
      // S_jk: nu_{j n+} = -nu_kn, |E| shared; T1 <- sum_m nu^m_{j n+} A^m_kk,
      // T2 <- sum_m nu^m_{j n+} B^m_jj, T4 <- S_jk, then T3 <- (T3 + T4^T) / 2
      {
        const double B11 = g.B[kk], B12 = g.B[Kp + kk], B21 = g.B[2 * Kp + kk], B22 = g.B[3 * Kp + kk];
        const double c0 = (nu1 * B22 - nu2 * B12);
        const double c1 = (-nu1 * B21 + nu2 * B11);
        double cq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int kd = g.kind[q * Kp + kk];
          const double w = kd == LDG_EDGE_INTERIOR ? 0.5 : (kd == LDG_EDGE_NEUMANN ? 1.0 : 0.0);
          cq[q] = -w * (nu1 * g.nu[(2 * q) * Kp + kk] + nu2 * g.nu[(2 * q + 1) * Kp + kk]) *
                  g.elen[q * Kp + kk];
        }
        if (work) {
#pragma unroll 1
          for (int c = 0; c < N; ++c) {
            const int e = ii * N + c;
            T1[e] = c0 * sm[e] + c1 * sm[NN + e] + cq[0] * sm[2 * NN + e] +
                    cq[1] * sm[3 * NN + e] + cq[2] * sm[4 * NN + e];
            T2[e] = -nu1 * get64(blocks, j, 0, NSLOT, e, NP) - nu2 * get64(blocks, j, 1, NSLOT, e, NP);
          }
        }
      }
      __syncthreads();
      if (work) {
        const double* So = sm + ref_so(npl, n) * NN;
        const double s1 = 0.5 * g.elen[n * Kp + kk] / g.area2[j];
        const double s2 = 1.0 / area2k;
#pragma unroll 1
        for (int c = 0; c < N; ++c) {
          double acc = -eta * So[ii * N + c];
#pragma unroll
          for (int l = 0; l < N; ++l)
            acc -= s1 * T2[ii * N + l] * So[l * N + c] +
                   s2 * get64(blocks, j, 2 + npl, NSLOT, ii * N + l, NP) * T1[l * N + c];
          T4[ii * N + c] = tau * acc;
        }
      }
      __syncthreads();
      if (work) {
#pragma unroll 1
        for (int c = 0; c < N; ++c) T3[ii * N + c] = 0.5 * (T3[ii * N + c] + T4[c * N + ii]);
      }
      __syncthreads();
    }
    // T2 <- W_j;  T1 <- T = S_kj W_j^T
    if (work) {
#pragma unroll 1
      for (int c = 0; c < N; ++c) T2[ii * N + c] = get64(w64, j, 0, 1, ii * N + c, NP);
    }
    __syncthreads();
    if (work) {
#pragma unroll 1
      for (int c = 0; c < N; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) acc += T3[ii * N + l] * T2[c * N + l];
        T1[ii * N + c] = acc;
      }
    }
    __syncthreads();
    // O = W_k T, row ii, straight to both sides; ||O||_F over the 16 lanes
    double nrm = 0.0;
    if (work) {
#pragma unroll 1
      for (int c = 0; c < N; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) acc += get64(w64, kk, 0, 1, ii * N + l, NP) * T1[l * N + c];
        nrm += acc * acc;
        if (act) {
          put<BT>(fo, k, n, 3, ii * N + c, N, acc);
          put<BT>(fo, j, npl, 3, c * N + ii, N, acc);
        }
      }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 16);
    if (act && i == 0) {
      const float ln = (float)log(fmax(sqrt(nrm), 1e-300));
      lognorm[n * Kp + k] = ln;
      lognorm[npl * Kp + j] = ln;
    }
    __syncthreads();
  }
}

// y = W x
template <int N, class T, class BW>
__global__ void __launch_bounds__(256) k_fac_w(int64_t Kpad, const BW* __restrict__ fw,
                                               const float* __restrict__ ws,
                                               const T* __restrict__ x, T* __restrict__ y) {
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= Kpad) return;
  T xv[N], acc[N];
  load_vec<N, T>(x, k, xv);
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0;
  tri_mv<N, BW, T, false>(fw, k, xv, acc);
  if constexpr (sizeof(BW) == 1) {
    const T sc = (T)wscale<BW>(ws, k);
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] *= sc;
  }
  store_vec<N, T>(y, k, acc);
}

// y = W^T x
template <int N, class T, class BW>
__global__ void __launch_bounds__(256) k_fac_wt(int64_t Kpad, const BW* __restrict__ fw,
                                                const float* __restrict__ ws,
                                                const T* __restrict__ x, T* __restrict__ y) {
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= Kpad) return;
  T xv[N], acc[N];
  load_vec<N, T>(x, k, xv);
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0;
  tri_mv<N, BW, T, true>(fw, k, xv, acc);
  if constexpr (sizeof(BW) == 1) {
    const T sc = (T)wscale<BW>(ws, k);
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] *= sc;
  }
  store_vec<N, T>(y, k, acc);
}

// out = (I + F) x  (NBR false: omega_kn), or (I + F)^T x  (NBR true: omega_{k+ n+},
// O_kn standing for O_{k+ n+}^T), followed by out = W^T out when WT.
// partials (optional): per-block sums of <r, out> for the preconditioned dot.
template <int N, class T, class BW, class BO, bool NBR, bool WT>
__global__ void __launch_bounds__(256) k_fac_f(Geo g, const BW* __restrict__ fw,
                                               const float* __restrict__ ws,
                                               const BO* __restrict__ fo,
                                               const float* __restrict__ om,
                                               const T* __restrict__ x, T* __restrict__ out,
                                               const T* __restrict__ r,
                                               double* __restrict__ partials) {
  __shared__ double red[4];
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t Kp = g.Kpad;
  double s = 0.0;
  if (k < Kp) {
    T acc[N];
    load_vec<N, T>(x, k, acc);
    if (k < g.K) {
      T tail[bp_tailn<N, BO>(3)];
      bp_tail_load<N, BO, T>(fo, k, 3, tail);
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        const int64_t j = g.nbr[n * Kp + k];
        if (j < 0) continue;
        const float w = NBR ? om[(int64_t)g.nbrn[n * Kp + k] * Kp + j] : om[n * Kp + k];
        T xj[N];
        load_vec<N, T>(x, j, xj);
#pragma unroll
        for (int i = 0; i < N; ++i) xj[i] *= -(T)w;
        block_mv_bp<N, BO, T>(fo, k, n, 3, tail, xj, acc);
      }
    }
    if (WT) {
      T o[N];
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] = 0;
      tri_mv<N, BW, T, true>(fw, k, acc, o);
      if constexpr (sizeof(BW) == 1) {
        const T sc = (T)wscale<BW>(ws, k);
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] *= sc;
      }
      store_vec<N, T>(out, k, o);
      if (partials) {
        T rv[N];
        load_vec<N, T>(r, k, rv);
#pragma unroll
        for (int i = 0; i < N; ++i) s += (double)rv[i] * (double)o[i];
      }
    } else {
      store_vec<N, T>(out, k, acc);
    }
  }
  if (partials == nullptr) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// d loss / d omega_kn = -(a_k^T O_kn beta_{k+} + alpha_k^T O_kn y_{k+}); 0 off the interior
template <int N, class BO>
__global__ void __launch_bounds__(256) k_fac_domega(Geo g, const BO* __restrict__ fo,
                                                    const double* __restrict__ a,
                                                    const double* __restrict__ beta,
                                                    const double* __restrict__ alpha,
                                                    const double* __restrict__ y,
                                                    float* __restrict__ dom) {
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t Kp = g.Kpad;
  if (k >= Kp) return;
  double ak[N], alk[N];
  load_vec<N, double>(a, k, ak);
  load_vec<N, double>(alpha, k, alk);
#pragma unroll 1   // one edge at a time keeps the gathers' registers short-lived
  for (int n = 0; n < 3; ++n) {
    const int64_t j = k < g.K ? g.nbr[n * Kp + k] : -1;
    double s = 0.0;
    if (j >= 0) {
      // a_k^T (O beta_j), then alpha_k^T (O y_j), through one gather buffer
      double v[N], u[N];
      load_vec<N, double>(beta, j, v);
#pragma unroll
      for (int i = 0; i < N; ++i) u[i] = 0.0;
      {
        double tl[bp_tailn<N, BO>(3)];
        bp_tail_load<N, BO, double>(fo, k, 3, tl);
        block_mv_bp<N, BO, double>(fo, k, n, 3, tl, v, u);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) s += ak[i] * u[i];
      load_vec<N, double>(y, j, v);
#pragma unroll
      for (int i = 0; i < N; ++i) u[i] = 0.0;
      {
        double tl[bp_tailn<N, BO>(3)];
        bp_tail_load<N, BO, double>(fo, k, 3, tl);
        block_mv_bp<N, BO, double>(fo, k, n, 3, tl, v, u);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) s += alk[i] * u[i];
    }
    dom[n * Kp + k] = (float)(-s);
  }
}

// rows of the factor blocks for the triangles elems[0..n): out[r][s][i][j] (FP64,
// s = 0 W, 1..3 O), lognorm[r][n] (may be NULL)
template <class BW, class BO>
__global__ void k_fac_export_rows(int64_t n, const int32_t* __restrict__ elems, int N,
                                  int64_t Kpad, const BW* __restrict__ fw,
                                  const float* __restrict__ ws,
                                  const BO* __restrict__ fo, const float* __restrict__ ln,
                                  double* __restrict__ out, float* __restrict__ lnout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int NN = N * N;
  if (t >= n * FAC_SLOTS * NN) return;
  const int f = (int)(t % NN);
  const int s = (int)((t / NN) % FAC_SLOTS);
  const int64_t r = t / ((int64_t)NN * FAC_SLOTS);
  const int64_t k = elems ? (int64_t)elems[r] : r;
  out[t] = s == 0 ? getw<BW>(fw, k, N, f / N, f % N) * (double)wscale<BW>(ws, k)
                  : get_any<BO>(fo, k, s - 1, 3, f, N);
  if (lnout && f == 0 && s < 3) lnout[r * 3 + s] = ln[s * Kpad + k];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// W storage BW and O storage BO: (F32, F32), (BF16, BF16), (BF16, FP8), (FP8, FP8)
#define LDG_SWITCH_FAC(FS, CALL)                                \
  if ((FS).wt == BT_FP8) {                                      \
    using BW = fp8;                                             \
    using BO = fp8;                                             \
    CALL;                                                       \
  } else if ((FS).ot == BT_FP8) {                               \
    using BW = bf16;                                            \
    using BO = fp8;                                             \
    CALL;                                                       \
  } else if ((FS).ot == BT_BF16) {                              \
    using BW = bf16;                                            \
    using BO = bf16;                                            \
    CALL;                                                       \
  } else {                                                      \
    using BW = float;                                           \
    using BO = float;                                           \
    CALL;                                                       \
  }

void launch_fac_setup(int N, const FacStore& fs, const Geo& g, const double* refs,
                      const double* blocks, const double* bj, double tau, double eta, double* w64,
                      float* lognorm, int* status, bool sym, hipStream_t st) {
  LDG_SWITCH_FAC(fs, {
    LDG_SWITCH_N(N, (k_fac_chol<NT, BW><<<nbk(g.Kpad * 16, 256), 256, 0, st>>>(
                        g, bj, w64, (BW*)fs.w, fs.ws, status, sym)));
    if (sym) {
      LDG_SWITCH_N(N, (k_fac_offdiag<NT, BO, true><<<nbk(g.Kpad, 4), 64, 0, st>>>(
                          g, refs, blocks, w64, tau, eta, (BO*)fs.o, lognorm)));
    } else {
      LDG_SWITCH_N(N, (k_fac_offdiag<NT, BO, false><<<nbk(g.Kpad, 4), 64, 0, st>>>(
                          g, refs, blocks, w64, tau, eta, (BO*)fs.o, lognorm)));
    }
  })
}

void launch_fac_apply(int N, const FacStore& fs, int vt, const Geo& g, const float* om,
                      const void* r, void* y, void* a, void* z, const Reducer* red,
                      hipStream_t st) {
  const unsigned nb = nbk(g.Kpad, 256);
  double* parts = red ? red->partials : nullptr;
  LDG_SWITCH_FAC(fs, {
    const BW* fw = (const BW*)fs.w;
    const BO* fo = (const BO*)fs.o;
    if (vt == VT_F64) {
      using T = double;
      LDG_SWITCH_N(N, (k_fac_w<NT, T, BW><<<nb, 256, 0, st>>>(g.Kpad, fw, fs.ws, (const T*)r, (T*)y)));
      LDG_SWITCH_N(N, (k_fac_f<NT, T, BW, BO, false, false><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, (const T*)y, (T*)a, nullptr, nullptr)));
      LDG_SWITCH_N(N, (k_fac_f<NT, T, BW, BO, true, true><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, (const T*)a, (T*)z, (const T*)r, parts)));
    } else {
      using T = float;
      LDG_SWITCH_N(N, (k_fac_w<NT, T, BW><<<nb, 256, 0, st>>>(g.Kpad, fw, fs.ws, (const T*)r, (T*)y)));
      LDG_SWITCH_N(N, (k_fac_f<NT, T, BW, BO, false, false><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, (const T*)y, (T*)a, nullptr, nullptr)));
      LDG_SWITCH_N(N, (k_fac_f<NT, T, BW, BO, true, true><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, (const T*)a, (T*)z, (const T*)r, parts)));
    }
  })
  if (red) reduce_partials((int)nb, red->partials, red->result, st, red->cg, red->cg_mode);
}

void launch_fac_w(int N, const FacStore& fs, const Geo& g, const double* x, double* y,
                  hipStream_t st) {
  LDG_SWITCH_FAC(fs, LDG_SWITCH_N(N, (k_fac_w<NT, double, BW><<<nbk(g.Kpad, 256), 256, 0, st>>>(
                                         g.Kpad, (const BW*)fs.w, fs.ws, x, y))))
}

void launch_fac_wt(int N, const FacStore& fs, const Geo& g, const double* x, double* y,
                   hipStream_t st) {
  LDG_SWITCH_FAC(fs, LDG_SWITCH_N(N, (k_fac_wt<NT, double, BW><<<nbk(g.Kpad, 256), 256, 0, st>>>(
                                         g.Kpad, (const BW*)fs.w, fs.ws, x, y))))
}

void launch_fac_f(int N, const FacStore& fs, const Geo& g, const float* om, bool transpose_and_wt,
                  const double* x, double* out, hipStream_t st) {
  const unsigned nb = nbk(g.Kpad, 256);
  LDG_SWITCH_FAC(fs, {
    const BW* fw = (const BW*)fs.w;
    const BO* fo = (const BO*)fs.o;
    if (transpose_and_wt) {
      LDG_SWITCH_N(N, (k_fac_f<NT, double, BW, BO, true, true><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, x, out, nullptr, nullptr)));
    } else {
      LDG_SWITCH_N(N, (k_fac_f<NT, double, BW, BO, false, false><<<nb, 256, 0, st>>>(
                          g, fw, fs.ws, fo, om, x, out, nullptr, nullptr)));
    }
  })
}

void launch_fac_domega(int N, const FacStore& fs, const Geo& g, const double* a,
                       const double* beta, const double* alpha, const double* y, float* dom,
                       hipStream_t st) {
  LDG_SWITCH_FAC(fs, LDG_SWITCH_N(N, (k_fac_domega<NT, BO><<<nbk(g.Kpad, 256), 256, 0, st>>>(
                                         g, (const BO*)fs.o, a, beta, alpha, y, dom))))
}

void launch_fac_export(int64_t K, int N, const FacStore& fs, double* out, hipStream_t st) {
  const unsigned nb = nbk(K * FAC_SLOTS * N * N, 256);
  LDG_SWITCH_FAC(fs, (k_fac_export_rows<BW, BO><<<nb, 256, 0, st>>>(
                         K, nullptr, N, 0, (const BW*)fs.w, fs.ws, (const BO*)fs.o, nullptr, out,
                         nullptr)))
}

void launch_fac_export_rows(int64_t n, const int32_t* elems, int N, const FacStore& fs,
                            int64_t Kpad, const float* lognorm, double* out, float* lnout,
                            hipStream_t st) {
  const unsigned nb = nbk(n * FAC_SLOTS * N * N, 256);
  LDG_SWITCH_FAC(fs, (k_fac_export_rows<BW, BO><<<nb, 256, 0, st>>>(
                         n, elems, N, Kpad, (const BW*)fs.w, fs.ws, (const BO*)fs.o, lognorm, out,
                         lnout)))
}

}  // namespace ldg
