// Vector kernels of the Krylov solver: FP64 inner products with a
// deterministic two-stage reduction (block partials written in a fixed
// grid order, then summed by one workgroup in a fixed order), the
// Gram-Schmidt update fused with the norm of its result, and BLAS-1 helpers.
#include "kernels.h"

namespace ldg {

namespace {
constexpr int KB = 256;       // threads per block
constexpr int KITEMS = 8;     // items per thread of the dot/update kernels
constexpr int CHUNK = KB * KITEMS;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum, result valid in thread 0; `red` holds KB/64 doubles
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < KB / 64; ++w) s += red[w];
  return s;
}
}  // namespace

int krylov_nblk(int64_t n) { return (int)((n + CHUNK - 1) / CHUNK); }

__global__ void __launch_bounds__(KB) k_dots(int64_t n, int nv, const double* __restrict__ V,
                                             int64_t ldv, const double* __restrict__ w,
                                             double* __restrict__ partials, int nblk) {
  __shared__ double red[KB / 64];
  const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double wl[KITEMS];
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    wl[t] = i < n ? w[i] : 0.0;
  }
  for (int j = 0; j < nv; ++j) {
    const double* Vj = V + j * ldv;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < KITEMS; ++t) {
      const int64_t i = base + (int64_t)t * KB;
      if (i < n) s += Vj[i] * wl[t];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partials[(int64_t)j * nblk + blockIdx.x] = s;
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) s += wl[t] * wl[t];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[(int64_t)nv * nblk + blockIdx.x] = s;
}

__global__ void __launch_bounds__(KB) k_update(int64_t n, int nv, const double* __restrict__ V,
                                               int64_t ldv, const double* __restrict__ h,
                                               double* __restrict__ w,
                                               double* __restrict__ partials) {
  __shared__ double red[KB / 64];
  const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double wl[KITEMS];
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    wl[t] = i < n ? w[i] : 0.0;
  }
  for (int j = 0; j < nv; ++j) {
    const double* Vj = V + j * ldv;
    const double hj = h[j];
#pragma unroll
    for (int t = 0; t < KITEMS; ++t) {
      const int64_t i = base + (int64_t)t * KB;
      if (i < n) wl[t] -= hj * Vj[i];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    if (i < n) {
      w[i] = wl[t];
      s += wl[t] * wl[t];
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// one block per output: result[j] = sum_b partials[j * nblk + b], fixed order
__global__ void __launch_bounds__(KB) k_reduce(int nblk, const double* __restrict__ partials,
                                               double* __restrict__ result) {
  __shared__ double red[KB / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KB) s += partials[(int64_t)j * nblk + b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) result[j] = s;
}

__global__ void k_lincomb(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                          const double* __restrict__ y, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s += y[j] * V[j * ldv + i];
  u[i] = s;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void k_rhs(Geo g, int N, const double* __restrict__ C, const double* __restrict__ KDN,
                      const double* __restrict__ F, double tau, double* __restrict__ b3) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.Kpad * N) return;
  const int64_t k = (t / (64 * N)) * 64 + (t % 64);
  const double a2 = k < g.K ? g.area2[k] : 0.0;
  b3[t] = a2 * C[t] + tau * (KDN[t] + a2 * F[t]);
}

__global__ void k_zrows(Geo g, int N, const double* __restrict__ Za, const double* __restrict__ Zb,
                        double s, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.Kpad * N) return;
  const int64_t k = (t / (64 * N)) * 64 + (t % 64);
  const double a2 = k < g.K ? g.area2[k] : 0.0;
  out[t] = s * a2 * (Za[t] - Zb[t]);
}

__global__ void __launch_bounds__(KB) k_cg_update(int64_t n, double a,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ q,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ partials) {
  __shared__ double red[KB / 64];
  const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    if (i < n) {
      x[i] += a * p[i];
      const double ri = r[i] - a * q[i];
      r[i] = ri;
      s += ri * ri;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(KB) k_mode_norms(int64_t Kpad, int N, const double* __restrict__ D,
                                                   double* __restrict__ partials, int nblk) {
  __shared__ double red[KB / 64];
  double s0 = 0.0, s1 = 0.0;
  const int64_t n = Kpad * N;
  for (int64_t t = (int64_t)blockIdx.x * KB + threadIdx.x; t < n; t += (int64_t)nblk * KB) {
    const int i = (int)((t / 64) % N);
    const double v = D[t];
    if (i == 0) s0 += v * v; else s1 += v * v;
  }
  s0 = block_sum(s0, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s0;
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) partials[nblk + blockIdx.x] = s1;
}

void reduce_partials(int nblk, const double* partials, double* result, hipStream_t st) {
  k_reduce<<<1, KB, 0, st>>>(nblk, partials, result);
}

void launch_cg_update(const Reducer& r, int64_t n, double a, const double* p, const double* q,
                      double* x, double* rv, hipStream_t st) {
  const int nb = krylov_nblk(n);
  k_cg_update<<<nb, KB, 0, st>>>(n, a, p, q, x, rv, r.partials);
  k_reduce<<<1, KB, 0, st>>>(nb, r.partials, r.result);
}

void launch_mode_norms(int N, const Geo& g, const double* D, const Reducer& red, hipStream_t st) {
  const int nb = red.nblk < 1024 ? red.nblk : 1024;
  k_mode_norms<<<nb, KB, 0, st>>>(g.Kpad, N, D, red.partials, nb);
  k_reduce<<<2, KB, 0, st>>>(nb, red.partials, red.result);
}

void launch_dots(const Reducer& r, int64_t n, int nv, const double* V, int64_t ldv,
                 const double* w, hipStream_t st) {
  const int nb = krylov_nblk(n);
  k_dots<<<nb, KB, 0, st>>>(n, nv, V, ldv, w, r.partials, nb);
  k_reduce<<<nv + 1, KB, 0, st>>>(nb, r.partials, r.result);
}

void launch_update(const Reducer& r, int64_t n, int nv, const double* V, int64_t ldv,
                   const double* h, double* w, hipStream_t st) {
  const int nb = krylov_nblk(n);
  k_update<<<nb, KB, 0, st>>>(n, nv, V, ldv, h, w, r.partials);
  k_reduce<<<1, KB, 0, st>>>(nb, r.partials, r.result);
}

void launch_lincomb(int64_t n, int nv, const double* V, int64_t ldv, const double* y, double* u,
                    hipStream_t st) {
  k_lincomb<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, nv, V, ldv, y, u);
}

void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  k_axpby<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, x, b, y);
}

void launch_rhs(const Geo& g, int N, const double* C, const double* KDN, const double* F,
                double tau, double* b3, hipStream_t st) {
  k_rhs<<<(unsigned)((g.Kpad * N + 255) / 256), 256, 0, st>>>(g, N, C, KDN, F, tau, b3);
}

void launch_zrows(const Geo& g, int N, const double* Za, const double* Zb, double s, double* out,
                  hipStream_t st) {
  k_zrows<<<(unsigned)((g.Kpad * N + 255) / 256), 256, 0, st>>>(g, N, Za, Zb, s, out);
}

}  // namespace ldg
