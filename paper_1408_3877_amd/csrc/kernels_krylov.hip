// Vector kernels of the Krylov solvers, templated on the storage type T of
// the vectors (double, or float for the inner solves of the mixed modes).
// Inner products and norms always accumulate in FP64 with a deterministic
// two-stage reduction: block partials written in a fixed grid order, then
// summed by one workgroup in a fixed order.
#include <cfloat>

#include "device_common.h"
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

inline unsigned nblk1(int64_t n) { return (unsigned)((n + 255) / 256); }
}  // namespace

int krylov_nblk(int64_t n) { return (int)((n + CHUNK - 1) / CHUNK); }

// Gram-Schmidt kernels (many basis vectors against one vector).  IT items per
// thread, chosen per vector length so that a launch has at least GS_MIN_BLOCKS
// blocks: short vectors (small meshes, long GMRES cycles) would otherwise leave
// most of the chip idle.  gs_items / gs_nblk fix the partition for a length,
// so the reductions stay deterministic.
constexpr int GS_MIN_BLOCKS = 2048;
constexpr int GS_JB = 8;   // basis vectors per block of k_dots

int gs_items(int64_t n) {
  for (int it = KITEMS; it > 1; it >>= 1)
    if (n / ((int64_t)KB * it) >= GS_MIN_BLOCKS) return it;
  return 1;
}

// partials[j][b] = <V_j, w> on block b (j < nv), partials[nv][b] = <w, w>.
// Grid (nblk, ceil(nv / GS_JB)): block (b, y) takes the vectors
// [y GS_JB, min(nv, (y + 1) GS_JB)); the last row also takes <w, w>.
template <class T, int IT>
__global__ void __launch_bounds__(KB) k_dots(int64_t n, int nv, const T* __restrict__ V,
                                             int64_t ldv, const T* __restrict__ w,
                                             double* __restrict__ partials, int nblk) {
  __shared__ double red[GS_JB + 1][KB / 64];
  const int64_t base = (int64_t)blockIdx.x * (KB * IT) + threadIdx.x;
  double wl[IT];
#pragma unroll
  for (int t = 0; t < IT; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    wl[t] = i < n ? (double)w[i] : 0.0;
  }
  const int j0 = blockIdx.y * GS_JB;
  const bool last = blockIdx.y == gridDim.y - 1;
  double acc[GS_JB + 1];
#pragma unroll
  for (int jj = 0; jj < GS_JB; ++jj) {
    double s = 0.0;
    const int j = j0 + jj;
    if (j < nv) {
      const T* Vj = V + j * ldv;
#pragma unroll
      for (int t = 0; t < IT; ++t) {
        const int64_t i = base + (int64_t)t * KB;
        if (i < n) s += (double)Vj[i] * wl[t];
      }
    }
    acc[jj] = s;
  }
  double ww = 0.0;
#pragma unroll
  for (int t = 0; t < IT; ++t) ww += wl[t] * wl[t];
  acc[GS_JB] = ww;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int jj = 0; jj <= GS_JB; ++jj) {
    const double v = wave_sum(acc[jj]);
    if (lane == 0) red[jj][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x <= GS_JB) {
    const int jj = threadIdx.x;
    const int j = jj < GS_JB ? j0 + jj : nv;
    if ((jj < GS_JB && j < nv) || (jj == GS_JB && last)) {
      double s = 0.0;
      for (int q = 0; q < KB / 64; ++q) s += red[jj][q];
      partials[(int64_t)j * nblk + blockIdx.x] = s;
    }
  }
}

// w -= sum_j h[j] V_j (FP64 arithmetic), partial sums of the new <w, w>
template <class T, int IT>
__global__ void __launch_bounds__(KB) k_update(int64_t n, int nv, const T* __restrict__ V,
                                               int64_t ldv, const double* __restrict__ h,
                                               T* __restrict__ w, double* __restrict__ partials) {
  __shared__ double red[KB / 64];
  const int64_t base = (int64_t)blockIdx.x * (KB * IT) + threadIdx.x;
  double wl[IT];
#pragma unroll
  for (int t = 0; t < IT; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    wl[t] = i < n ? (double)w[i] : 0.0;
  }
  for (int j = 0; j < nv; ++j) {
    const T* Vj = V + j * ldv;
    const double hj = h[j];
#pragma unroll
    for (int t = 0; t < IT; ++t) {
      const int64_t i = base + (int64_t)t * KB;
      if (i < n) wl[t] -= hj * (double)Vj[i];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < IT; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    if (i < n) {
      const T v = (T)wl[t];
      w[i] = v;
      s += (double)v * (double)v;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// CG scalars from a reduced dot product (one thread): the step length from
// <p, A p> (CG_ALPHA), or the direction coefficient from the new <r, z>
// (CG_BETA): a non-positive curvature or <r, z> sets the flag and a step of 0,
// which every later update honours
__device__ inline void cg_alpha(double v, double* __restrict__ s) {
  s[CGS_PQ] = v;
  if (s[CGS_FLAG] != 0.0 || !(v > 0.0) || !(v <= DBL_MAX) || !(s[CGS_RZ] > 0.0)) {
    s[CGS_ALPHA] = 0.0;
    s[CGS_FLAG] = 1.0;
  } else {
    s[CGS_ALPHA] = s[CGS_NUM] / v;
    s[CGS_ITER] += 1.0;
  }
}

__device__ inline void cg_beta(double v, double* __restrict__ s) {
  if (s[CGS_FLAG] != 0.0 || !(v > 0.0) || !(v <= DBL_MAX)) {
    s[CGS_BETA] = 0.0;
    s[CGS_FLAG] = 1.0;
    return;
  }
  s[CGS_BETA] = v / s[CGS_RZ];
  s[CGS_RZ] = v;
  s[CGS_NUM] = v;
}

// one block per output: result[j] = sum_b partials[j * nblk + b], fixed order;
// RB threads (the partials of one output are few thousand: a wide block keeps
// each thread's share short).  cg_mode (single output): the CG scalar that
// follows from the result, in the same launch.
constexpr int RB = 1024;
__global__ void __launch_bounds__(RB) k_reduce(int nblk, const double* __restrict__ partials,
                                               double* __restrict__ result,
                                               double* __restrict__ cg, int cg_mode) {
  __shared__ double red[RB / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RB) s += partials[(int64_t)j * nblk + b];
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < RB / 64; ++w) t += red[w];
    result[j] = t;
    if (cg_mode == CG_ALPHA) cg_alpha(t, cg);
    else if (cg_mode == CG_BETA) cg_beta(t, cg);
  }
}

template <class T>
__global__ void k_lincomb(int64_t n, int nv, const T* __restrict__ V, int64_t ldv,
                          const double* __restrict__ y, T* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s += y[j] * (double)V[j * ldv + i];
  u[i] = (T)s;
}

template <class T>
__global__ void k_axpby(int64_t n, double a, const T* __restrict__ x, double b,
                        T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = (T)(a * (double)x[i] + (b == 0.0 ? 0.0 : b * (double)y[i]));
}

// y = x + (*bdev) y, KITEMS entries per thread like the CG update
template <class T>
__global__ void __launch_bounds__(KB) k_xpby_dev(int64_t n, const T* __restrict__ x,
                                                 const double* __restrict__ bdev,
                                                 T* __restrict__ y) {
  const double b = *bdev;
  const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    if (i < n) y[i] = (T)((double)x[i] + (b == 0.0 ? 0.0 : b * (double)y[i]));
  }
}

// CG scalars on the device, s[CGS_*] (one thread each).  start: <r, z> and the
// numerator of the first step length.  alpha: a = num / <p, A p>, or 0 with a
// flag once a curvature <p, A p> or <r, z> is not positive (every later update
// then leaves the iterate alone).  beta: b = <r, z>_new / <r, z>, the new
// <r, z> becoming the numerator of the next step length.
__global__ void k_cg_start(double* __restrict__ s, double rz, double num) {
  s[CGS_RZ] = rz;
  s[CGS_NUM] = num;
  s[CGS_PQ] = 0.0;
  s[CGS_ALPHA] = 0.0;
  s[CGS_BETA] = 0.0;
  s[CGS_FLAG] = 0.0;
  s[CGS_ITER] = 0.0;
}



// CG: x += a p, r -= a q, partial sums of the new <r, r>; with adev the step
// length is read from the device (CG scalars kept on the device)
template <class T>
__global__ void __launch_bounds__(KB) k_cg_update(int64_t n, double a, const double* __restrict__ adev,
                                                  const T* __restrict__ p,
                                                  const T* __restrict__ q, T* __restrict__ x,
                                                  T* __restrict__ r,
                                                  double* __restrict__ partials) {
  __shared__ double red[KB / 64];
  if (adev) a = *adev;
  const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < KITEMS; ++t) {
    const int64_t i = base + (int64_t)t * KB;
    if (i < n) {
      T ri = r[i];
      if (a != 0.0) {   // a step of 0 (a stopped device-side CG) leaves x and r alone
        x[i] = (T)((double)x[i] + a * (double)p[i]);
        ri = (T)((double)ri - a * (double)q[i]);
        r[i] = ri;
      }
      s += (double)ri * (double)ri;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// precision casts: out = a * in
template <class Ti, class To>
__global__ void k_cast_scale(int64_t n, double a, const Ti* __restrict__ in, To* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (To)(a * (double)in[i]);
}

// y (FP64) += a * x (any precision)
template <class T>
__global__ void k_axpy_into64(int64_t n, double a, const T* __restrict__ x,
                              double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] += a * (double)x[i];
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

__global__ void k_rhs(Geo g, int N, const double* __restrict__ C, const double* __restrict__ KDN,
                      const double* __restrict__ F, double tau, double* __restrict__ b3) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.Kpad * N) return;
  const int64_t k = (t / (64 * N)) * 64 + (t % 64);
  const double a2 = k < g.K ? g.area2[k] : 0.0;
  b3[t] = (C ? a2 * C[t] : 0.0) + tau * (KDN[t] + a2 * F[t]);
}

__global__ void k_zrows(Geo g, int N, const double* __restrict__ Za, const double* __restrict__ Zb,
                        double s, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.Kpad * N) return;
  const int64_t k = (t / (64 * N)) * 64 + (t % 64);
  const double a2 = k < g.K ? g.area2[k] : 0.0;
  out[t] = s * a2 * (Za[t] - Zb[t]);
}

// ---------------------------------------------------------------------------
// launchers (vt = VT_F64 / VT_F32 selects T)
// ---------------------------------------------------------------------------
#define LDG_VT(vt, CALL)                          \
  if ((vt) == VT_F64) { using T = double; CALL; } \
  else { using T = float; CALL; }

void reduce_partials(int nblk, const double* partials, double* result, hipStream_t st,
                     double* cg, int cg_mode) {
  k_reduce<<<1, RB, 0, st>>>(nblk, partials, result, cg, cg_mode);
}

int gs_nblk(int64_t n) {
  const int64_t chunk = (int64_t)KB * gs_items(n);
  return (int)((n + chunk - 1) / chunk);
}

#define LDG_GS_IT(n, CALL)                                 \
  switch (gs_items(n)) {                                   \
    case 8: { constexpr int IT = 8; CALL; } break;         \
    case 4: { constexpr int IT = 4; CALL; } break;         \
    case 2: { constexpr int IT = 2; CALL; } break;         \
    default: { constexpr int IT = 1; CALL; } break;        \
  }

void launch_dots(int vt, const Reducer& r, int64_t n, int nv, const void* V, int64_t ldv,
                 const void* w, hipStream_t st) {
  const int nb = gs_nblk(n);
  const dim3 grid(nb, nv > 0 ? (nv + GS_JB - 1) / GS_JB : 1);   // nv = 0: <w, w> only
  LDG_VT(vt, LDG_GS_IT(n, (k_dots<T, IT><<<grid, KB, 0, st>>>(n, nv, (const T*)V, ldv,
                                                                (const T*)w, r.partials, nb))));
  k_reduce<<<nv + 1, RB, 0, st>>>(nb, r.partials, r.result, nullptr, CG_NONE);
}

void launch_update(int vt, const Reducer& r, int64_t n, int nv, const void* V, int64_t ldv,
                   const double* h, void* w, hipStream_t st) {
  const int nb = gs_nblk(n);
  LDG_VT(vt, LDG_GS_IT(n, (k_update<T, IT><<<nb, KB, 0, st>>>(n, nv, (const T*)V, ldv, h, (T*)w,
                                                                r.partials))));
  k_reduce<<<1, RB, 0, st>>>(nb, r.partials, r.result, nullptr, CG_NONE);
}

void launch_lincomb(int vt, int64_t n, int nv, const void* V, int64_t ldv, const double* y,
                    void* u, hipStream_t st) {
  LDG_VT(vt, (k_lincomb<T><<<nblk1(n), 256, 0, st>>>(n, nv, (const T*)V, ldv, y, (T*)u)));
}

void launch_axpby(int vt, int64_t n, double a, const void* x, double b, void* y, hipStream_t st) {
  LDG_VT(vt, (k_axpby<T><<<nblk1(n), 256, 0, st>>>(n, a, (const T*)x, b, (T*)y)));
}

void launch_cg_update(int vt, const Reducer& r, int64_t n, double a, const void* p, const void* q,
                      void* x, void* rv, hipStream_t st, const double* adev, bool reduce) {
  const int nb = krylov_nblk(n);
  LDG_VT(vt, (k_cg_update<T><<<nb, KB, 0, st>>>(n, a, adev, (const T*)p, (const T*)q, (T*)x,
                                                (T*)rv, r.partials)));
  if (reduce) k_reduce<<<1, RB, 0, st>>>(nb, r.partials, r.result, nullptr, CG_NONE);
}

void launch_xpby_dev(int vt, int64_t n, const void* x, const double* bdev, void* y,
                     hipStream_t st) {
  LDG_VT(vt, (k_xpby_dev<T><<<krylov_nblk(n), KB, 0, st>>>(n, (const T*)x, bdev, (T*)y)));
}

void launch_cg_start(double* s, double rz, double num, hipStream_t st) {
  k_cg_start<<<1, 1, 0, st>>>(s, rz, num);
}


void launch_cast(int vt_in, int vt_out, int64_t n, double a, const void* in, void* out,
                 hipStream_t st) {
  if (vt_in == VT_F64 && vt_out == VT_F32)
    k_cast_scale<double, float><<<nblk1(n), 256, 0, st>>>(n, a, (const double*)in, (float*)out);
  else if (vt_in == VT_F32 && vt_out == VT_F64)
    k_cast_scale<float, double><<<nblk1(n), 256, 0, st>>>(n, a, (const float*)in, (double*)out);
  else if (vt_in == VT_F64)
    k_cast_scale<double, double><<<nblk1(n), 256, 0, st>>>(n, a, (const double*)in, (double*)out);
  else
    k_cast_scale<float, float><<<nblk1(n), 256, 0, st>>>(n, a, (const float*)in, (float*)out);
}

void launch_axpy_into64(int vt, int64_t n, double a, const void* x, double* y, hipStream_t st) {
  LDG_VT(vt, (k_axpy_into64<T><<<nblk1(n), 256, 0, st>>>(n, a, (const T*)x, y)));
}

void launch_mode_norms(int N, const Geo& g, const double* D, const Reducer& red, hipStream_t st) {
  const int nb = red.nblk < 1024 ? red.nblk : 1024;
  k_mode_norms<<<nb, KB, 0, st>>>(g.Kpad, N, D, red.partials, nb);
  k_reduce<<<2, RB, 0, st>>>(nb, red.partials, red.result, nullptr, CG_NONE);
}

void launch_rhs(const Geo& g, int N, const double* C, const double* KDN, const double* F,
                double tau, double* b3, hipStream_t st) {
  k_rhs<<<nblk1(g.Kpad * N), 256, 0, st>>>(g, N, C, KDN, F, tau, b3);
}

void launch_zrows(const Geo& g, int N, const double* Za, const double* Zb, double s, double* out,
                  hipStream_t st) {
  k_zrows<<<nblk1(g.Kpad * N), 256, 0, st>>>(g, N, Za, Zb, s, out);
}

}  // namespace ldg
