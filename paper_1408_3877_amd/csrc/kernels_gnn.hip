// Graph-network preconditioner on the element graph: features, inference,
// training (backward + Adam).  FP32, one lane per triangle, weights of the
// current layer in LDS (every lane reads the same address: broadcast).
// Messages are computed by the receiving triangle from its neighbours
// (owner computes, no atomics); in the backward pass each triangle gathers
// the gradient its own state received through its neighbours' messages.
// Weight gradients are sums over triangles (or directed edges) of outer
// products; the kernels write the two factors row by row and a tall-skinny
// A^T B kernel reduces them in a fixed order, in FP64.
//
//   node input  x_k = [r_hat_k (N), log dbar_k, D_k[1:]/D_k0, log(|T_k|/mean|T|),
//                      log(dt dbar_k/|T_k|), eta]                          (2N+3)
//   edge input  e_kn = [nu_kn, log(|E_kn|/sqrt(mean|T|)), onehot(3n+n+), log(dbar_k+/dbar_k)]  (13)
//   h0 = relu(x W_enc + b_enc); 3 layers: a_k = sum_n relu(h_{k+} W_m + e_kn W_e + b_m),
//   h_k <- h_k + relu([h_k, a_k] W_u + b_u); g = h3 W_dec + b_dec.
#include "device_common.h"
#include "kernels.h"

namespace ldg {

namespace {
constexpr int W = GNN_WIDTH;
constexpr int EIN = GNN_EIN;
constexpr int LSZ = (W + EIN + 1) * W + (2 * W + 1) * W;  // floats per layer

__device__ inline float relu(float x) { return x > 0.f ? x : 0.f; }

template <int NF>
__device__ inline void load_f(const float* __restrict__ v, int64_t k, float* x) {
#pragma unroll
  for (int i = 0; i < NF; ++i) x[i] = v[vidx(k, i, NF)];
}
template <int NF>
__device__ inline void store_f(float* __restrict__ v, int64_t k, const float* x) {
#pragma unroll
  for (int i = 0; i < NF; ++i) v[vidx(k, i, NF)] = x[i];
}

__device__ inline void load_lds(float* s, const float* __restrict__ g, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) s[t] = g[t];
  __syncthreads();
}
}  // namespace

// ---------------------------------------------------------------------------
// features from the projected coefficient D (tiled FP64)
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_gnn_features(Geo g, const double* __restrict__ D, double dt, double eta,
                               double meanA, float* __restrict__ node, float* __restrict__ edge) {
  constexpr int NF = N + 3;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  const int64_t Kp = g.Kpad;
  float f[NF];
  float e[3][EIN];
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int c = 0; c < EIN; ++c) e[n][c] = 0.f;
  if (k < g.K) {
    const double d0 = D[vidx(k, 0, N)];
    const double dbar = fabs(1.4142135623730951 * d0);
    f[0] = (float)log(dbar);
#pragma unroll
    for (int i = 1; i < N; ++i) f[i] = (float)(D[vidx(k, i, N)] / d0);
    const double area = 0.5 * g.area2[k];
    f[N] = (float)log(area / meanA);
    f[N + 1] = (float)log(dt * dbar / area);
    f[N + 2] = (float)eta;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t kp = g.nbr[n * Kp + k];
      if (kp < 0) continue;
      e[n][0] = (float)g.nu[(2 * n) * Kp + k];
      e[n][1] = (float)g.nu[(2 * n + 1) * Kp + k];
      e[n][2] = (float)log(g.elen[n * Kp + k] / sqrt(meanA));
      const int hot = 3 * n + g.nbrn[n * Kp + k];   // one-hot (n, n+), compile-time slots
#pragma unroll
      for (int c = 0; c < 9; ++c) e[n][3 + c] = c == hot ? 1.f : 0.f;
      const double dp = fabs(1.4142135623730951 * D[vidx(kp, 0, N)]);
      e[n][12] = (float)log(dp / dbar);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NF; ++i) f[i] = 0.f;
  }
  store_f<NF>(node, k, f);
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int c = 0; c < EIN; ++c) edge[vidx(k, n * EIN + c, 3 * EIN)] = e[n][c];
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// h0 = relu(x W_enc + b_enc); keeps z0 when z0 != NULL.  NR = N: x = [r_hat, node];
// NR = 0: x = node (the factored preconditioner's network sees no residual)
template <int N, int NR>
__global__ void __launch_bounds__(256) k_gnn_encode(Geo g, const float* __restrict__ rhat,
                                                    const float* __restrict__ node,
                                                    const float* __restrict__ P,
                                                    float* __restrict__ z0, float* __restrict__ h0) {
  constexpr int NIN = NR + N + 3;
  __shared__ float sw[(NIN + 1) * W];
  load_lds(sw, P, (NIN + 1) * W);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  float x[NIN];
  if (NR > 0) load_f<N>(rhat, k, x);
  load_f<N + 3>(node, k, x + NR);
  float h[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    float s = sw[NIN * W + o];
#pragma unroll
    for (int i = 0; i < NIN; ++i) s += x[i] * sw[i * W + o];
    if (z0) z0[vidx(k, o, W)] = s;
    h[o] = k < g.K ? relu(s) : 0.f;
  }
  store_f<W>(h0, k, h);
}

// one message-passing layer; keeps a and u when they are not NULL.
// Inputs stream in one channel at a time (runtime loop) against 32 unrolled
// output accumulators, so only the accumulators live in registers.
__global__ void __launch_bounds__(256) k_gnn_layer(Geo g, const float* __restrict__ hin,
                                                   const float* __restrict__ edge,
                                                   const float* __restrict__ PL,
                                                   float* __restrict__ hout, float* __restrict__ aout,
                                                   float* __restrict__ uout) {
  __shared__ float sw[LSZ];
  __shared__ float sa[256 * (W + 1)];
  load_lds(sw, PL, LSZ);
  const float* Wm = sw;
  const float* We = sw + W * W;
  const float* bm = sw + (W + EIN) * W;
  const float* Wu = sw + (W + EIN + 1) * W;
  const float* bu = Wu + 2 * W * W;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  const int64_t Kp = g.Kpad;
  const bool valid = k < g.K;
  // the three messages into k together: every weight read serves all three
  int64_t kp[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) kp[n] = valid ? g.nbr[n * Kp + k] : -1;
  float s[3][W];
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int o = 0; o < W; ++o) s[n][o] = bm[o];
  for (int i = 0; i < W; ++i) {
    float x[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) x[n] = kp[n] >= 0 ? hin[vidx(kp[n], i, W)] : 0.f;
#pragma unroll
    for (int o = 0; o < W; ++o) {
      const float w = Wm[i * W + o];
#pragma unroll
      for (int n = 0; n < 3; ++n) s[n][o] += x[n] * w;
    }
  }
  for (int c = 0; c < EIN; ++c) {
    float x[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) x[n] = edge[vidx(k, n * EIN + c, 3 * EIN)];
#pragma unroll
    for (int o = 0; o < W; ++o) {
      const float w = We[c * W + o];
#pragma unroll
      for (int n = 0; n < 3; ++n) s[n][o] += x[n] * w;
    }
  }
  float a[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    float t = 0.f;
#pragma unroll
    for (int n = 0; n < 3; ++n) t += kp[n] >= 0 ? relu(s[n][o]) : 0.f;
    a[o] = t;
  }
  float* my = sa + threadIdx.x * (W + 1);
#pragma unroll
  for (int o = 0; o < W; ++o) my[o] = a[o];
  if (aout) store_f<W>(aout, k, a);
  float u[W];
#pragma unroll
  for (int o = 0; o < W; ++o) u[o] = bu[o];
  for (int i = 0; i < W; ++i) {
    const float x = hin[vidx(k, i, W)];
    const float y = my[i];
#pragma unroll
    for (int o = 0; o < W; ++o) u[o] += x * Wu[i * W + o] + y * Wu[(W + i) * W + o];
  }
#pragma unroll
  for (int o = 0; o < W; ++o) {
    if (uout) uout[vidx(k, o, W)] = u[o];
    hout[vidx(k, o, W)] = valid ? hin[vidx(k, o, W)] + relu(u[o]) : 0.f;
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_gnn_decode(Geo g, const float* __restrict__ h3,
                                                    const float* __restrict__ PD,
                                                    float* __restrict__ out) {
  __shared__ float sw[(W + 1) * N];
  load_lds(sw, PD, (W + 1) * N);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  float h[W], y[N];
  load_f<W>(h3, k, h);
#pragma unroll
  for (int o = 0; o < N; ++o) {
    float s = sw[W * N + o];
#pragma unroll
    for (int i = 0; i < W; ++i) s += h[i] * sw[i * N + o];
    y[o] = k < g.K ? s : 0.f;
  }
  store_f<N>(out, k, y);
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// dg = 2 (g - t) / (K N), or dg = dout when the loss gradient with respect to
// g is given; dh3 = dg W_dec^T; rows for the W_dec / b_dec gradient;
// per-block partial sums of (g - t)^2 in partials[blockIdx]
template <int N>
__global__ void __launch_bounds__(256) k_gnn_decode_bwd(Geo g, const float* __restrict__ gout,
                                                        const float* __restrict__ target,
                                                        const float* __restrict__ dout,
                                                        const float* __restrict__ h3,
                                                        const float* __restrict__ PD,
                                                        float* __restrict__ dh3,
                                                        float* __restrict__ rowA,
                                                        float* __restrict__ rowB,
                                                        double* __restrict__ partials) {
  __shared__ float sw[(W + 1) * N];
  __shared__ double red[4];
  load_lds(sw, PD, (W + 1) * N);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double se = 0.0;
  if (k < g.K) {
    const float sc = 2.0f / (float)((double)g.K * N);
    float dg[N], h[W];
#pragma unroll
    for (int o = 0; o < N; ++o) {
      const float r = gout[vidx(k, o, N)] - target[vidx(k, o, N)];
      se += (double)r * (double)r;
      dg[o] = dout ? dout[vidx(k, o, N)] : sc * r;
      rowB[k * N + o] = dg[o];
    }
    load_f<W>(h3, k, h);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < N; ++o) s += dg[o] * sw[i * N + o];
      dh3[vidx(k, i, W)] = s;
      rowA[k * (W + 1) + i] = h[i];
    }
    rowA[k * (W + 1) + W] = 1.f;
  } else if (k < g.Kpad) {
#pragma unroll
    for (int i = 0; i < W; ++i) dh3[vidx(k, i, W)] = 0.f;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = se;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// layer backward, part 1 (per triangle k):
//   du = dh o [u > 0]; dh_part = dh + du W_u[0:W]^T; da = du W_u[W:2W]^T;
//   rows [h_k, a_k, 1] and du for the W_u / b_u gradient
__global__ void __launch_bounds__(256) k_gnn_layer_bwd1(Geo g, const float* __restrict__ dh,
                                                        const float* __restrict__ hprev,
                                                        const float* __restrict__ a,
                                                        const float* __restrict__ u,
                                                        const float* __restrict__ PL,
                                                        float* __restrict__ dhpart,
                                                        float* __restrict__ da,
                                                        float* __restrict__ rowA,
                                                        float* __restrict__ rowB) {
  __shared__ float sw[2 * W * W];
  load_lds(sw, PL + (W + EIN + 1) * W, 2 * W * W);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.Kpad) return;
  if (k >= g.K) {
#pragma unroll
    for (int i = 0; i < W; ++i) dhpart[vidx(k, i, W)] = da[vidx(k, i, W)] = 0.f;
    return;
  }
  float du[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    const float d = dh[vidx(k, o, W)];
    du[o] = u[vidx(k, o, W)] > 0.f ? d : 0.f;
    rowB[k * W + o] = du[o];
  }
#pragma unroll
  for (int i = 0; i < W; ++i) {
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int o = 0; o < W; ++o) {
      s1 += du[o] * sw[i * W + o];
      s2 += du[o] * sw[(W + i) * W + o];
    }
    dhpart[vidx(k, i, W)] = dh[vidx(k, i, W)] + s1;
    da[vidx(k, i, W)] = s2;
    rowA[k * (2 * W + 1) + i] = hprev[vidx(k, i, W)];
    rowA[k * (2 * W + 1) + W + i] = a[vidx(k, i, W)];
  }
  rowA[k * (2 * W + 1) + 2 * W] = 1.f;
}

// layer backward, part 2 (per triangle j, over its three directed edges j -> k):
//   p = h_j W_m + e_(k, n') W_e + b_m with n' = edge of k facing j,
//   dp = da_k o [p > 0], dh_j = dh_part_j + sum dp W_m^T,
//   rows [h_j, e, 1] and dp for the W_m / W_e / b_m gradient (zero rows on boundaries)
__global__ void __launch_bounds__(256) k_gnn_layer_bwd2(Geo g, const float* __restrict__ hprev,
                                                        const float* __restrict__ edge,
                                                        const float* __restrict__ da,
                                                        const float* __restrict__ dhpart,
                                                        const float* __restrict__ PL,
                                                        float* __restrict__ dhout,
                                                        float* __restrict__ rowA,
                                                        float* __restrict__ rowB) {
  __shared__ float sw[(W + EIN + 1) * W];
  load_lds(sw, PL, (W + EIN + 1) * W);
  const float* Wm = sw;
  const float* We = sw + W * W;
  const float* bm = sw + (W + EIN) * W;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.Kpad) return;
  const int64_t Kp = g.Kpad;
  float acc[W], hj[W];
  load_f<W>(dhpart, j, acc);
  load_f<W>(hprev, j, hj);
  for (int n = 0; n < 3; ++n) {
    const int64_t r = 3 * j + n;
    const int64_t k = j < g.K ? g.nbr[n * Kp + j] : -1;
    if (k < 0) {
      if (j < g.K) {
        for (int c = 0; c <= W + EIN; ++c) rowA[r * (W + EIN + 1) + c] = 0.f;
        for (int o = 0; o < W; ++o) rowB[r * W + o] = 0.f;
      }
      continue;
    }
    const int nk = g.nbrn[n * Kp + j];
    float e[EIN];
#pragma unroll
    for (int c = 0; c < EIN; ++c) e[c] = edge[vidx(k, nk * EIN + c, 3 * EIN)];
    float dp[W];
#pragma unroll
    for (int o = 0; o < W; ++o) {
      float s = bm[o];
#pragma unroll
      for (int i = 0; i < W; ++i) s += hj[i] * Wm[i * W + o];
#pragma unroll
      for (int c = 0; c < EIN; ++c) s += e[c] * We[c * W + o];
      dp[o] = s > 0.f ? da[vidx(k, o, W)] : 0.f;
      rowB[r * W + o] = dp[o];
    }
#pragma unroll
    for (int i = 0; i < W; ++i) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < W; ++o) s += dp[o] * Wm[i * W + o];
      acc[i] += s;
      rowA[r * (W + EIN + 1) + i] = hj[i];
    }
#pragma unroll
    for (int c = 0; c < EIN; ++c) rowA[r * (W + EIN + 1) + W + c] = e[c];
    rowA[r * (W + EIN + 1) + W + EIN] = 1.f;
  }
  if (j >= g.K) {
#pragma unroll
    for (int i = 0; i < W; ++i) acc[i] = 0.f;
  }
  store_f<W>(dhout, j, acc);
}

// encoder backward: rows [x_k, 1] and dz0 = dh0 o [z0 > 0]
template <int N, int NR>
__global__ void __launch_bounds__(256) k_gnn_encode_bwd(Geo g, const float* __restrict__ rhat,
                                                        const float* __restrict__ node,
                                                        const float* __restrict__ z0,
                                                        const float* __restrict__ dh0,
                                                        float* __restrict__ rowA,
                                                        float* __restrict__ rowB) {
  constexpr int NIN = NR + N + 3;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.K) return;
#pragma unroll
  for (int i = 0; i < NR; ++i) rowA[k * (NIN + 1) + i] = rhat[vidx(k, i, N)];
#pragma unroll
  for (int i = 0; i < N + 3; ++i) rowA[k * (NIN + 1) + NR + i] = node[vidx(k, i, N + 3)];
  rowA[k * (NIN + 1) + NIN] = 1.f;
#pragma unroll
  for (int o = 0; o < W; ++o)
    rowB[k * W + o] = z0[vidx(k, o, W)] > 0.f ? dh0[vidx(k, o, W)] : 0.f;
}

// partial[b][i][j] = sum over the rows of block b of A[r][i] B[r][j] (FP64)
__global__ void __launch_bounds__(256) k_tn_partial(int64_t rows, int pa, int qb,
                                                    const float* __restrict__ A,
                                                    const float* __restrict__ B, int rows_per_block,
                                                    double* __restrict__ partials) {
  constexpr int MAXO = 9;   // outputs per thread: up to (2W+1) x W = 2080 per block
  __shared__ float sA[32 * 80];   // pa <= 80
  __shared__ float sB[32 * 32];
  const int nout = pa * qb;
  double acc[MAXO];
#pragma unroll
  for (int t = 0; t < MAXO; ++t) acc[t] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  for (int64_t rc = r0; rc < r1; rc += 32) {
    const int nr = (int)min((int64_t)32, r1 - rc);
    __syncthreads();
    for (int t = threadIdx.x; t < 32 * pa; t += blockDim.x) {
      const int rr = t / pa, c = t % pa;
      sA[rr * pa + c] = rr < nr ? A[(rc + rr) * pa + c] : 0.f;
    }
    for (int t = threadIdx.x; t < 32 * qb; t += blockDim.x) {
      const int rr = t / qb, c = t % qb;
      sB[rr * qb + c] = rr < nr ? B[(rc + rr) * qb + c] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXO; ++t) {
      const int o = threadIdx.x + t * 256;
      if (o >= nout) break;
      const int i = o / qb, jj = o % qb;
      double s = 0.0;
      for (int rr = 0; rr < nr; ++rr) s += (double)sA[rr * pa + i] * (double)sB[rr * qb + jj];
      acc[t] += s;
    }
  }
#pragma unroll
  for (int t = 0; t < MAXO; ++t) {
    const int o = threadIdx.x + t * 256;
    if (o < nout) partials[(int64_t)blockIdx.x * nout + o] = acc[t];
  }
}

// out[o] = sum_b partials[b][o] in block order (one thread per output)
__global__ void k_tn_reduce(int nblk, int nout, const double* __restrict__ partials,
                            float* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partials[(int64_t)b * nout + o];
  out[o] = (float)s;
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ gr,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// edge head of the factored preconditioner
//   omega_kn = OMEGA_MAX sigmoid(h_k.w_hk + h_{k+}.w_hj + e_kn.w_e + w_o lognorm_kn + b_o)
// on interior edges, 0 elsewhere; head parameters [w_hk (W), w_hj (W), w_e (EIN), w_o, b_o]
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fac_head(Geo g, const float* __restrict__ h3,
                                                  const float* __restrict__ edge,
                                                  const float* __restrict__ lognorm,
                                                  const float* __restrict__ PH,
                                                  float* __restrict__ om) {
  __shared__ float sw[FAC_HEAD];
  load_lds(sw, PH, FAC_HEAD);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Kp = g.Kpad;
  if (k >= Kp) return;
  float hk[W];
  load_f<W>(h3, k, hk);
  float base = sw[2 * W + EIN + 1];
#pragma unroll
  for (int o = 0; o < W; ++o) base += hk[o] * sw[o];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const int64_t j = k < g.K ? g.nbr[n * Kp + k] : -1;
    float w = 0.f;
    if (j >= 0) {
      float a = base + sw[2 * W + EIN] * lognorm[n * Kp + k];
#pragma unroll
      for (int o = 0; o < W; ++o) a += h3[vidx(j, o, W)] * sw[W + o];
#pragma unroll
      for (int c = 0; c < EIN; ++c) a += edge[vidx(k, n * EIN + c, 3 * EIN)] * sw[2 * W + c];
      w = FAC_OMEGA_MAX / (1.f + expf(-a));
    }
    om[n * Kp + k] = w;
  }
}

// da_kn = dom_kn d omega / d a = dom_kn omega (1 - omega / OMEGA_MAX); rows
// [h_k, h_{k+}, e_kn, lognorm_kn, 1] and da per directed edge (row n K + k) for
// the head gradient; dh3_k = w_hk sum_n da_kn + w_hj sum_n da_{k+ n+}
__global__ void __launch_bounds__(256) k_fac_head_bwd(Geo g, const float* __restrict__ h3,
                                                      const float* __restrict__ edge,
                                                      const float* __restrict__ lognorm,
                                                      const float* __restrict__ PH,
                                                      const float* __restrict__ om,
                                                      const float* __restrict__ dom,
                                                      float* __restrict__ dh3,
                                                      float* __restrict__ rowA,
                                                      float* __restrict__ rowB) {
  constexpr int HR = FAC_HEAD;
  __shared__ float sw[FAC_HEAD];
  load_lds(sw, PH, FAC_HEAD);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Kp = g.Kpad;
  const int64_t K = g.K;
  if (k >= Kp) return;
  float dh[W];
#pragma unroll
  for (int o = 0; o < W; ++o) dh[o] = 0.f;
  if (k < K) {
    float hk[W];
    load_f<W>(h3, k, hk);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int64_t j = g.nbr[n * Kp + k];
      float* ra = rowA + (n * K + k) * HR;
      float da = 0.f;
      if (j >= 0) {
        const float w = om[n * Kp + k];
        da = dom[n * Kp + k] * w * (1.f - w / FAC_OMEGA_MAX);
#pragma unroll
        for (int o = 0; o < W; ++o) {
          dh[o] += da * sw[o];
          ra[o] = hk[o];
          ra[W + o] = h3[vidx(j, o, W)];
        }
#pragma unroll
        for (int c = 0; c < EIN; ++c) ra[2 * W + c] = edge[vidx(k, n * EIN + c, 3 * EIN)];
        ra[2 * W + EIN] = lognorm[n * Kp + k];
        ra[2 * W + EIN + 1] = 1.f;
        // the neighbour's edge towards k
        const int64_t jn = g.nbrn[n * Kp + k];
        const float wj = om[jn * Kp + j];
        const float daj = dom[jn * Kp + j] * wj * (1.f - wj / FAC_OMEGA_MAX);
#pragma unroll
        for (int o = 0; o < W; ++o) dh[o] += daj * sw[W + o];
      } else {
        for (int c = 0; c < HR; ++c) ra[c] = 0.f;
      }
      rowB[n * K + k] = da;
    }
  }
  store_f<W>(dh3, k, dh);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }
}

// flat parameter layouts: trunk = [W_enc (nin x W), b_enc, 3 layers], then the
// node decoder [W_dec (W x N), b_dec] (residual correction, nin = 2N + 3) or the
// edge head [w_hk (W), w_hj (W), w_e (EIN), w_o, b_o] (factored, nin = N + 3)
int64_t gnn_off_layer_nin(int nin, int l) { return (int64_t)(nin + 1) * W + (int64_t)l * LSZ; }
int64_t gnn_num_params(int N) { return gnn_off_layer_nin(2 * N + 3, 3) + (int64_t)(W + 1) * N; }
int64_t gnn_off_layer(int N, int l) { return gnn_off_layer_nin(2 * N + 3, l); }
int64_t gnn_off_dec(int N) { return gnn_off_layer(N, 3); }
int64_t fac_num_params(int N) { return gnn_off_layer_nin(N + 3, 3) + FAC_HEAD; }
int64_t fac_off_head(int N) { return gnn_off_layer_nin(N + 3, 3); }

void launch_gnn_features(int N, const Geo& g, const double* D, double dt, double eta, double meanA,
                         float* node, float* edge, hipStream_t st) {
  LDG_SWITCH_N(N, (k_gnn_features<NT><<<nb256(g.Kpad), 256, 0, st>>>(g, D, dt, eta, meanA, node,
                                                                     edge)));
}

namespace {
// encoder and layers; rhat == nullptr: node features only
void gnn_trunk(int N, const Geo& g, const float* P, const float* node, const float* edge,
               const float* rhat, GnnActs& A, hipStream_t st) {
  const unsigned nb = nb256(g.Kpad);
  const int nin = (rhat ? N : 0) + N + 3;
  if (rhat) {
    LDG_SWITCH_N(N, (k_gnn_encode<NT, NT><<<nb, 256, 0, st>>>(g, rhat, node, P, A.z0, A.h[0])));
  } else {
    LDG_SWITCH_N(N, (k_gnn_encode<NT, 0><<<nb, 256, 0, st>>>(g, rhat, node, P, A.z0, A.h[0])));
  }
  for (int l = 0; l < 3; ++l)
    k_gnn_layer<<<nb, 256, 0, st>>>(g, A.h[l], edge, P + gnn_off_layer_nin(nin, l), A.h[l + 1],
                                    A.a[l], A.u[l]);
}
}  // namespace

void launch_gnn_forward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                        const float* rhat, GnnActs& A, float* out, hipStream_t st) {
  const unsigned nb = nb256(g.Kpad);
  gnn_trunk(N, g, P, node, edge, rhat, A, st);
  LDG_SWITCH_N(N, (k_gnn_decode<NT><<<nb, 256, 0, st>>>(g, A.h[3], P + gnn_off_dec(N), out)));
}

namespace {
void tn_reduce(int64_t rows, int pa, int qb, const float* A, const float* B, double* partials,
               float* out, hipStream_t st) {
  const int rpb = 4096;
  const int nblk = (int)((rows + rpb - 1) / rpb);
  k_tn_partial<<<nblk, 256, 0, st>>>(rows, pa, qb, A, B, rpb, partials);
  k_tn_reduce<<<(unsigned)((pa * qb + 255) / 256), 256, 0, st>>>(nblk, pa * qb, partials, out);
}
}  // namespace

size_t gnn_partials_size(int64_t K) {
  const int64_t rows = 3 * K;
  return (size_t)((rows + 4095) / 4096) * (2 * W + 1) * W + 64;
}

void launch_gnn_backward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                         const float* rhat, const float* target, const float* dout,
                         const GnnActs& A, const float* out, GnnScratch& S, float* grad,
                         double* loss_partials, hipStream_t st) {
  const unsigned nb = nb256(g.Kpad);
  const int64_t K = g.K;
  LDG_SWITCH_N(N, (k_gnn_decode_bwd<NT><<<nb, 256, 0, st>>>(g, out, target, dout, A.h[3],
                                                            P + gnn_off_dec(N), S.dh[0], S.rowA,
                                                            S.rowB, loss_partials)));
  tn_reduce(K, W + 1, N, S.rowA, S.rowB, S.partials, grad + gnn_off_dec(N), st);
  gnn_trunk_backward(N, g, P, node, edge, rhat, A, S, grad, st);
}

// from d loss / d h3 in S.dh[0]: the layers' and the encoder's gradients
void gnn_trunk_backward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                        const float* rhat, const GnnActs& A, GnnScratch& S, float* grad,
                        hipStream_t st) {
  const unsigned nb = nb256(g.Kpad);
  const int64_t K = g.K;
  const int nin = (rhat ? N : 0) + N + 3;
  int cur = 0;
  for (int l = 2; l >= 0; --l) {
    const float* PL = P + gnn_off_layer_nin(nin, l);
    float* gL = grad + gnn_off_layer_nin(nin, l);
    k_gnn_layer_bwd1<<<nb, 256, 0, st>>>(g, S.dh[cur], A.h[l], A.a[l], A.u[l], PL, S.dhpart,
                                         S.da, S.rowA, S.rowB);
    tn_reduce(K, 2 * W + 1, W, S.rowA, S.rowB, S.partials, gL + (W + EIN + 1) * W, st);
    k_gnn_layer_bwd2<<<nb, 256, 0, st>>>(g, A.h[l], edge, S.da, S.dhpart, PL, S.dh[1 - cur],
                                         S.rowA, S.rowB);
    tn_reduce(3 * K, W + EIN + 1, W, S.rowA, S.rowB, S.partials, gL, st);
    cur = 1 - cur;
  }
  if (rhat) {
    LDG_SWITCH_N(N, (k_gnn_encode_bwd<NT, NT><<<nb, 256, 0, st>>>(g, rhat, node, A.z0, S.dh[cur],
                                                                  S.rowA, S.rowB)));
  } else {
    LDG_SWITCH_N(N, (k_gnn_encode_bwd<NT, 0><<<nb, 256, 0, st>>>(g, rhat, node, A.z0, S.dh[cur],
                                                                 S.rowA, S.rowB)));
  }
  tn_reduce(K, nin + 1, W, S.rowA, S.rowB, S.partials, grad, st);
}

__global__ void k_to_tiled_f(int64_t K, int64_t Kpad, int N, const float* __restrict__ src,
                             float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Kpad * N) return;
  const int64_t k = t / N;
  const int i = (int)(t % N);
  dst[vidx(k, i, N)] = k < K ? src[t] : 0.f;
}

__global__ void k_from_tiled_f(int64_t K, int N, const float* __restrict__ src,
                               float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * N) return;
  dst[t] = src[vidx(t / N, (int)(t % N), N)];
}

void launch_to_tiled_f(int64_t K, int64_t Kpad, int N, const float* src, float* dst,
                       hipStream_t st) {
  k_to_tiled_f<<<nb256(Kpad * N), 256, 0, st>>>(K, Kpad, N, src, dst);
}

void launch_from_tiled_f(int64_t K, int N, const float* src, float* dst, hipStream_t st) {
  k_from_tiled_f<<<nb256(K * N), 256, 0, st>>>(K, N, src, dst);
}

void launch_adam(int64_t n, float* p, const float* gr, float* m, float* v, float lr, int step,
                 hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<nb256(n), 256, 0, st>>>(n, p, gr, m, v, lr, b1, b2, c1, c2, 1e-8f);
}

void launch_fac_omega(int N, const Geo& g, const float* P, const float* node, const float* edge,
                      const float* lognorm, GnnActs& A, float* om, hipStream_t st) {
  gnn_trunk(N, g, P, node, edge, nullptr, A, st);
  k_fac_head<<<nb256(g.Kpad), 256, 0, st>>>(g, A.h[3], edge, lognorm, P + fac_off_head(N), om);
}

void launch_fac_omega_backward(int N, const Geo& g, const float* P, const float* node,
                               const float* edge, const float* lognorm, const GnnActs& A,
                               const float* om, const float* dom, GnnScratch& S, float* grad,
                               hipStream_t st) {
  k_fac_head_bwd<<<nb256(g.Kpad), 256, 0, st>>>(g, A.h[3], edge, lognorm, P + fac_off_head(N),
                                                  om, dom, S.dh[0], S.rowA, S.rowB);
  tn_reduce(3 * g.K, FAC_HEAD, 1, S.rowA, S.rowB, S.partials, grad + fac_off_head(N), st);
  gnn_trunk_backward(N, g, P, node, edge, nullptr, A, S, grad, st);
}

}  // namespace ldg
