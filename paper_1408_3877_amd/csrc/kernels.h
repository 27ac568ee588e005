// Launchers of the device kernels (host side), all asynchronous on `st`.
#pragma once
#include "ldg_internal.h"

namespace ldg {

void launch_project(int N, int64_t K, int64_t Kpad, int R, const double* samples, const double* W,
                    double* out, hipStream_t st);
void launch_boundary(int N, const Geo& g, int64_t nbe, const int32_t* belem, int R1,
                     const double* Wb, const double* ws, const double* cD, const double* gN,
                     int64_t nbnd, const double* D, double eta, double* J1, double* J2,
                     double* KDN, hipStream_t st);
// vector storage (VT_*) and block storage (BT_*) precisions
enum { VT_F64 = 0, VT_F32 = 1 };
enum { BT_F64 = 0, BT_F32 = 1, BT_BF16 = 2, BT_FP8 = 3 };

// kernels_apply.hip
// Quadrature form of the FP32 apply (no stored blocks), with Q =
// edge_trace_points(N) Gauss points per edge and RV = vol_points(N) volume points:
//   dE    [Kpad][3Q] tiled: d_h at the points of the triangle's own edges
//   dvol  [Kpad][RV] tiled: w_q d_h(x_q) at the volume points
//   trace [3][Q][N]: phi_j at point q of reference edge n (trace64: the same in FP64)
//   lift  [3][Q][N]: w_q phi_i at the same points
//   vtab  [RV][3][N]: phi_i, dphi_i/dx1_hat, dphi_i/dx2_hat at x_q
//   vol64 [RV][N]: w_q phi_l(x_q) in FP64
//   sig   [Kpad][3Q] tiled: d_h nu.Z_h at the edge points (interior and
//         Dirichlet edges), written by the gradient half, read by the
//         triangle itself and its neighbours in the divergence half
//   pen   [Kpad][N] tiled: the penalty rows, written by the gradient half
struct EdgeTraces {
  float* dE;
  float* dvol;
  const float* trace;
  const float* lift;
  const float* vtab;
  const double* trace64;
  const double* vol64;
  float* sig;
  float* pen;
  float eta;
};
// refs: the 14 reference matrices in FP64 (N x N each); refs32: the same in FP32;
// tr (FP32 only, optional): also write the flux traces tr->sig and the penalty rows tr->pen
void launch_grad(int N, int vt, const Geo& g, const double* refs, const float* refs32,
                 const void* C, const void* J1, const void* J2, void* Z1, void* Z2,
                 hipStream_t st, const EdgeTraces* tr = nullptr);
struct Reducer;
// red (optional): red->result[0] = <C, y> afterwards; tr (FP32, optional):
// the quadrature form, blocks not read
void launch_div(int N, int vt, int bt, const Geo& g, const double* refs, const void* blocks,
                const void* C, const void* Z1, const void* Z2, double alpha, double tau,
                double eta, void* y, hipStream_t st, const Reducer* red = nullptr,
                const EdgeTraces* tr = nullptr);
// dE and dvol of EdgeTraces from the FP64 tiled coefficients D
void launch_edge_d(int N, const Geo& g, const double* D, const EdgeTraces& tr, hipStream_t st);
// z = P^{-1} r; with red != NULL also red->result[0] = <r, z>
void launch_bj_apply(int N, int vt, int bt, const Geo& g, const void* bj, const void* r, void* z,
                     const Reducer* red, hipStream_t st);
void launch_convert_blocks(int bt, int64_t Kpad, int N, int ns, const double* src, void* dst,
                           hipStream_t st);
size_t block_bytes(int bt, int64_t Kpad, int N, int ns);
// FP64 stored blocks of the listed triangles as [n][ns][N][N]
void launch_export_rows(int64_t n, const int32_t* elems, int N, int ns, const double* src,
                        double* dst, hipStream_t st);
// kernels_assemble_mfma.hip: the 5 D-dependent blocks per triangle on the
// matrix cores; T = reference tensors in the operand layout of precision bt
void launch_assemble_mfma(int N, int bt, const Geo& g, const double* D, const void* T, void* blocks,
                          hipStream_t st);
// export stored blocks of any precision as FP64 [K][ns][N][N]
void launch_export_blocks_any(int bt, int64_t K, int N, int ns, const void* src, double* dst,
                              hipStream_t st);
// matrix-free block terms: y += tau (sum_m B^m Z^m + sum_n U_kn w_n) with the
// blocks contracted from D on the matrix cores; table from mf_build_table (FP64,
// or converted to FP32 for vt = VT_F32); red (optional): <C, y> of the result
int mf_table_size(int N);
void mf_build_table(int N, const double* const* tens, double* out);
void launch_mf_blocks(int N, int vt, const Geo& g, const double* D, const void* table,
                      const void* C, const void* Z1, const void* Z2, double tau, void* y,
                      const Reducer* red, hipStream_t st);
// out[k][l] = sum_i C(k, i) phiL[l][i] (K x nL, element-major); C tiled or element-major
void launch_lagrange(int64_t K, int N, int nL, const double* C, bool tiled, const double* phiL,
                     double* out, hipStream_t st);
// alpha scales the mass term (1 for a time step, 0 for the stationary operator)
void launch_bj_setup(int N, const Geo& g, const double* refs, const double* blocks, double alpha,
                     double tau, double eta, double* bj, int* status, hipStream_t st);
void launch_to_tiled(int64_t K, int64_t Kpad, int N, const double* src, double* dst,
                     hipStream_t st);
void launch_from_tiled(int64_t K, int N, const double* src, double* dst, hipStream_t st);
void launch_export_blocks(int64_t K, int N, int ns, const double* src, double* dst,
                          hipStream_t st);
void launch_sample_vol(const Geo& g, int R, const double* q, int kind, double t, const double* dT,
                       double* d, double* f, double* c0, double* xo, double* yo, hipStream_t st);
void launch_sample_bnd(const Geo& g, int R1, const double* s, int64_t nbnd, const int32_t* bk,
                       const int8_t* bn, int kind, double t, double* cD, double* gN, double* xo,
                       double* yo, hipStream_t st);

// kernels_gnn.hip: graph-network preconditioner (FP32)
constexpr int GNN_WIDTH = 32;
constexpr int GNN_EIN = 13;
struct GnnActs {
  float* z0 = nullptr;                      // encoder pre-activation (training only)
  float* h[4] = {nullptr, nullptr, nullptr, nullptr};
  float* a[3] = {nullptr, nullptr, nullptr};  // aggregated messages (training only)
  float* u[3] = {nullptr, nullptr, nullptr};  // update pre-activations (training only)
};
struct GnnScratch {
  float* dh[2] = {nullptr, nullptr};
  float* dhpart = nullptr;
  float* da = nullptr;
  float* rowA = nullptr;      // 3K x (W + EIN + 1) at most
  float* rowB = nullptr;      // 3K x W at most
  double* partials = nullptr; // gnn_partials_size(K)
};
int64_t gnn_num_params(int N);
int64_t gnn_off_layer(int N, int l);
int64_t gnn_off_dec(int N);
// the factored preconditioner's network: trunk on node features only, edge head
constexpr int FAC_HEAD = 2 * GNN_WIDTH + GNN_EIN + 2;
constexpr float FAC_OMEGA_MAX = 0.95f;
int64_t fac_num_params(int N);
int64_t fac_off_head(int N);
size_t gnn_partials_size(int64_t K);
void launch_gnn_features(int N, const Geo& g, const double* D, double dt, double eta, double meanA,
                         float* node, float* edge, hipStream_t st);
void launch_gnn_forward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                        const float* rhat, GnnActs& A, float* out, hipStream_t st);
// gradient of mean (out - target)^2 into grad, or, when dout is given, of the loss
// whose gradient with respect to out is dout; loss_partials[b] = sums of
// (out - target)^2 per block
void launch_gnn_backward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                         const float* rhat, const float* target, const float* dout,
                         const GnnActs& A, const float* out, GnnScratch& S, float* grad,
                         double* loss_partials, hipStream_t st);
// d loss / d h3 in S.dh[0] -> trunk gradients (rhat == nullptr: node features only)
void gnn_trunk_backward(int N, const Geo& g, const float* P, const float* node, const float* edge,
                        const float* rhat, const GnnActs& A, GnnScratch& S, float* grad,
                        hipStream_t st);
// omega [3][Kpad] from the network (activations kept in A when its training slots are set)
void launch_fac_omega(int N, const Geo& g, const float* P, const float* node, const float* edge,
                      const float* lognorm, GnnActs& A, float* om, hipStream_t st);
// gradient of the loss with respect to the parameters given d loss / d omega
void launch_fac_omega_backward(int N, const Geo& g, const float* P, const float* node,
                               const float* edge, const float* lognorm, const GnnActs& A,
                               const float* om, const float* dom, GnnScratch& S, float* grad,
                               hipStream_t st);
void launch_adam(int64_t n, float* p, const float* gr, float* m, float* v, float lr, int step,
                 hipStream_t st);

// kernels_factor.hip: factor blocks W_k (one slot, storage wt) and O_k0..2
// (three slots, storage ot), BT_F32 / BT_BF16 / BT_FP8, arithmetic in the vector type
constexpr int FAC_SLOTS = 4;   // W_k, O_k0, O_k1, O_k2 in the exports
struct FacStore {
  int wt = BT_BF16, ot = BT_FP8;
  void* w = nullptr;   // W: Kpad x 1 slot, the upper triangle packed row by row
  void* o = nullptr;   // O: Kpad x 3 slots
  float* ws = nullptr; // per-triangle power-of-two scale of W when wt = BT_FP8 (W = ws W8)
};
// W (FP64 scratch w64 and the W store), O blocks and log ||O||_F from the FP64
// operator blocks and block-Jacobi inverses; status |= 2 on a failed Cholesky
void launch_fac_setup(int N, const FacStore& fs, const Geo& g, const double* refs,
                      const double* blocks, const double* bj, double tau, double eta, double* w64,
                      float* lognorm, int* status, bool sym, hipStream_t st);
// z = P r through y, a (work vectors); red: result[0] = <r, z>
void launch_fac_apply(int N, const FacStore& fs, int vt, const Geo& g, const float* om,
                      const void* r, void* y, void* a, void* z, const Reducer* red,
                      hipStream_t st);
void launch_fac_w(int N, const FacStore& fs, const Geo& g, const double* x, double* y,
                  hipStream_t st);
void launch_fac_wt(int N, const FacStore& fs, const Geo& g, const double* x, double* y,
                   hipStream_t st);
// out = (I + F) x, or W^T (I + F)^T x
void launch_fac_f(int N, const FacStore& fs, const Geo& g, const float* om, bool transpose_and_wt,
                  const double* x, double* out, hipStream_t st);
void launch_fac_domega(int N, const FacStore& fs, const Geo& g, const double* a,
                       const double* beta, const double* alpha, const double* y, float* dom,
                       hipStream_t st);
// out[k][s][i][j] (FP64): s = 0 W_k, s = 1..3 O_k(s-1); rows = all K, or elems[0..n)
void launch_fac_export(int64_t K, int N, const FacStore& fs, double* out, hipStream_t st);
void launch_fac_export_rows(int64_t n, const int32_t* elems, int N, const FacStore& fs,
                            int64_t Kpad, const float* lognorm, double* out, float* lnout,
                            hipStream_t st);
void launch_to_tiled_f(int64_t K, int64_t Kpad, int N, const float* src, float* dst,
                       hipStream_t st);
void launch_from_tiled_f(int64_t K, int N, const float* src, float* dst, hipStream_t st);

// Krylov vector kernels (kernels_krylov.hip); n = vector length, V = basis
// with vectors at V + j*ldv; vt selects the vector storage type.  Inner
// products accumulate in FP64; reductions are two-stage and fixed-order.
struct Reducer {
  double* partials = nullptr;
  double* result = nullptr;     // device
  int nblk = 0;
  int maxv = 0;
  // the single-result reductions of the applies (reduce_partials) can derive
  // a CG scalar from their result in the same launch: cg_mode CG_ALPHA or
  // CG_BETA on the scalars cg (CGS_*)
  double* cg = nullptr;
  int cg_mode = 0;
};
int krylov_nblk(int64_t n);
// blocks of the Gram-Schmidt kernels (launch_dots, launch_update) for vectors of length n
int gs_nblk(int64_t n);
enum { CG_NONE = 0, CG_ALPHA = 1, CG_BETA = 2 };
void reduce_partials(int nblk, const double* partials, double* result, hipStream_t st,
                     double* cg = nullptr, int cg_mode = CG_NONE);
// result[j] = <V_j, w> for j < nv, result[nv] = <w, w>
void launch_dots(int vt, const Reducer& r, int64_t n, int nv, const void* V, int64_t ldv,
                 const void* w, hipStream_t st);
// w -= sum_j h[j] V_j (h device); result[0] = <w, w> afterwards
void launch_update(int vt, const Reducer& r, int64_t n, int nv, const void* V, int64_t ldv,
                   const double* h, void* w, hipStream_t st);
// u = sum_j y[j] V_j (y device)
void launch_lincomb(int vt, int64_t n, int nv, const void* V, int64_t ldv, const double* y,
                    void* u, hipStream_t st);
// y = a x + b y
void launch_axpby(int vt, int64_t n, double a, const void* x, double b, void* y, hipStream_t st);
// CG: x += a p, r -= a q; result[0] = <r, r> afterwards (a = *adev when adev != NULL;
// reduce = false leaves the partial sums unreduced)
void launch_cg_update(int vt, const Reducer& r, int64_t n, double a, const void* p, const void* q,
                      void* x, void* rv, hipStream_t st, const double* adev = nullptr,
                      bool reduce = true);
// CG scalars kept on the device: s[CGS_*], set by one-thread kernels in stream
// order, so the host reads them only when it checks convergence
enum { CGS_RZ = 0, CGS_NUM = 1, CGS_PQ = 2, CGS_ALPHA = 3, CGS_BETA = 4, CGS_FLAG = 5, CGS_ITER = 6,
       CGS_N = 8 };
void launch_cg_start(double* s, double rz, double num, hipStream_t st);
// (the reductions' CG_ALPHA epilogue: s[ALPHA] = s[NUM] / <p, A p> and
// s[ITER] += 1, or 0 and s[FLAG] = 1 on a non-positive curvature, an update
// with step 0 leaving x and r alone; CG_BETA: s[BETA] = <r, z> / s[RZ], then
// s[RZ] = s[NUM] = <r, z>, the flag on <r, z> <= 0)
// y = x + s[BETA] y, the coefficient read on the device
void launch_xpby_dev(int vt, int64_t n, const void* x, const double* bdev, void* y, hipStream_t st);
// out = a * in across precisions
void launch_cast(int vt_in, int vt_out, int64_t n, double a, const void* in, void* out,
                 hipStream_t st);
// y += a x with y FP64
void launch_axpy_into64(int vt, int64_t n, double a, const void* x, double* y, hipStream_t st);
// result[0] = sum_k D_k0^2, result[1] = sum_k sum_{i>0} D_ki^2
void launch_mode_norms(int N, const Geo& g, const double* D, const Reducer& red, hipStream_t st);
// b3 = 2|T| C + tau (KDN + 2|T| F) in the tiled layout; C = nullptr drops the history term
void launch_rhs(const Geo& g, int N, const double* C, const double* KDN, const double* F,
                double tau, double* b3, hipStream_t st);
// out = s * area2 * (Za - Zb) per element (full-operator rows 1, 2)
void launch_zrows(const Geo& g, int N, const double* Za, const double* Zb, double s, double* out,
                  hipStream_t st);

}  // namespace ldg
