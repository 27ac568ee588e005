// C ABI of the LDG library: context, data upload, one implicit Euler step
// (projection, assembly, preconditioner, restarted GMRES, recovery of Z).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"

using namespace ldg;

// orders of the learned preconditioner and of the matrix-free apply (their
// kernels are instantiated for N <= 15); the stored-block path runs to p = 6
constexpr int kMaxLearnedOrder = 4;

struct ldg_ctx {
  std::string err;
  // host copies of the mesh (file output) and the basis at the Lagrange points
  std::vector<double> h_coordV;
  std::vector<int32_t> h_V0T;
  int nL = 1;
  double* phiL = nullptr;   // device [nL][N]
  ldg_options opt{};
  hipStream_t st = nullptr;
  int device = 0;
  int p = 0, N = 1, NN = 1, NP = 1, R = 1, R1 = 1;
  int64_t K = 0, Kpad = 0, nbnd = 0, nbe = 0, Eint = 0, nvec = 0;
  RefData ref;
  Geo geo{};
  std::vector<void*> allocs;
  // geometry
  double *area2 = nullptr, *B = nullptr, *a1 = nullptr, *elen = nullptr, *nu = nullptr;
  float *ainv32 = nullptr, *B32 = nullptr, *elen32 = nullptr, *nu32 = nullptr;
  int32_t *nbr = nullptr, *bidx = nullptr, *belem = nullptr, *bk = nullptr;
  int8_t *nbrn = nullptr, *kind = nullptr, *bn = nullptr;
  // reference data
  double* refs = nullptr;
  float* refs32 = nullptr;
  double *Wvol = nullptr, *qvol = nullptr, *Wb = nullptr, *ws = nullptr, *sb = nullptr;
  // state and work, element-fastest layout
  double *C = nullptr, *Z1 = nullptr, *Z2 = nullptr, *D = nullptr, *F = nullptr;
  double *J1 = nullptr, *J2 = nullptr, *KDN = nullptr, *b3 = nullptr;
  double *r = nullptr, *w = nullptr, *z = nullptr, *u = nullptr, *X = nullptr;
  double *tZ1 = nullptr, *tZ2 = nullptr, *tmp = nullptr;
  double *blocks = nullptr, *bj = nullptr, *V = nullptr;
  double *d64 = nullptr, *u2 = nullptr, *iz1 = nullptr, *iz2 = nullptr;
  // mixed modes: FP32 work vectors, low-precision blocks, FP32 block-Jacobi
  float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  float *u32 = nullptr, *tz1_32 = nullptr, *tz2_32 = nullptr, *V32 = nullptr;
  void *blocks_f32 = nullptr, *blocks_bf16 = nullptr, *bj_f32 = nullptr;
  // edge-trace form of the off-diagonal edge blocks in the FP32 apply
  bool tr = false;
  EdgeTraces etr{};
  // reference tensors in the MFMA operand layouts (FP64, FP32, BF16)
  void *Tm64 = nullptr, *Tm32 = nullptr, *Tm16 = nullptr;
  bool blocks_f32_ready = false;
  double *hdev = nullptr, *ydev = nullptr;
  int* status = nullptr;
  Reducer red, red2;
  double* host_buf = nullptr;  // pinned
  int mmax = 0;        // restart length the GMRES buffers hold
  int restart_cur = 0;  // current GMRES restart length (grows on stagnating cycles)
  bool gmres_full = false;  // the last GMRES cycle ran restart_cur iterations
  double t = 0.0;
  bool blocks_ready = false;
  // graph-network preconditioner
  float *gP = nullptr, *gGrad = nullptr, *gM = nullptr, *gV = nullptr;
  int64_t gnP = 0;
  bool gnn_params_set = false, gnn_alloc_inf = false, gnn_alloc_train = false;
  int gstep = 0;
  float *gnode = nullptr, *gedge = nullptr, *g_rhat = nullptr, *g_out = nullptr, *g_tgt = nullptr;
  GnnActs gA;          // inference activations (two buffers alternate)
  GnnActs gT;          // training activations (all kept)
  GnnScratch gS;
  double* g_loss = nullptr;
  double meanA = 0.0;
  // training loss: LDG_GNN_LOSS_MSE or LDG_GNN_LOSS_ENERGY (the latter needs the
  // FP64 blocks of the context coefficient and its time step)
  int gloss = 0;
  double gtau = 0.0;
  bool g_energy_ready = false;
  float* g_dout = nullptr;
  // network mode (LDG_GNN_CORRECTION / LDG_GNN_FACTOR) and the factored
  // preconditioner's buffers: factor blocks (FP32), FP64 W, log ||O||, omega,
  // d loss / d omega, FP64 and FP32 work vectors
  int gmode = 0;
  bool fac_alloc_inf = false, fac_alloc_train = false, fac_on = false, fac_built = false;
  FacStore fac;           // factor blocks W (one slot) and O (three slots)
  float *fac_lognorm = nullptr, *fac_om = nullptr, *fac_dom = nullptr;
  double* fac_w64 = nullptr;
  double* fac_v[8] = {};
  float *fac_y32 = nullptr, *fac_a32 = nullptr;
  // collection of (r, e) pairs from the FP64 CG solve of the next step
  int col_n = 0, col_done = 0, col_taken = 0, col_cap = 0;
  std::vector<int> col_iters;
  float *col_rhat = nullptr, *col_tgt = nullptr;
  double* col_snap = nullptr;
  // kernel timing
  struct Pending { int id; hipEvent_t a, b; double bytes, flops; };
  bool timing = false;
  std::vector<hipEvent_t> evpool;
  std::vector<Pending> pending;
  ldg_kernel_stat stats[LDG_K_COUNT] = {};
  int stat_as = -1;   // >= 0: count the timed launches under this kernel id instead
  int64_t n_sd = 0, n_nd = 0;   // local edges that are not Neumann / not Dirichlet
  double inner_rho = 1.0;       // residual reduction the last inner solve reported
  // CG state kept across the refinement sweeps of one step: the last search
  // direction and its image (L.p, L.q of the level it ran at) and <p, A p>
  bool cg_kept = false;
  double cg_kept_pq = 0.0;
  double* cgs = nullptr;   // CG scalars on the device (CGS_*)
  // time scheme: implicit Euler, or two-step backward differentiation with the
  // state of the previous step (kept after every step) and its step size
  int tscheme = 0;
  double *Cprev = nullptr, *Cstar = nullptr;
  bool have_prev = false;
  double dt_prev = 0.0;
  double alpha = 1.0;   // mass coefficient of the operator (0 for the stationary system)
  // host field callbacks: host copies of the sample points, device sample buffers
  std::vector<double> cb_x, cb_y, cb_bx, cb_by, cb_nx, cb_ny;
  double *cb_d = nullptr, *cb_f = nullptr, *cb_cD = nullptr, *cb_gN = nullptr, *cb_c0 = nullptr;
  // matrix-free apply: the block terms contracted from D on the matrix cores
  bool mf = false;
  double* mf64 = nullptr;
  float* mf32 = nullptr;
};

namespace {

uint16_t host_bf16(float x) {   // round to nearest even
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

ldg_status fail(ldg_ctx* c, ldg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, LDG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
ldg_status dalloc(ldg_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, LDG_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return LDG_OK;
}

template <class T>
void dfree(ldg_ctx* c, T*& p) {
  if (!p) return;
  for (auto& q : c->allocs)
    if (q == static_cast<void*>(p)) {
      q = c->allocs.back();
      c->allocs.pop_back();
      break;
    }
  (void)hipFree(p);
  p = nullptr;
}

template <class T>
ldg_status upload(ldg_ctx* c, T* dst, const std::vector<T>& src) {
  if (src.empty()) return LDG_OK;
  HIPCHK(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->st));
  return LDG_OK;
}

#define TRY(expr)                      \
  do {                                 \
    ldg_status s_ = (expr);            \
    if (s_ != LDG_OK) return s_;       \
  } while (0)

ldg_status check_launch(ldg_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, LDG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return LDG_OK;
}

hipEvent_t ev_get(ldg_ctx* c) {
  if (!c->evpool.empty()) {
    hipEvent_t e = c->evpool.back();
    c->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records HIP events around the launches of its scope when timing is on.
struct Timed {
  ldg_ctx* c;
  int id;
  double bytes, flops;
  hipEvent_t a = nullptr;
  Timed(ldg_ctx* c_, int id_, double bytes_, double flops_)
      : c(c_), id(c_->stat_as >= 0 ? c_->stat_as : id_), bytes(bytes_), flops(flops_) {
    if (c->timing) {
      a = ev_get(c);
      if (a) (void)hipEventRecord(a, c->st);   // timing is best effort
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = ev_get(c);
    if (!b) return;
    (void)hipEventRecord(b, c->st);
    c->pending.push_back({id, a, b, bytes, flops});
  }
};

void drain_events(ldg_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& s = c->stats[p.id];
      s.launches += 1;
      s.total_ms += ms;
      s.bytes += p.bytes;
      s.flops += p.flops;
    }
    c->evpool.push_back(p.a);
    c->evpool.push_back(p.b);
  }
  c->pending.clear();
}

ldg_status sync(ldg_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (!c->pending.empty()) drain_events(c);
  return LDG_OK;
}

// ---- one precision level of the solver ------------------------------------
// vt: vector storage, bt: stored-block storage; work vectors of that level.
struct Level {
  int vt = VT_F64, bt = BT_F64;
  const void* blocks = nullptr;
  const void* bj = nullptr;
  const EdgeTraces* tr = nullptr;   // FP32 level of a context in the edge-trace form
  void *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *d = nullptr, *u = nullptr;
  void *tz1 = nullptr, *tz2 = nullptr, *V = nullptr;
  double vbytes = 8.0, bbytes = 8.0;   // bytes per vector / block entry
};

double div_bytes(const ldg_ctx* c, const Level& L) {
  const double NN = (double)c->N * c->N;
  // geometry: kind, k+, n+, the normals and |T| (the normals in FP32 for the FP32 kernels)
  const double geo = L.vbytes == 8.0 ? 74.0 : 50.0;
  const double vec = L.vbytes * 4.0 * c->N * c->K;
  if (L.tr) {
    // quadrature form: C, Z^1, Z^2, the penalty rows and y; d_h at the volume
    // points; the flux traces of the triangle's interior and Dirichlet edges and
    // of the neighbours (Q per edge side); kind, k+, n+, FP32 B, edge lengths, |T|
    const double Q = edge_trace_points(c->N), RV = vol_points(c->N);
    const double n_tr = c->n_sd;   // interior edge sides + Dirichlet edges
    return 4.0 * 5.0 * c->N * c->K + 4.0 * RV * c->K + 4.0 * Q * (n_tr + 2.0 * c->Eint) +
           62.0 * c->K;
  }
  return L.bbytes * NN * (2.0 * c->K + 2.0 * c->Eint) + vec + geo * c->K;
}
double div_flops(const ldg_ctx* c, const Level& L) {
  const double NN = (double)c->N * c->N;
  const double pen = 2.0 * NN * (c->n_sd + 2.0 * c->Eint) + 2.0 * c->N * c->K;
  if (L.tr) {
    // the volume rule (4N per point) and one lift per interior or Dirichlet edge
    return 2.0 * 4.0 * c->N * vol_points(c->N) * c->K + 2.0 * c->N * edge_trace_points(c->N) * c->n_sd +
           2.0 * c->N * c->K;
  }
  return 2.0 * NN * (2.0 * c->K + 2.0 * c->Eint) + pen;
}
// matrix-free apply: the divergence kernel without blocks (C own and three
// neighbours, Z not read, y written), and the block-term kernel: D own and
// three neighbours (FP64), Z^1, Z^2 own and three neighbours, C, y read and
// written, geometry; flops of the useful contraction (8 tensors, N^3 each)
double mf_div_bytes(const ldg_ctx* c, const Level& L) {
  return L.vbytes * 5.0 * c->N * c->K + 74.0 * c->K;
}
double mf_div_flops(const ldg_ctx* c) {
  const double NN = (double)c->N * c->N;
  return 2.0 * NN * (c->n_sd + 2.0 * c->Eint) + 2.0 * c->N * c->K;
}
double mf_bytes(const ldg_ctx* c, const Level& L) {
  return 8.0 * c->N * (c->K + 2.0 * c->Eint) + L.vbytes * c->N * (2.0 * c->K + 4.0 * c->Eint) +
         L.vbytes * 3.0 * c->N * c->K + 130.0 * c->K;
}
double mf_flops(const ldg_ctx* c) {
  const double N3 = (double)c->N * c->N * c->N;
  return 2.0 * N3 * (5.0 * c->K + 2.0 * c->Eint);
}
double grad_bytes(const ldg_ctx* c, const Level& L, bool with_j) {
  // geometry: |T|, B, edge lengths, normals, kind, k+, n+ (FP32 copies for the FP32 kernel);
  // quadrature form: d_h read and the flux traces written at Q points per interior edge
  // side and Dirichlet edge, the penalty rows written
  const double n_tr = c->n_sd;   // interior edge sides + Dirichlet edges
  const double geo = L.vbytes == 8.0 ? 130.0 : 74.0;
  const double tr = L.tr ? 8.0 * edge_trace_points(c->N) * n_tr + 4.0 * c->N * c->K : 0.0;
  return L.vbytes * (with_j ? 5.0 : 3.0) * c->N * c->K + geo * c->K + tr;
}
double grad_flops(const ldg_ctx* c, const Level& L) {
  const double NN = (double)c->N * c->N;
  const double tr = L.tr ? 2.0 * c->N * (2.0 + edge_trace_points(c->N)) * c->n_sd : 0.0;
  return 2.0 * NN * (2.0 * c->K + c->n_nd + 2.0 * c->Eint) + 6.0 * c->N * c->K + tr;
}

// y = M x + tau (eta S' x + sum_m B^m Z^m(x)), Z^m(x) = -M^{-1}(A^m x [+ J^m])
// y = A x; with dot, also <x, y> into red.result[0] (fused into the divergence half)
void apply_op(ldg_ctx* c, const Level& L0, double tau, const void* x, bool with_j, void* Zx1,
              void* Zx2, void* y, bool dot = false) {
  Level L = L0;
  if (c->mf) L.tr = nullptr;   // the matrix-free apply contracts every block term itself
  {
    Timed tm(c, LDG_K_GRAD, grad_bytes(c, L, with_j), grad_flops(c, L));
    launch_grad(c->N, L.vt, c->geo, c->refs, c->refs32, x, with_j ? c->J1 : nullptr, with_j ? c->J2 : nullptr,
                Zx1, Zx2, c->st, L.tr);
  }
  if (c->mf) {
    {
      Timed tm(c, LDG_K_DIV, mf_div_bytes(c, L), mf_div_flops(c));
      launch_div(c->N, L.vt, L.bt, c->geo, c->refs, nullptr, x, Zx1, Zx2, c->alpha, tau,
                 c->opt.eta, y, c->st, nullptr);
    }
    Timed tm(c, LDG_K_MF, mf_bytes(c, L), mf_flops(c));
    launch_mf_blocks(c->N, L.vt, c->geo, c->D, L.vt == VT_F64 ? (const void*)c->mf64 : c->mf32, x,
                     Zx1, Zx2, tau, y, dot ? &c->red : nullptr, c->st);
    return;
  }
  Timed tm(c, LDG_K_DIV, div_bytes(c, L), div_flops(c, L));
  launch_div(c->N, L.vt, L.bt, c->geo, c->refs, L.blocks, x, Zx1, Zx2, c->alpha, tau, c->opt.eta,
             y, c->st, dot ? &c->red : nullptr, L.tr);
}

void bj_apply(ldg_ctx* c, const Level& L, const void* r, void* z, bool dot) {
  const double NN = (double)c->N * c->N;
  const double bb = L.vt == VT_F64 ? 8.0 : 4.0;   // the preconditioner is FP32 in the mixed modes
  Timed tm(c, LDG_K_BJ_APPLY, (bb * NN + 2.0 * L.vbytes * c->N) * c->K, 2.0 * NN * c->K);
  launch_bj_apply(c->N, L.vt, L.vt == VT_F64 ? BT_F64 : BT_F32, c->geo, L.bj, r, z,
                  dot ? &c->red : nullptr, c->st);
}

void kdots(ldg_ctx* c, const Level& L, int nv, const void* V, const void* w) {
  Timed tm(c, LDG_K_KRYLOV, L.vbytes * (nv + 1) * c->nvec, 2.0 * (nv + 1) * c->nvec);
  launch_dots(L.vt, c->red, c->nvec, nv, V, c->nvec, w, c->st);
}

void kupdate(ldg_ctx* c, const Level& L, int nv, const void* V, const double* h, void* w) {
  Timed tm(c, LDG_K_KRYLOV, L.vbytes * (nv + 2) * c->nvec, 2.0 * (nv + 1) * c->nvec);
  launch_update(L.vt, c->red2, c->nvec, nv, V, c->nvec, h, w, c->st);
}

void kaxpby(ldg_ctx* c, const Level& L, double a, const void* x, double b, void* y) {
  Timed tm(c, LDG_K_KRYLOV, L.vbytes * (b == 0.0 ? 2.0 : 3.0) * c->nvec, 2.0 * c->nvec);
  launch_axpby(L.vt, c->nvec, a, x, b, y, c->st);
}

// host copy of Reducer results
ldg_status fetch(ldg_ctx* c, const double* dev, int n, double* host) {
  HIPCHK(c, hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  return LDG_OK;
}

ldg_status norm2(ldg_ctx* c, const Level& L, const void* x, double* out) {
  kdots(c, L, 0, nullptr, x);
  TRY(check_launch(c));
  return fetch(c, c->red.result, 1, out);
}

Level level64(ldg_ctx* c) {
  Level L;
  L.vt = VT_F64;
  L.bt = BT_F64;
  L.blocks = c->blocks;
  L.bj = c->bj;
  L.r = c->r; L.z = c->z; L.p = c->u; L.q = c->w; L.d = c->d64; L.u = c->u2;
  L.tz1 = c->iz1; L.tz2 = c->iz2; L.V = c->V;
  L.vbytes = 8.0;
  L.bbytes = 8.0;
  return L;
}

Level level_lo(ldg_ctx* c, int bt) {
  Level L;
  L.vt = VT_F32;
  L.bt = bt;
  L.blocks = bt == BT_BF16 ? c->blocks_bf16 : c->blocks_f32;
  L.bj = c->bj_f32;
  L.r = c->r32; L.z = c->z32; L.p = c->p32; L.q = c->q32; L.d = c->d32; L.u = c->u32;
  L.tz1 = c->tz1_32; L.tz2 = c->tz2_32; L.V = c->V32;
  L.tr = c->tr ? &c->etr : nullptr;
  L.vbytes = 4.0;
  L.bbytes = bt == BT_BF16 ? 2.0 : 4.0;
  return L;
}

// ---- inner solvers: A d = r at level L, d from zero --------------------------
// Preconditioned CG.  *not_spd is set when a curvature p^T A p <= 0 appears.
ldg_status snapshot(ldg_ctx* c, const Level& L, int it) {
  // iterate X + d of the first FP64 sweep at the requested CG iterations
  if (c->col_n == 0 || L.vt != VT_F64 || c->col_taken >= c->col_n) return LDG_OK;
  if (c->col_iters[c->col_taken] != it) return LDG_OK;
  double* snap = c->col_snap + (size_t)c->col_taken * c->nvec;
  HIPCHK(c, hipMemcpyAsync(snap, c->X, c->nvec * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  launch_axpy_into64(VT_F64, c->nvec, 1.0, L.d, snap, c->st);
  c->col_taken += 1;
  return check_launch(c);
}

void fac_apply(ldg_ctx* c, const Level& L, const void* r, void* z);

// keep: continue from the direction the previous sweep of this step left in
// L.p (with A p in L.q and <p, A p> in c->cg_kept_pq) instead of starting
// from p = P r.  The FP64 residual that replaced the iterated one is not
// orthogonal to the kept direction, so the new direction is made conjugate to
// it, p = P r - (<P r, A p_kept> / <p_kept, A p_kept>) p_kept, and the first
// step length is the minimiser along it, <r, p> / <p, A p>.  Both are free of
// the scale the refinement gives the residual.
ldg_status inner_cg(ldg_ctx* c, const Level& L, double tau, double tol_abs, int maxit, int* iters,
                    bool* not_spd, bool factor = false, bool keep = false) {
  double* hb = c->host_buf;
  *not_spd = false;
  const bool resume = keep && c->cg_kept && c->cg_kept_pq > 0.0;
  c->cg_kept = false;
  kaxpby(c, L, 0.0, L.r, 0.0, L.d);   // d = 0
  TRY(snapshot(c, L, 0));
  double r0 = 0.0, rp_old = 0.0;
  if (resume) {
    kdots(c, L, 1, L.p, L.r);   // <p_kept, r>, <r, r>
    TRY(check_launch(c));
    TRY(fetch(c, c->red.result, 2, hb));
    rp_old = hb[0];
    r0 = hb[1];
  } else {
    TRY(norm2(c, L, L.r, &r0));
  }
  r0 = std::sqrt(r0);
  double rlast = r0;
  if (factor) fac_apply(c, L, L.r, L.z);
  else bj_apply(c, L, L.r, L.z, true);
  TRY(fetch(c, c->red.result, 1, hb));
  const double rz = hb[0];
  double rp = rz;   // <r, p> of the first direction
  if (resume) {
    kdots(c, L, 1, L.q, L.z);   // <A p_kept, z>
    TRY(check_launch(c));
    TRY(fetch(c, c->red.result, 1, hb));
    const double b = -hb[0] / c->cg_kept_pq;
    kaxpby(c, L, 1.0, L.z, b, L.p);
    rp = rz + b * rp_old;
  } else {
    kaxpby(c, L, 1.0, L.z, 0.0, L.p);
  }
  // The step lengths and the coefficients of the directions stay on the
  // device (set by the epilogues of the reductions of <p, A p> and <r, z>,
  // in stream order), and the residual norm is read back only at checks: the
  // next check is placed at half the iterations the rate so far needs to
  // reach the tolerance (at most 16 ahead), so the loop syncs a few dozen
  // times per solve instead of three times per iteration and overshoots the
  // tolerance by an iteration or so.
  if (!(rz > 0.0) || !std::isfinite(rz)) {   // the preconditioner is not positive on r
    *not_spd = true;
    *iters = 0;
    c->inner_rho = 1.0;
    return LDG_OK;
  }
  launch_cg_start(c->cgs, rz, rp, c->st);
  int it = 0, next_check = 1;
  bool converged = false;
  const bool every = c->col_n > 0;   // iterate snapshots: check every iteration
  // the reductions of <p, A p> and <r, z> also set the step length and the
  // direction coefficient (Reducer::cg_mode), in the same launches
  struct CgModeReset {
    Reducer& r;
    ~CgModeReset() { r.cg = nullptr; r.cg_mode = CG_NONE; }
  } reset{c->red};
  c->red.cg = c->cgs;
  while (true) {
    c->red.cg_mode = CG_ALPHA;
    apply_op(c, L, tau, L.p, false, L.tz1, L.tz2, L.q, true);   // q = A p, <p, q>, step
    c->red.cg_mode = CG_NONE;
    const bool check = every || it + 1 >= next_check || it + 1 >= maxit;
    {
      Timed tm(c, LDG_K_KRYLOV, 6.0 * L.vbytes * c->nvec, 6.0 * c->nvec);
      launch_cg_update(L.vt, c->red2, c->nvec, 0.0, L.p, L.q, L.d, L.r, c->st,
                       c->cgs + CGS_ALPHA, check);   // x += a p, r -= a q (<r, r> at checks)
    }
    c->red.cg_mode = CG_BETA;
    if (factor) fac_apply(c, L, L.r, L.z);   // z = P r, <r, z>, direction coefficient
    else bj_apply(c, L, L.r, L.z, true);
    c->red.cg_mode = CG_NONE;
    ++it;
    TRY(snapshot(c, L, it));
    if (check) {
      HIPCHK(c, hipMemcpyAsync(hb, c->red2.result, sizeof(double), hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipMemcpyAsync(hb + 1, c->cgs, CGS_N * sizeof(double), hipMemcpyDeviceToHost,
                               c->st));
      TRY(sync(c));
      const double rn = std::sqrt(hb[0]);
      if (hb[1 + CGS_FLAG] != 0.0) {
        // a curvature or <r, z> that was not positive: the updates stopped there
        *not_spd = true;
        break;
      }
      if (!std::isfinite(rn)) return fail(c, LDG_ENOCONV, "non-finite CG residual");
      rlast = rn;
      if (rn <= tol_abs) {
        converged = true;
        c->cg_kept_pq = hb[1 + CGS_PQ];
        break;
      }
      if (it >= maxit) break;
      const double rate = std::pow(rn / r0, 1.0 / it);
      int gap = 16;
      if (rate < 1.0 && rate > 0.0) {
        const double need = std::log(tol_abs / rn) / std::log(rate);
        gap = (int)std::min(16.0, std::max(1.0, 0.5 * need));
      }
      next_check = it + gap;
    }
    {
      Timed tm(c, LDG_K_KRYLOV, 3.0 * L.vbytes * c->nvec, 2.0 * c->nvec);
      launch_xpby_dev(L.vt, c->nvec, L.z, c->cgs + CGS_BETA, L.p, c->st);   // p = z + b p
    }
  }
  *iters = (int)hb[1 + CGS_ITER];   // iterations that updated the iterate
  c->inner_rho = r0 > 0.0 ? rlast / r0 : 1.0;
  c->cg_kept = converged && it > 0;
  return LDG_OK;
}

// The GMRES basis (FP64, and FP32 in the mixed modes), the Hessenberg column
// buffers and the reduction buffers for restart length m; called between
// cycles (nothing in flight uses the old buffers after the sync).
constexpr double kGmresBasisBytes = 2.0 * 1024 * 1024 * 1024;

ldg_status krylov_buffers(ldg_ctx* c, int m) {
  const int64_t nv = c->nvec;
  const size_t nb = std::max<size_t>(c->red.nblk, gs_nblk(nv));
  size_t np = (size_t)(m + 2) * nb;
  const size_t nbj = (size_t)(c->Kpad / 64 + 1);   // per-block partials of the apply kernels
  if (np < nbj) np = nbj;
  if (np < 2048) np = 2048;
  TRY(dalloc(c, &c->V, (size_t)(m + 1) * nv));
  if (c->opt.precision != LDG_FP64) TRY(dalloc(c, &c->V32, (size_t)(m + 1) * nv));
  TRY(dalloc(c, &c->hdev, m + 2));
  TRY(dalloc(c, &c->ydev, m + 2));
  TRY(dalloc(c, &c->red.partials, np));
  TRY(dalloc(c, &c->red.result, m + 2));
  HIPCHK(c, hipHostMalloc((void**)&c->host_buf, (2 * m + 8) * sizeof(double)));
  c->red.maxv = c->red2.maxv = m + 1;
  c->mmax = m;
  return LDG_OK;
}

// largest restart length allowed by the system size and the basis budget
int gmres_cap(const ldg_ctx* c) {
  const double es = c->opt.precision == LDG_FP64 ? 8.0 : 12.0;
  const double by_mem = kGmresBasisBytes / (es * (double)c->nvec) - 1.0;
  const double by_dim = (double)c->K * c->N;
  return (int)std::max(1.0, std::min(by_mem, by_dim));
}

ldg_status grow_gmres(ldg_ctx* c, int m) {
  if (m <= c->mmax) {
    c->restart_cur = m;
    return LDG_OK;
  }
  TRY(sync(c));
  dfree(c, c->V);
  dfree(c, c->V32);
  dfree(c, c->hdev);
  dfree(c, c->ydev);
  dfree(c, c->red.partials);
  dfree(c, c->red.result);
  if (c->host_buf) (void)hipHostFree(c->host_buf);
  c->host_buf = nullptr;
  TRY(krylov_buffers(c, m));
  c->restart_cur = m;
  return LDG_OK;
}

// One cycle of right-preconditioned GMRES(m) with classical Gram-Schmidt and
// one conditional re-orthogonalisation; rnorm = ||r||.
ldg_status inner_gmres(ldg_ctx* c, const Level& L, double tau, double rnorm, double tol_abs,
                       int maxit, int* iters, bool factor = false) {
  const int64_t n = c->nvec;
  const int m = std::min(c->restart_cur, maxit);
  const size_t es = L.vt == VT_F64 ? 8 : 4;
  // Hessenberg by columns, built as the cycle runs (column j holds rows 0..j+1)
  std::vector<std::vector<double>> Hc;
  std::vector<double> cs(m), sn(m), g(m + 1, 0.0), y(m);
  double* hb = c->host_buf;
  char* V = static_cast<char*>(L.V);
  kaxpby(c, L, 1.0 / rnorm, L.r, 0.0, V);
  g[0] = rnorm;
  int jend = 0;
  for (int j = 0; j < m; ++j) {
    void* vj = V + (size_t)j * n * es;
    void* vn = V + (size_t)(j + 1) * n * es;
    if (factor) fac_apply(c, L, vj, L.z);
    else bj_apply(c, L, vj, L.z, false);
    apply_op(c, L, tau, L.z, false, L.tz1, L.tz2, vn);
    kdots(c, L, j + 1, V, vn);
    kupdate(c, L, j + 1, V, c->red.result, vn);
    TRY(check_launch(c));
    HIPCHK(c, hipMemcpyAsync(hb, c->red.result, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(hb + m + 2, c->red2.result, sizeof(double), hipMemcpyDeviceToHost, c->st));
    TRY(sync(c));
    const double wn0 = std::sqrt(hb[j + 1]);
    double wn = std::sqrt(hb[m + 2]);
    Hc.emplace_back(j + 2, 0.0);
    std::vector<double>& h = Hc.back();
    for (int i = 0; i <= j; ++i) h[i] = hb[i];
    if (wn < 0.7 * wn0) {
      kdots(c, L, j + 1, V, vn);
      kupdate(c, L, j + 1, V, c->red.result, vn);
      HIPCHK(c, hipMemcpyAsync(hb, c->red.result, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipMemcpyAsync(hb + m + 2, c->red2.result, sizeof(double), hipMemcpyDeviceToHost, c->st));
      TRY(sync(c));
      for (int i = 0; i <= j; ++i) h[i] += hb[i];
      wn = std::sqrt(hb[m + 2]);
    }
    h[j + 1] = wn;
    if (wn > 0.0) kaxpby(c, L, 1.0 / wn, vn, 0.0, vn);
    for (int i = 0; i < j; ++i) {
      const double a = h[i], b = h[i + 1];
      h[i] = cs[i] * a + sn[i] * b;
      h[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = h[j], b = h[j + 1];
    const double rr = std::hypot(a, b);
    cs[j] = rr > 0.0 ? a / rr : 1.0;
    sn[j] = rr > 0.0 ? b / rr : 0.0;
    h[j] = rr;
    h[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    jend = j + 1;
    if (!std::isfinite(g[j + 1])) return fail(c, LDG_ENOCONV, "non-finite Krylov residual");
    if (std::fabs(g[j + 1]) <= tol_abs || wn == 0.0) break;
  }
  for (int i = jend - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < jend; ++k) s -= Hc[k][i] * y[k];
    y[i] = s / Hc[i][i];
  }
  HIPCHK(c, hipMemcpyAsync(c->ydev, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, c->st));
  {
    Timed tm(c, LDG_K_KRYLOV, L.vbytes * (jend + 1) * n, 2.0 * jend * n);
    launch_lincomb(L.vt, n, jend, V, n, c->ydev, L.u, c->st);
  }
  if (factor) fac_apply(c, L, L.u, L.d);
  else bj_apply(c, L, L.u, L.d, false);
  *iters = jend;
  c->inner_rho = jend > 0 ? std::fabs(g[jend]) / rnorm : 1.0;
  c->gmres_full = jend == c->restart_cur;
  return LDG_OK;
}

// ---- graph-network preconditioner ---------------------------------------------
int64_t gnn_count(const ldg_ctx* c) {
  return c->gmode == LDG_GNN_FACTOR ? fac_num_params(c->N) : gnn_num_params(c->N);
}

int64_t gnn_count_max(const ldg_ctx* c) {
  return std::max(fac_num_params(c->N), gnn_num_params(c->N));
}

// the network and factor kernels exist for p <= 4 (N <= 15)
ldg_status gnn_order_ok(ldg_ctx* c) {
  if (c && c->p > kMaxLearnedOrder)
    return fail(c, LDG_EINVAL, "the learned preconditioner supports p <= 4");
  return LDG_OK;
}

ldg_status gnn_alloc(ldg_ctx* c, bool training) {
  const int64_t nf = c->Kpad * GNN_WIDTH;
  c->gnP = gnn_count(c);
  if (!c->gnn_alloc_inf) {
    TRY(dalloc(c, &c->gP, gnn_count_max(c)));
    TRY(dalloc(c, &c->gnode, c->Kpad * (c->N + 3)));
    TRY(dalloc(c, &c->gedge, c->Kpad * 3 * GNN_EIN));
    TRY(dalloc(c, &c->g_rhat, c->nvec));
    TRY(dalloc(c, &c->g_out, c->nvec));
    TRY(dalloc(c, &c->g_tgt, c->nvec));
    float* hb0 = nullptr;
    float* hb1 = nullptr;
    TRY(dalloc(c, &hb0, nf));
    TRY(dalloc(c, &hb1, nf));
    c->gA.h[0] = hb0; c->gA.h[1] = hb1; c->gA.h[2] = hb0; c->gA.h[3] = hb1;
    c->gnn_alloc_inf = true;
  }
  if (training && !c->gnn_alloc_train) {
    const int64_t pm = gnn_count_max(c);
    TRY(dalloc(c, &c->gGrad, pm));
    TRY(dalloc(c, &c->gM, pm));
    TRY(dalloc(c, &c->gV, pm));
    HIPCHK(c, hipMemsetAsync(c->gM, 0, pm * sizeof(float), c->st));
    HIPCHK(c, hipMemsetAsync(c->gV, 0, pm * sizeof(float), c->st));
    TRY(dalloc(c, &c->gT.z0, nf));
    for (int l = 0; l < 4; ++l) TRY(dalloc(c, &c->gT.h[l], nf));
    for (int l = 0; l < 3; ++l) {
      TRY(dalloc(c, &c->gT.a[l], nf));
      TRY(dalloc(c, &c->gT.u[l], nf));
    }
    TRY(dalloc(c, &c->gS.dh[0], nf));
    TRY(dalloc(c, &c->gS.dh[1], nf));
    TRY(dalloc(c, &c->gS.dhpart, nf));
    TRY(dalloc(c, &c->gS.da, nf));
    TRY(dalloc(c, &c->gS.rowA, (size_t)3 * c->K * std::max(2 * GNN_WIDTH + 1, FAC_HEAD)));
    TRY(dalloc(c, &c->gS.rowB, (size_t)3 * c->K * GNN_WIDTH));
    TRY(dalloc(c, &c->gS.partials, gnn_partials_size(c->K)));
    TRY(dalloc(c, &c->g_loss, (size_t)(c->Kpad / 256 + 2)));
    TRY(dalloc(c, &c->g_dout, c->nvec));
    c->gnn_alloc_train = true;
  }
  return LDG_OK;
}

ldg_status fac_alloc(ldg_ctx* c, bool training) {
  if (!c->fac_alloc_inf) {
    // sized for FP32 storage (BF16 and FP8 use less)
    const size_t per_slot = (size_t)c->Kpad * ((c->N * c->N + 3) / 4) * 4;
    float* fw = nullptr;
    float* fo = nullptr;
    TRY(dalloc(c, &fw, per_slot));
    TRY(dalloc(c, &fo, 3 * per_slot));
    // boundary edges have no O block: their entries (and the unused places of
    // the shared tail groups) stay zero
    HIPCHK(c, hipMemsetAsync(fo, 0, 3 * per_slot * sizeof(float), c->st));
    c->fac.w = fw;
    c->fac.o = fo;
    TRY(dalloc(c, &c->fac.ws, (size_t)c->Kpad));
    TRY(dalloc(c, &c->fac_w64, (size_t)c->Kpad * npairs(c->N) * 2));
    TRY(dalloc(c, &c->fac_lognorm, (size_t)3 * c->Kpad));
    TRY(dalloc(c, &c->fac_om, (size_t)3 * c->Kpad));
    TRY(dalloc(c, &c->fac_dom, (size_t)3 * c->Kpad));
    TRY(dalloc(c, &c->fac_v[0], c->nvec));
    TRY(dalloc(c, &c->fac_v[1], c->nvec));
    TRY(dalloc(c, &c->fac_y32, c->nvec));
    TRY(dalloc(c, &c->fac_a32, c->nvec));
    c->fac_alloc_inf = true;
  }
  if (training && !c->fac_alloc_train) {
    for (int q = 2; q < 8; ++q) TRY(dalloc(c, &c->fac_v[q], c->nvec));
    c->fac_alloc_train = true;
  }
  return LDG_OK;
}

// W, O blocks and log ||O|| of the current FP64 blocks and block-Jacobi inverses
// sym: build from the symmetric part of the operator (nonsymmetric steps)
ldg_status fac_build(ldg_ctx* c, double tau, bool sym = false) {
  TRY(fac_alloc(c, false));
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(int), c->st));
  {
    const double NN = (double)c->NN;
    Timed tm(c, LDG_K_FACTOR, 8.0 * NN * (8.0 * c->K), 2.0 * NN * c->N * (8.0 * c->Eint));
    launch_fac_setup(c->N, c->fac, c->geo, c->refs, c->blocks, c->bj, tau, c->opt.eta,
                     c->fac_w64, c->fac_lognorm, c->status, sym, c->st);
  }
  TRY(check_launch(c));
  HIPCHK(c, hipMemcpyAsync(c->host_buf, c->status, sizeof(int), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  int stv = 0;
  std::memcpy(&stv, c->host_buf, sizeof(int));
  if (stv) return fail(c, LDG_ENOCONV, "block-Jacobi inverse without a Cholesky factor");
  c->fac_built = true;
  return LDG_OK;
}

// omega from the network for the current context (inference activations)
ldg_status fac_omega(ldg_ctx* c) {
  Timed tm(c, LDG_K_GNN, 0.0, 0.0);
  launch_fac_omega(c->N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gA, c->fac_om,
                   c->st);
  return check_launch(c);
}

// z = P r (factored) with <r, z> in red.result[0]
void fac_apply(ldg_ctx* c, const Level& L, const void* r, void* z) {
  // W (upper triangular, N(N+1)/2 entries) read twice, the three O blocks twice
  const double NN = (double)c->N * c->N, NT = 0.5 * c->N * (c->N + 1);
  const double bw = c->fac.wt == BT_F32 ? 4.0 : (c->fac.wt == BT_BF16 ? 2.0 : 1.0);
  const double bo = c->fac.ot == BT_F32 ? 4.0 : (c->fac.ot == BT_BF16 ? 2.0 : 1.0);
  Timed tm(c, LDG_K_FACTOR, (2.0 * bw * NT + 6.0 * bo * NN + 7.0 * L.vbytes * c->N) * c->K,
           2.0 * (2.0 * NT + 6.0 * NN) * c->K);
  void* y = L.vt == VT_F64 ? (void*)c->fac_v[0] : (void*)c->fac_y32;
  void* a = L.vt == VT_F64 ? (void*)c->fac_v[1] : (void*)c->fac_a32;
  launch_fac_apply(c->N, c->fac, L.vt, c->geo, c->fac_om, r, y, a, z, &c->red, c->st);
}

// z = BJ^{-1} r + rho g(BJ^{-1} r / rho), rho = RMS of BJ^{-1} r  (FP32 network)
// z = P(r) = BJ^{-1} r + rho g(BJ^{-1} r / rho); *rz_bj = <r, BJ^{-1} r>
ldg_status gnn_precond(ldg_ctx* c, const Level& L, const void* r, void* z, double* rz_bj) {
  bj_apply(c, L, r, z, true);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  *rz_bj = c->host_buf[0];
  double nz = 0.0;
  TRY(norm2(c, L, z, &nz));
  const double rho = std::sqrt(nz / ((double)c->K * c->N));
  if (!(rho > 0.0)) return LDG_OK;
  const int64_t n = c->nvec;
  Timed tm(c, LDG_K_GNN, 0.0, 0.0);
  launch_cast(L.vt, VT_F32, n, 1.0 / rho, z, c->g_rhat, c->st);
  launch_gnn_forward(c->N, c->geo, c->gP, c->gnode, c->gedge, c->g_rhat, c->gA, c->g_out, c->st);
  if (L.vt == VT_F64)
    launch_axpy_into64(VT_F32, n, rho, c->g_out, static_cast<double*>(z), c->st);
  else
    launch_axpby(VT_F32, n, rho, c->g_out, 1.0, z, c->st);
  return check_launch(c);
}

// Flexible CG (one-step A-orthogonalisation) with the learned preconditioner;
// *broke is set to an ldg_fallback reason when it has to give up.
// An iteration whose learned direction gives <r, P r> < FCG_GUARD <r, BJ^{-1} r>
// takes the block-Jacobi direction instead (*guarded counts them).
ldg_status fcg_direction(ldg_ctx* c, const Level& L, double* rz, int* guarded) {
  constexpr double FCG_GUARD = 0.25;
  double rz_bj = 0.0;
  TRY(gnn_precond(c, L, L.r, L.z, &rz_bj));
  kdots(c, L, 1, L.r, L.z);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  *rz = c->host_buf[0];
  if (!(*rz >= FCG_GUARD * rz_bj)) {
    bj_apply(c, L, L.r, L.z, true);
    TRY(fetch(c, c->red.result, 1, c->host_buf));
    *rz = c->host_buf[0];
    *guarded += 1;
  }
  return LDG_OK;
}

ldg_status inner_fcg(ldg_ctx* c, const Level& L, double tau, double tol_abs, int maxit, int* iters,
                     int* broke, int* guarded) {
  double* hb = c->host_buf;
  *broke = LDG_FB_NONE;
  kaxpby(c, L, 0.0, L.r, 0.0, L.d);
  TRY(snapshot(c, L, 0));
  double rz = 0.0;
  TRY(fcg_direction(c, L, &rz, guarded));
  kaxpby(c, L, 1.0, L.z, 0.0, L.p);
  kdots(c, L, 0, nullptr, L.r);
  TRY(fetch(c, c->red.result, 1, hb));
  // stagnation: no new residual minimum (by 1%) within FCG_PLATEAU iterations;
  // CG residual norms oscillate, so a fixed early reduction is not asked for
  constexpr int FCG_PLATEAU = 200;
  const double r0 = std::sqrt(hb[0]);
  double rlast = r0;
  double best = r0;
  int it_best = 0;
  int it = 0;
  while (it < maxit) {
    apply_op(c, L, tau, L.p, false, L.tz1, L.tz2, L.q, true);   // q = A p, <p, q>
    TRY(fetch(c, c->red.result, 1, hb));
    const double pq = hb[0];
    if (!(pq > 0.0) || !(rz > 0.0)) {
      *broke = !(pq > 0.0) ? LDG_FB_CURVATURE : LDG_FB_RZ;
      break;
    }
    const double alpha = rz / pq;
    {
      Timed tm(c, LDG_K_KRYLOV, 6.0 * L.vbytes * c->nvec, 6.0 * c->nvec);
      launch_cg_update(L.vt, c->red2, c->nvec, alpha, L.p, L.q, L.d, L.r, c->st);
    }
    TRY(fetch(c, c->red2.result, 1, hb));
    ++it;
    TRY(snapshot(c, L, it));
    const double rn = std::sqrt(hb[0]);
    rlast = rn;
    if (rn < 0.99 * best) {
      best = rn;
      it_best = it;
    }
    if (!std::isfinite(rn)) {
      *broke = LDG_FB_NONFINITE;
      break;
    }
    if (it - it_best > FCG_PLATEAU) {
      *broke = LDG_FB_STAGNATION;
      break;
    }
    if (rn <= tol_abs) break;
    double rz_new = 0.0;
    TRY(fcg_direction(c, L, &rz_new, guarded));
    kdots(c, L, 1, L.z, L.q);
    TRY(fetch(c, c->red.result, 1, hb));
    const double beta = -hb[0] / pq;
    rz = rz_new;
    kaxpby(c, L, 1.0, L.z, beta, L.p);
  }
  *iters = it;
  c->inner_rho = r0 > 0.0 ? rlast / r0 : 1.0;
  return LDG_OK;
}

// One inner solve at level L (rnorm = ||r|| for GMRES); a breakdown moves the
// step to the next solver: learned -> block-Jacobi CG, CG -> GMRES.
ldg_status inner_solve(ldg_ctx* c, const Level& L, double tau, double tol, int left, double rnorm,
                       bool* cg_mode, bool* gnn_on, ldg_step_info* info, int* it,
                       bool keep = false) {
  *it = 0;
  if (*cg_mode && *gnn_on && c->gmode == LDG_GNN_CORRECTION) {
    int broke = LDG_FB_NONE;
    TRY(inner_fcg(c, L, tau, tol, left, it, &broke, &info->guarded_iters));
    info->learned_iters += *it;
    if (broke != LDG_FB_NONE) {   // the learned preconditioner failed: block-Jacobi from here on
      info->fallbacks += 1;
      info->fallback_reason = broke;
      *gnn_on = false;
    }
  } else if (*cg_mode) {
    const bool factor = *gnn_on;  // the factored preconditioner of this step
    bool not_spd = false;
    TRY(inner_cg(c, L, tau, tol, left, it, &not_spd, factor, keep));
    if (factor) info->learned_iters += *it;
    if (not_spd) {
      info->fallbacks += 1;
      info->fallback_reason = LDG_FB_CURVATURE;
      if (factor) {
        *gnn_on = false;
      } else {
        *cg_mode = false;
        info->krylov = LDG_KRYLOV_GMRES;
      }
    }
  }
  if (!*cg_mode && *it == 0) {
    const bool factor = *gnn_on && c->fac_on && c->gmode == LDG_GNN_FACTOR;
    TRY(inner_gmres(c, L, tau, rnorm, tol, left, it, factor));
    if (factor) info->learned_iters += *it;
  }
  return LDG_OK;
}

// ---- the step's solve: FP64 refinement around the inner solver ---------------
// Unknown C of the eliminated system, residual r = b3 - F(C) with
// F(C) = M C + tau(eta S' C + sum_m B^m Z^m(C)), Z^m(C) = -M^{-1}(A^m C + J^m_D):
// the row-3 residual of the full 3KN system, rows 1 and 2 holding exactly by
// the recovery of Z.  Each sweep: FP64 residual, inner solve A d = r at the
// working precision, C += d in FP64.  In FP64 the inner solve targets the
// final tolerance (one sweep per GMRES cycle, or a CG run confirmed by the
// true residual); in the mixed modes it targets inner_rtol relative.
ldg_status solve_step(ldg_ctx* c, double tau, double bnorm, bool use_cg, ldg_step_info* info) {
  const int64_t n = c->nvec;
  const double target = c->opt.rtol * bnorm;
  Level L64 = level64(c);
  Level L = c->opt.precision == LDG_FP64
                ? L64
                : level_lo(c, c->opt.precision == LDG_MIXED_BF16 ? BT_BF16 : BT_F32);
  double* hb = c->host_buf;
  int iters = 0, sweeps = 0;
  double beta = 0.0, beta_prev = 0.0;
  bool cg_mode = use_cg;
  c->gmres_full = false;
  c->cg_kept = false;
  // the learned preconditioner runs inside flexible CG (SPD case); for GMRES
  // problems it is not used and the step counts one fallback
  bool gnn_on = c->opt.precond == LDG_PC_GNN && cg_mode &&
                (c->gmode == LDG_GNN_CORRECTION || c->fac_on);
  // nonsymmetric steps: GMRES with the factored preconditioner of the
  // symmetric part where it was built, else block-Jacobi GMRES (a fallback)
  bool fac_gmres = c->opt.precond == LDG_PC_GNN && !cg_mode && c->fac_on &&
                   c->gmode == LDG_GNN_FACTOR;
  if (c->opt.precond == LDG_PC_GNN && !cg_mode && !fac_gmres) {
    info->fallbacks += 1;
    info->fallback_reason = LDG_FB_NONSYMMETRIC;
  }
  if (fac_gmres) gnn_on = true;
  info->krylov = cg_mode ? LDG_KRYLOV_CG : LDG_KRYLOV_GMRES;
  while (true) {
    c->stat_as = LDG_K_RESIDUAL;   // the sweep's FP64 residual, apart from the inner applies
    apply_op(c, L64, tau, c->X, true, c->tZ1, c->tZ2, c->w);
    c->stat_as = -1;
    {
      Timed tm(c, LDG_K_KRYLOV, 24.0 * n, 2.0 * n);
      launch_axpby(VT_F64, n, 1.0, c->b3, -1.0, c->w, c->st);   // w = b3 - F(X)
    }
    TRY(norm2(c, L64, c->w, hb));
    beta = std::sqrt(hb[0]);
    if (!std::isfinite(beta)) return fail(c, LDG_ENOCONV, "non-finite residual");
    if (beta <= target || iters >= c->opt.max_iters) break;
    bool escalate = L.vt != VT_F64 && sweeps > 0 && beta > 0.5 * beta_prev &&
                    beta > 4.0 * c->inner_rho * beta_prev;
    if (!cg_mode && !escalate && sweeps > 0 && beta > 0.5 * beta_prev && c->gmres_full &&
        c->inner_rho > 0.5 && 2 * c->restart_cur <= gmres_cap(c)) {
      // the last GMRES cycle ran its full length and, by its own estimate as
      // well as the FP64 residual, did not halve the residual: restarted GMRES
      // stagnates (indefinite steps), so double the restart length.  A cycle
      // whose estimate fell but whose FP64 residual did not is a precision or
      // rounding limit, not a short restart, and leaves the length alone.
      TRY(grow_gmres(c, 2 * c->restart_cur));
      // the basis and the pinned host buffer moved
      hb = c->host_buf;
      L64.V = c->V;
      L.V = L.vt == VT_F64 ? static_cast<void*>(c->V) : static_cast<void*>(c->V32);
    }
    if (escalate) {
      // refinement stagnates at this precision (the FP64 residual fell far less
      // than the inner solve reported): BF16 -> FP32 -> FP64
      c->cg_kept = false;   // the kept direction lives in the old level's vectors
      info->fallbacks += 1;
      info->fallback_reason = LDG_FB_PRECISION;
      if (L.bt == BT_BF16) {
        if (!c->blocks_f32_ready) {
          launch_convert_blocks(BT_F32, c->Kpad, c->N, NSLOT, c->blocks, c->blocks_f32, c->st);
          c->blocks_f32_ready = true;
        }
        L = level_lo(c, BT_F32);
      } else {
        L = L64;
      }
    }
    // mixed modes: CG continues from the previous sweep's direction (the FP64
    // residual replacing the iterated one) unless the options ask for a fresh
    // start.  In FP64 the residual overwrites that level's A p (L.q), and a
    // second sweep is rare there.
    const bool keep = c->opt.cg_keep_direction && sweeps > 0 && cg_mode && L.vt != VT_F64;
    beta_prev = beta;
    ++sweeps;
    int it = 0;
    double scale;
    if (L.vt == VT_F64) {
      HIPCHK(c, hipMemcpyAsync(L.r, c->w, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
      scale = 1.0;
      const int left = c->opt.max_iters - iters;
      TRY(inner_solve(c, L, tau, 0.9 * target, left, beta, &cg_mode, &gnn_on, info, &it, keep));
    } else {
      {
        Timed tm(c, LDG_K_KRYLOV, 12.0 * n, (double)n);
        launch_cast(VT_F64, VT_F32, n, 1.0 / beta, c->w, L.r, c->st);
      }
      scale = beta;
      const double tol = std::max(c->opt.inner_rtol, 0.5 * target / beta);
      const int left = c->opt.max_iters - iters;
      TRY(inner_solve(c, L, tau, tol, left, 1.0, &cg_mode, &gnn_on, info, &it, keep));
    }
    iters += it;
    {
      Timed tm(c, LDG_K_KRYLOV, (L.vbytes + 16.0) * n, 2.0 * n);
      launch_axpy_into64(L.vt, n, scale, L.d, c->X, c->st);
    }
  }
  info->iters = iters;
  info->gmres_restart = c->restart_cur;
  info->restarts = sweeps;
  info->ir_steps = c->opt.precision == LDG_FP64 ? 0 : sweeps;
  info->rel_residual = beta / bnorm;
  if (!(beta <= target)) {
    char msg[128];
    std::snprintf(msg, sizeof(msg), "solver reached %d iterations at relative residual %.3e",
                  iters, beta / bnorm);
    return fail(c, LDG_ENOCONV, msg);
  }
  return LDG_OK;
}

ldg_status assemble_lowp(ldg_ctx* c) {
  const int bt = c->opt.precision == LDG_MIXED_BF16 ? BT_BF16 : BT_F32;
  const double NN = (double)c->NN;
  {
    Timed tm(c, LDG_K_ASSEMBLE, (bt == BT_BF16 ? 2.0 : 4.0) * NN * (2.0 * c->K + 2.0 * c->Eint) +
                                    8.0 * c->N * c->K,
             2.0 * NN * c->N * (5.0 * c->K + 2.0 * c->Eint));
    launch_assemble_mfma(c->N, bt, c->geo, c->D, bt == BT_BF16 ? c->Tm16 : c->Tm32,
                         bt == BT_BF16 ? c->blocks_bf16 : c->blocks_f32, c->st);
    if (c->tr) launch_edge_d(c->N, c->geo, c->D, c->etr, c->st);
  }
  {
    Timed tm(c, LDG_K_BJ_SETUP, 12.0 * NN * c->K, 0.0);
    launch_convert_blocks(BT_F32, c->Kpad, c->N, 1, c->bj, c->bj_f32, c->st);
  }
  c->blocks_f32_ready = bt == BT_F32;
  return check_launch(c);
}

// true when D has no within-element variation (relative to its mean part)
ldg_status coefficient_is_elementwise_constant(ldg_ctx* c, bool* yes) {
  launch_mode_norms(c->N, c->geo, c->D, c->red, c->st);
  TRY(check_launch(c));
  TRY(fetch(c, c->red.result, 2, c->host_buf));
  *yes = c->host_buf[1] <= 1e-24 * c->host_buf[0];
  return LDG_OK;
}

// (r, e) pairs from the snapshots x_s of the solve just finished (x* = X):
//   e = x* - x_s, r = A e, z = BJ^{-1} r, rho = RMS(z),
//   r_hat = z / rho, target = (e - z) / rho  ->  caller buffers, element-major
ldg_status finish_collect(ldg_ctx* c, double tau) {
  const int64_t n = c->nvec;
  const Level L = level64(c);
  const int64_t KN = c->K * c->N;
  for (int s = 0; s < c->col_taken; ++s) {
    const double* snap = c->col_snap + (size_t)s * n;
    launch_axpby(VT_F64, n, -1.0, snap, 0.0, c->u2, c->st);
    launch_axpby(VT_F64, n, 1.0, c->X, 1.0, c->u2, c->st);                // e
    apply_op(c, L, tau, c->u2, false, c->iz1, c->iz2, c->w);               // r = A e
    bj_apply(c, L, c->w, c->z, false);                                     // z = BJ^{-1} r
    double nz = 0.0;
    TRY(norm2(c, L, c->z, &nz));
    const double rho = std::sqrt(nz / ((double)c->K * c->N));
    const double ir = rho > 0.0 ? 1.0 / rho : 0.0;
    launch_cast(VT_F64, VT_F32, n, ir, c->z, c->g_rhat, c->st);
    launch_axpby(VT_F64, n, -1.0, c->z, 1.0, c->u2, c->st);               // e - z
    launch_cast(VT_F64, VT_F32, n, ir, c->u2, c->g_tgt, c->st);
    launch_from_tiled_f(c->K, c->N, c->g_rhat, c->col_rhat + (size_t)s * KN, c->st);
    launch_from_tiled_f(c->K, c->N, c->g_tgt, c->col_tgt + (size_t)s * KN, c->st);
  }
  c->col_done = c->col_taken;
  c->col_n = 0;
  TRY(check_launch(c));
  return sync(c);
}

}  // namespace

namespace {
thread_local std::string g_err;   // last failure of a call without a context
ldg_status fail_noctx(ldg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace

extern "C" {

// ---- workspace of the allocation-free operator apply --------------------
// ldg_apply_schur_noalloc keeps its four tiled FP64 vectors (C, Z1, Z2, y; Kpad*N
// values each) in this fixed device array instead of the context's buffers.
// Every device the library runs on holds its own copy until the process ends.
// In host code `scratch` only names the symbol: its device address is taken
// once per device (with that device current) by noalloc_setup and kept in
// g_scratch; kernels receive that address, never the array's name.
constexpr size_t kNoAllocBytes = size_t(64) << 20;   // 64 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// called by ldg_create with the context's device current
ldg_status noalloc_setup(ldg_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, LDG_EDEVICE, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[c->device]) return LDG_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(c, LDG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[c->device] = p;
  return LDG_OK;
}

void* noalloc_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}
}  // namespace

ldg_status ldg_options_default(ldg_options* o) {
  if (!o) return LDG_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->p = 1;
  o->eta = 1.0;
  o->precision = LDG_FP64;
  o->precond = LDG_PC_BLOCK_JACOBI;
  o->rtol = 1e-8;
  o->restart = 30;
  o->max_iters = 5000;
  o->stream = nullptr;
  o->krylov = LDG_KRYLOV_AUTO;
  o->inner_rtol = 1e-3;
  o->quad = LDG_QUAD_EXACT;
  o->cg_keep_direction = 1;
  o->edge_traces = 1;
  return LDG_OK;
}

const char* ldg_last_error(const ldg_ctx* c) {
  if (c) return c->err.c_str();
  return g_err.empty() ? "null context" : g_err.c_str();
}

void ldg_destroy(ldg_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);   // teardown: nothing to report to
  for (auto& p : c->pending) { c->evpool.push_back(p.a); c->evpool.push_back(p.b); }
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->host_buf) (void)hipHostFree(c->host_buf);
  delete c;
}

ldg_status ldg_create(const double* coordV, int64_t numV, const int32_t* V0T, int64_t K,
                      const int8_t* edge_kind, const ldg_options* opt, ldg_ctx** out) {
  if (!out) return LDG_EINVAL;
  *out = nullptr;
  if (!coordV || !V0T || !edge_kind || !opt) return LDG_EINVAL;
  if (opt->p < 0 || opt->p > 6 || !(opt->eta > 0.0) || !(opt->rtol > 0.0) || opt->restart < 1 ||
      opt->restart > 200 || opt->max_iters < 1 || opt->krylov < LDG_KRYLOV_AUTO ||
      opt->krylov > LDG_KRYLOV_CG)
    return LDG_EINVAL;
  if (opt->precision < LDG_FP64 || opt->precision > LDG_MIXED_BF16) return LDG_EINVAL;
  if (opt->precision != LDG_FP64 && !(opt->inner_rtol > 0.0 && opt->inner_rtol < 1.0))
    return LDG_EINVAL;
  if (opt->precond != LDG_PC_BLOCK_JACOBI && opt->precond != LDG_PC_GNN) return LDG_EINVAL;
  if (opt->precond == LDG_PC_GNN && opt->p > kMaxLearnedOrder) return LDG_EINVAL;
  if (opt->quad != LDG_QUAD_EXACT && opt->quad != LDG_QUAD_PAPER) return LDG_EINVAL;
  if (opt->cg_keep_direction != 0 && opt->cg_keep_direction != 1) return LDG_EINVAL;
  if (opt->edge_traces != 0 && opt->edge_traces != 1) return LDG_EINVAL;
  ldg_ctx* c = new ldg_ctx();
  *out = c;
  c->opt = *opt;
  c->st = static_cast<hipStream_t>(opt->stream);
  HIPCHK(c, hipGetDevice(&c->device));
  TRY(noalloc_setup(c));
  HostMesh hm;
  bool mesh_err = false;
  const std::string msg = build_mesh(coordV, numV, V0T, K, edge_kind, hm, &mesh_err);
  if (!msg.empty()) return fail(c, mesh_err ? LDG_EMESH : LDG_EINVAL, msg);
  c->h_coordV.assign(coordV, coordV + 2 * numV);
  c->h_V0T.assign(V0T, V0T + 3 * K);
  c->ref = build_refdata(opt->p, opt->quad);
  const RefData& rf = c->ref;
  for (int i = 0; i < rf.N; ++i)
    for (int j = 0; j < rf.N; ++j)
      if (std::fabs(rf.M[i * rf.N + j] - (i == j ? 1.0 : 0.0)) > 1e-12)
        return fail(c, LDG_EINVAL, "reference mass matrix is not the identity");
  c->p = opt->p;
  c->N = rf.N;
  c->NN = rf.NN;
  c->NP = npairs(rf.N);
  c->R = rf.R;
  c->R1 = rf.R1;
  c->K = hm.K;
  c->Kpad = hm.Kpad;
  c->nbnd = (int64_t)hm.bedge_k.size();
  c->nbe = (int64_t)hm.belem.size();
  c->Eint = hm.E_int;
  c->nvec = c->Kpad * c->N;
  for (int64_t k = 0; k < 3 * K; ++k) {
    c->n_sd += edge_kind[k] != LDG_EDGE_NEUMANN;
    c->n_nd += edge_kind[k] != LDG_EDGE_DIRICHLET;
  }
  const int64_t Kp = c->Kpad;
  const int N = c->N, NN = c->NN;
  // geometry
  TRY(dalloc(c, &c->area2, Kp));
  TRY(dalloc(c, &c->B, 4 * Kp));
  TRY(dalloc(c, &c->a1, 2 * Kp));
  TRY(dalloc(c, &c->elen, 3 * Kp));
  TRY(dalloc(c, &c->nu, 6 * Kp));
  TRY(dalloc(c, &c->nbr, 3 * Kp));
  TRY(dalloc(c, &c->bidx, 3 * Kp));
  TRY(dalloc(c, &c->nbrn, 3 * Kp));
  TRY(dalloc(c, &c->kind, 3 * Kp));
  TRY(dalloc(c, &c->belem, c->nbe));
  TRY(dalloc(c, &c->bk, c->nbnd));
  TRY(dalloc(c, &c->bn, c->nbnd));
  TRY(upload(c, c->area2, hm.area2));
  TRY(upload(c, c->B, hm.B));
  TRY(upload(c, c->a1, hm.a1));
  TRY(upload(c, c->elen, hm.elen));
  TRY(upload(c, c->nu, hm.nu));
  TRY(upload(c, c->nbr, hm.nbr));
  TRY(upload(c, c->bidx, hm.bidx));
  TRY(upload(c, c->nbrn, hm.nbrn));
  TRY(upload(c, c->kind, hm.kind));
  TRY(upload(c, c->belem, hm.belem));
  TRY(upload(c, c->bk, hm.bedge_k));
  TRY(upload(c, c->bn, hm.bedge_n));
  {
    double sa = 0.0;
    for (int64_t k = 0; k < c->K; ++k) sa += 0.5 * hm.area2[k];
    c->meanA = sa / (double)c->K;
  }
  // FP32 copies of the geometry the FP32 apply kernels read (host vectors kept
  // until the create's final sync, like the mesh arrays)
  auto f32 = [](const std::vector<double>& v) {
    std::vector<float> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
    return o;
  };
  std::vector<float> ainv_h(hm.area2.size());
  for (size_t i = 0; i < ainv_h.size(); ++i)
    ainv_h[i] = hm.area2[i] != 0.0 ? (float)(-1.0 / hm.area2[i]) : 0.0f;
  const std::vector<float> B_h = f32(hm.B), elen_h = f32(hm.elen), nu_h = f32(hm.nu);
  TRY(dalloc(c, &c->ainv32, Kp));
  TRY(dalloc(c, &c->B32, 4 * Kp));
  TRY(dalloc(c, &c->elen32, 3 * Kp));
  TRY(dalloc(c, &c->nu32, 6 * Kp));
  TRY(upload(c, c->ainv32, ainv_h));
  TRY(upload(c, c->B32, B_h));
  TRY(upload(c, c->elen32, elen_h));
  TRY(upload(c, c->nu32, nu_h));
  c->geo = Geo{c->K,    c->Kpad, c->area2, c->B,    c->a1,     c->elen, c->nu,     c->nbr,
               c->nbrn, c->kind, c->bidx,  c->ainv32, c->B32, c->elen32, c->nu32};
  // reference data
  std::vector<double> refs(14 * NN);
  for (int f = 0; f < NN; ++f) {
    refs[0 * NN + f] = rf.H[0][f];
    refs[1 * NN + f] = rf.H[1][f];
    for (int n = 0; n < 3; ++n) refs[(2 + n) * NN + f] = rf.Sd[n][f];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) refs[(5 + 3 * a + b) * NN + f] = rf.So[a][b][f];
  }
  std::vector<double> Wvol(c->R * N), qv(2 * c->R), Wb(3 * c->R1 * N);
  for (int r = 0; r < c->R; ++r) {
    qv[2 * r] = rf.q1[r];
    qv[2 * r + 1] = rf.q2[r];
    for (int i = 0; i < N; ++i) Wvol[r * N + i] = rf.w[r] * phi_hat(i, rf.q1[r], rf.q2[r]);
  }
  for (int n = 0; n < 3; ++n)
    for (int r = 0; r < c->R1; ++r) {
      const double s = rf.s[r];
      double x1 = n == 0 ? 1.0 - s : (n == 1 ? 0.0 : s);
      double x2 = n == 0 ? s : (n == 1 ? 1.0 - s : 0.0);
      for (int i = 0; i < N; ++i) Wb[(n * c->R1 + r) * N + i] = phi_hat(i, x1, x2);
    }
  TRY(dalloc(c, &c->refs, refs.size()));
  TRY(dalloc(c, &c->Wvol, Wvol.size()));
  TRY(dalloc(c, &c->qvol, qv.size()));
  TRY(dalloc(c, &c->Wb, Wb.size()));
  TRY(dalloc(c, &c->ws, rf.ws.size()));
  TRY(dalloc(c, &c->sb, rf.s.size()));
  TRY(upload(c, c->refs, refs));
  {
    // FP32 gradient kernel: the 14 matrices, then the traces of the basis at the
    // p + 1 Gauss points of each reference edge, tc[n][q][j] = phi_j(x_q), and
    // lc[n][q][i] = w_q phi_i(x_q); it skips the entries of H1, H2 that vanish
    // by degree (phi_j of degree >= that of phi_i), checked here
    std::vector<float> r32(refs.begin(), refs.end());
    const int Q = c->p + 1;
    std::vector<float> tc(3 * Q * N), lc(3 * Q * N);
    for (int n = 0; n < 3; ++n)
      for (int q = 0; q < Q; ++q) {
        const double s = rf.s[q];
        const double x1 = n == 0 ? 1.0 - s : (n == 1 ? 0.0 : s);
        const double x2 = n == 0 ? s : (n == 1 ? 1.0 - s : 0.0);
        for (int i = 0; i < N; ++i) {
          const double ph = phi_hat(i, x1, x2);
          tc[(n * Q + q) * N + i] = (float)ph;
          lc[(n * Q + q) * N + i] = (float)(rf.ws[q] * ph);
        }
      }
    r32.insert(r32.end(), tc.begin(), tc.end());
    r32.insert(r32.end(), lc.begin(), lc.end());
    double hmax = 0.0, hskip = 0.0;
    for (int m = 0; m < 2; ++m)
      for (int i = 0; i < N; ++i) {
        int d = 0;
        while ((d + 1) * (d + 2) / 2 <= i) ++d;
        for (int j = 0; j < N; ++j) {
          const double v = std::fabs(rf.H[m][i * N + j]);
          hmax = std::max(hmax, v);
          if (j >= d * (d + 1) / 2) hskip = std::max(hskip, v);
        }
      }
    if (!(hskip <= 1e-12 * hmax) || (int)rf.s.size() != Q)
      return fail(c, LDG_EDEVICE, "internal: reference data do not have the assumed structure");
    TRY(dalloc(c, &c->refs32, r32.size()));
    TRY(upload(c, c->refs32, r32));
  }
  TRY(upload(c, c->Wvol, Wvol));
  TRY(upload(c, c->qvol, qv));
  TRY(upload(c, c->Wb, Wb));
  TRY(upload(c, c->ws, rf.ws));
  TRY(upload(c, c->sb, rf.s));
  {
    // tensors t = G1, G2, Rd0..2, Ro(a,b) as A operands: [t][l < LR][f] (FP64, FP32,
    // LR = mfma_lrows(N) >= N) and [t][f][l < 32] (BF16, N <= 28), zero beyond N
    // and N*N
    const int NFP = (NN + 15) / 16 * 16;
    const int LR = mfma_lrows(N);
    if (N > LR || N > 32) return fail(c, LDG_EINVAL, "order beyond the assembly tables");
    std::vector<double> T64((size_t)14 * LR * NFP, 0.0);
    std::vector<float> T32((size_t)14 * LR * NFP, 0.f);
    std::vector<uint16_t> T16((size_t)14 * NFP * 32, 0);
    auto tens = [&](int t, int l, int f) -> double {
      if (t < 2) return rf.G[t][(size_t)l * NN + f];
      if (t < 5) return rf.Rd[t - 2][(size_t)l * NN + f];
      const int ab = t - 5;
      return rf.Ro[ab / 3][ab % 3][(size_t)l * NN + f];
    };
    for (int t = 0; t < 14; ++t)
      for (int l = 0; l < N; ++l)
        for (int f = 0; f < NN; ++f) {
          const double v = tens(t, l, f);
          T64[((size_t)t * LR + l) * NFP + f] = v;
          T32[((size_t)t * LR + l) * NFP + f] = (float)v;
          T16[((size_t)t * NFP + f) * 32 + l] = host_bf16((float)v);
        }
    double* p64 = nullptr;
    float* p32 = nullptr;
    uint16_t* p16 = nullptr;
    TRY(dalloc(c, &p64, T64.size()));
    TRY(dalloc(c, &p32, T32.size()));
    TRY(dalloc(c, &p16, T16.size()));
    TRY(upload(c, p64, T64));
    TRY(upload(c, p32, T32));
    TRY(upload(c, p16, T16));
    TRY(sync(c));
    c->Tm64 = p64;
    c->Tm32 = p32;
    c->Tm16 = p16;
  }
  // state and work vectors
  const int64_t nv = c->nvec;
  double** vecs[] = {&c->C,  &c->Z1, &c->Z2, &c->D,   &c->F,   &c->J1,  &c->J2,  &c->KDN,
                     &c->b3, &c->r,  &c->w,  &c->z,   &c->u,   &c->X,   &c->tZ1, &c->tZ2,
                     &c->tmp, &c->d64, &c->u2, &c->iz1, &c->iz2};
  for (double** v : vecs) {
    TRY(dalloc(c, v, nv));
    HIPCHK(c, hipMemsetAsync(*v, 0, nv * sizeof(double), c->st));
  }
  TRY(dalloc(c, &c->blocks, (size_t)Kp * NSLOT * c->NP * 2));
  TRY(dalloc(c, &c->bj, (size_t)Kp * c->NP * 2));
  if (opt->precision != LDG_FP64) {
    float** v32[] = {&c->r32, &c->z32, &c->p32, &c->q32, &c->d32, &c->u32, &c->tz1_32, &c->tz2_32};
    for (float** v : v32) {
      TRY(dalloc(c, v, nv));
      HIPCHK(c, hipMemsetAsync(*v, 0, nv * sizeof(float), c->st));
    }
    char* p8 = nullptr;
    TRY(dalloc(c, &p8, block_bytes(BT_F32, Kp, N, NSLOT)));
    c->blocks_f32 = p8;
    TRY(dalloc(c, &p8, block_bytes(BT_F32, Kp, N, 1)));
    c->bj_f32 = p8;
    if (opt->precision == LDG_MIXED_BF16) {
      TRY(dalloc(c, &p8, block_bytes(BT_BF16, Kp, N, NSLOT)));
      HIPCHK(c, hipMemsetAsync(p8, 0, block_bytes(BT_BF16, Kp, N, NSLOT), c->st));   // tail padding
      c->blocks_bf16 = p8;
    }
    // the quadrature form of the FP32 apply: Gauss rules exact for the
    // degree-3p edge integrands and the degree-(3p-1) volume integrand, so
    // with the exact reference tensors only (the paper's rules under-integrate
    // these terms, and the stored blocks carry that)
    c->tr = opt->edge_traces && opt->quad == LDG_QUAD_EXACT;
    if (c->tr) {
      const int Q = edge_trace_points(N);
      std::vector<double> sq, wq;
      gauss_legendre(Q, sq, wq);
      std::vector<double> tr64(3 * Q * N);
      std::vector<float> tr32(3 * Q * N), lift32(3 * Q * N);
      for (int n = 0; n < 3; ++n)
        for (int q = 0; q < Q; ++q) {
          // point s_q of reference edge n (from vertex n+1 to vertex n+2)
          const double s = sq[q];
          const double x1 = n == 0 ? 1.0 - s : (n == 1 ? 0.0 : s);
          const double x2 = n == 0 ? s : (n == 1 ? 1.0 - s : 0.0);
          for (int i = 0; i < N; ++i) {
            const double ph = phi_hat(i, x1, x2);
            tr64[(n * Q + q) * N + i] = ph;
            tr32[(n * Q + q) * N + i] = (float)ph;
            lift32[(n * Q + q) * N + i] = (float)(wq[q] * ph);
          }
        }
      // volume rule: the unit square collapsed onto the triangle, Gauss-Jacobi
      // points for the weight 1 - u (the Jacobian) in u, Gauss-Legendre in v
      const int nqu = vol_points_u(N), nqv = vol_points_v(N), RV = nqu * nqv;
      std::vector<double> vol64(std::max(RV, 1) * N, 0.0);
      std::vector<float> vtab(std::max(RV, 1) * 3 * N, 0.0f);
      if (RV > 0) {
        std::vector<double> gu, gwu, gv, gwv;
        gauss_jacobi10(nqu, gu, gwu);
        gauss_legendre(nqv, gv, gwv);
        for (int a = 0; a < nqu; ++a)
          for (int b = 0; b < nqv; ++b) {
            const int q = a * nqv + b;
            const double x1 = gu[a], x2 = (1.0 - gu[a]) * gv[b];
            const double w = gwu[a] * gwv[b];
            for (int i = 0; i < N; ++i) {
              vol64[q * N + i] = w * phi_hat(i, x1, x2);
              vtab[(q * 3 + 0) * N + i] = (float)phi_hat(i, x1, x2);
              vtab[(q * 3 + 1) * N + i] = (float)dphi_hat(i, 0, x1, x2);
              vtab[(q * 3 + 2) * N + i] = (float)dphi_hat(i, 1, x1, x2);
            }
          }
      }
      float *t32 = nullptr, *l32 = nullptr, *vt32 = nullptr, *dE = nullptr, *dvol = nullptr;
      float *sig = nullptr, *pen = nullptr;
      double *t64 = nullptr, *v64 = nullptr;
      TRY(dalloc(c, &t64, tr64.size()));
      TRY(upload(c, t64, tr64));
      TRY(dalloc(c, &v64, vol64.size()));
      TRY(upload(c, v64, vol64));
      TRY(dalloc(c, &t32, tr32.size()));
      TRY(upload(c, t32, tr32));
      TRY(dalloc(c, &l32, lift32.size()));
      TRY(upload(c, l32, lift32));
      TRY(dalloc(c, &vt32, vtab.size()));
      TRY(upload(c, vt32, vtab));
      const size_t ne = (size_t)Kp * 3 * Q, nvq = (size_t)Kp * std::max(RV, 1);
      TRY(dalloc(c, &dE, ne));
      TRY(dalloc(c, &sig, ne));
      TRY(dalloc(c, &dvol, nvq));
      TRY(dalloc(c, &pen, nv));
      HIPCHK(c, hipMemsetAsync(dE, 0, ne * sizeof(float), c->st));
      HIPCHK(c, hipMemsetAsync(sig, 0, ne * sizeof(float), c->st));
      HIPCHK(c, hipMemsetAsync(dvol, 0, nvq * sizeof(float), c->st));
      HIPCHK(c, hipMemsetAsync(pen, 0, nv * sizeof(float), c->st));
      c->etr = EdgeTraces{dE, dvol, t32, l32, vt32, t64, v64, sig, pen, (float)opt->eta};
    }
  }
  TRY(dalloc(c, &c->status, 1));
  {
    // Lagrange points of Sec. 3.8: the barycentre (p = 0), the vertices
    // (p = 1), the vertices and the midpoints of the edges opposite vertices
    // 1, 2, 3 (p >= 2; for p > 2 the quadratic points, as the VTK output
    // holds at most quadratic cells)
    static const double L1[6] = {0.0, 1.0, 0.0, 0.5, 0.0, 0.5};
    static const double L2[6] = {0.0, 0.0, 1.0, 0.5, 0.5, 0.0};
    c->nL = c->N == 1 ? 1 : (c->N == 3 ? 3 : 6);
    std::vector<double> ph((size_t)c->nL * c->N);
    for (int l = 0; l < c->nL; ++l)
      for (int i = 0; i < c->N; ++i)
        ph[(size_t)l * c->N + i] = c->N == 1 ? phi_hat(i, 1.0 / 3.0, 1.0 / 3.0)
                                             : phi_hat(i, L1[l], L2[l]);
    TRY(dalloc(c, &c->phiL, ph.size()));
    TRY(upload(c, c->phiL, ph));
  }
  c->red.nblk = c->red2.nblk = krylov_nblk(nv);
  TRY(krylov_buffers(c, opt->restart));
  c->restart_cur = opt->restart;
  // red2 also takes the per-block sums of the fused CG update (one per 256 triangles)
  TRY(dalloc(c, &c->red2.partials,
             std::max<size_t>({(size_t)c->red2.nblk, (size_t)gs_nblk(nv), (size_t)(Kp / 64 + 1)}) +
                 2048));
  TRY(dalloc(c, &c->red2.result, 1));
  TRY(dalloc(c, &c->cgs, CGS_N));
  TRY(sync(c));
  c->t = 0.0;
  c->err.clear();
  return LDG_OK;
}

ldg_status ldg_get_sizes(const ldg_ctx* c, ldg_sizes* o) {
  if (!c || !o) return LDG_EINVAL;
  o->K = c->K;
  o->N = c->N;
  o->R = c->R;
  o->R1 = c->R1;
  o->n_bnd = c->nbnd;
  o->E_int = c->Eint;
  return LDG_OK;
}

ldg_status ldg_quad_points(ldg_ctx* c, int kind, double* x, double* y) {
  if (!c || !x || !y || kind < 0 || kind > 2) return fail(c, LDG_EINVAL, "bad arguments");
  if (kind == 0)
    launch_sample_vol(c->geo, c->R, c->qvol, 0, 0.0, nullptr, nullptr, nullptr, nullptr, x, y,
                      c->st);
  else
    launch_sample_bnd(c->geo, c->R1, c->sb, c->nbnd, c->bk, c->bn, kind == 2 ? -1 : 0, 0.0,
                      nullptr, nullptr, x, y, c->st);
  return check_launch(c);
}

ldg_status ldg_project(ldg_ctx* c, const double* samples, double* out) {
  if (!c || !samples || !out) return fail(c, LDG_EINVAL, "bad arguments");
  launch_project(c->N, c->K, c->Kpad, c->R, samples, c->Wvol, c->tmp, c->st);
  launch_from_tiled(c->K, c->N, c->tmp, out, c->st);
  return check_launch(c);
}

ldg_status ldg_set_state(ldg_ctx* c, const double* C, int on_device, double t) {
  if (!c || !C) return fail(c, LDG_EINVAL, "bad arguments");
  c->have_prev = false;
  const double* src = C;
  if (!on_device) {
    HIPCHK(c, hipMemcpyAsync(c->u, C, c->K * c->N * sizeof(double), hipMemcpyHostToDevice, c->st));
    src = c->u;
  }
  launch_to_tiled(c->K, c->Kpad, c->N, src, c->C, c->st);
  c->t = t;
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_set_initial_samples(ldg_ctx* c, const double* c0, double t0) {
  if (!c || !c0) return fail(c, LDG_EINVAL, "bad arguments");
  c->have_prev = false;
  launch_project(c->N, c->K, c->Kpad, c->R, c0, c->Wvol, c->C, c->st);
  c->t = t0;
  return check_launch(c);
}

namespace {
ldg_status hist_alloc(ldg_ctx* c) {
  if (!c->Cprev) {
    TRY(dalloc(c, &c->Cprev, c->nvec));
    TRY(dalloc(c, &c->Cstar, c->nvec));
  }
  return LDG_OK;
}
}  // namespace

ldg_status ldg_set_time_scheme(ldg_ctx* c, int scheme) {
  if (!c || (scheme != LDG_TIME_EULER && scheme != LDG_TIME_BDF2))
    return fail(c, LDG_EINVAL, "unknown time scheme");
  c->tscheme = scheme;
  return LDG_OK;
}

ldg_status ldg_set_history(ldg_ctx* c, const double* Cprev, double dt_prev) {
  if (!c || !Cprev || !(dt_prev > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  TRY(hist_alloc(c));
  launch_to_tiled(c->K, c->Kpad, c->N, Cprev, c->Cprev, c->st);
  c->have_prev = true;
  c->dt_prev = dt_prev;
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_get_solution(ldg_ctx* c, double* C, double* Z1, double* Z2, int on_device) {
  if (!c) return LDG_EINVAL;
  const size_t bytes = c->K * c->N * sizeof(double);
  double* srcs[3] = {c->C, c->Z1, c->Z2};
  double* dsts[3] = {C, Z1, Z2};
  for (int q = 0; q < 3; ++q) {
    if (!dsts[q]) continue;
    if (on_device) {
      launch_from_tiled(c->K, c->N, srcs[q], dsts[q], c->st);
    } else {
      launch_from_tiled(c->K, c->N, srcs[q], c->u, c->st);
      HIPCHK(c, hipMemcpyAsync(dsts[q], c->u, bytes, hipMemcpyDeviceToHost, c->st));
    }
  }
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_assemble(ldg_ctx* c, const double* Dem) {
  if (!c || !Dem) return fail(c, LDG_EINVAL, "bad arguments");
  launch_to_tiled(c->K, c->Kpad, c->N, Dem, c->D, c->st);
  launch_assemble_mfma(c->N, BT_F64, c->geo, c->D, c->Tm64, c->blocks, c->st);
  if (c->opt.precision != LDG_FP64) {
    const int bt = c->opt.precision == LDG_MIXED_BF16 ? BT_BF16 : BT_F32;
    launch_assemble_mfma(c->N, bt, c->geo, c->D, bt == BT_BF16 ? c->Tm16 : c->Tm32,
                         bt == BT_BF16 ? c->blocks_bf16 : c->blocks_f32, c->st);
    if (c->tr) launch_edge_d(c->N, c->geo, c->D, c->etr, c->st);
  }
  c->blocks_ready = true;
  return check_launch(c);
}

ldg_status ldg_get_blocks(ldg_ctx* c, double* out) {
  if (!c || !out) return fail(c, LDG_EINVAL, "bad arguments");
  launch_export_blocks(c->K, c->N, NSLOT, c->blocks, out, c->st);
  return check_launch(c);
}

ldg_status ldg_get_blocks_rows(ldg_ctx* c, const int32_t* elems, int64_t n, double* out) {
  if (!c || (n > 0 && (!elems || !out)) || n < 0) return fail(c, LDG_EINVAL, "bad arguments");
  launch_export_rows(n, elems, c->N, NSLOT, c->blocks, out, c->st);
  return check_launch(c);
}

ldg_status ldg_get_bj_rows(ldg_ctx* c, const int32_t* elems, int64_t n, double* out) {
  if (!c || (n > 0 && (!elems || !out)) || n < 0) return fail(c, LDG_EINVAL, "bad arguments");
  launch_export_rows(n, elems, c->N, 1, c->bj, out, c->st);
  return check_launch(c);
}

ldg_status ldg_get_blocks_lowp(ldg_ctx* c, double* out) {
  if (!c || !out) return fail(c, LDG_EINVAL, "bad arguments");
  if (c->opt.precision == LDG_FP64) return fail(c, LDG_EINVAL, "context has no low-precision blocks");
  const int bt = c->opt.precision == LDG_MIXED_BF16 ? BT_BF16 : BT_F32;
  launch_export_blocks_any(bt, c->K, c->N, NSLOT, bt == BT_BF16 ? c->blocks_bf16 : c->blocks_f32,
                           out, c->st);
  return check_launch(c);
}

ldg_status ldg_apply_schur(ldg_ctx* c, double dt, const double* Cem, double* y) {
  if (!c || !Cem || !y || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  if (!c->blocks_ready) return fail(c, LDG_EINVAL, "no blocks assembled");
  launch_to_tiled(c->K, c->Kpad, c->N, Cem, c->u, c->st);
  apply_op(c, level64(c), dt, c->u, false, c->tZ1, c->tZ2, c->w);
  launch_from_tiled(c->K, c->N, c->w, y, c->st);
  return check_launch(c);
}

ldg_status ldg_apply_schur_lowp(ldg_ctx* c, double dt, const double* Cem, double* y) {
  if (!c || !Cem || !y || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  if (c->opt.precision == LDG_FP64) return fail(c, LDG_EINVAL, "context has no low-precision blocks");
  if (!c->blocks_ready) return fail(c, LDG_EINVAL, "no blocks assembled");
  const Level L = level_lo(c, c->opt.precision == LDG_MIXED_BF16 ? BT_BF16 : BT_F32);
  launch_to_tiled(c->K, c->Kpad, c->N, Cem, c->u, c->st);
  launch_cast(VT_F64, VT_F32, c->nvec, 1.0, c->u, L.p, c->st);
  apply_op(c, L, dt, L.p, false, L.tz1, L.tz2, L.q);
  launch_cast(VT_F32, VT_F64, c->nvec, 1.0, L.q, c->w, c->st);
  launch_from_tiled(c->K, c->N, c->w, y, c->st);
  return check_launch(c);
}

ldg_status ldg_apply_schur_noalloc(ldg_ctx* c, double dt, const double* Cem, double* y) {
  if (!c || !Cem || !y || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  if (!c->blocks_ready) return fail(c, LDG_EINVAL, "no blocks assembled");
  const size_t need = 4 * (size_t)c->nvec * sizeof(double);
  if (need > kNoAllocBytes)
    return fail(c, LDG_EINVAL, "mesh too large for the allocation-free apply: it needs " +
                                   std::to_string(need) + " bytes of workspace, the limit is " +
                                   std::to_string(kNoAllocBytes) +
                                   " (Kpad * N <= 2097152, Kpad = K rounded up to 64)");
  double* ws = static_cast<double*>(noalloc_workspace(c->device));
  if (!ws) return fail(c, LDG_EDEVICE, "workspace address of this device not set up");
  double* u = ws;
  double* z1 = u + c->nvec;
  double* z2 = z1 + c->nvec;
  double* w = z2 + c->nvec;
  // every part of the workspace the kernels read is written first in this call
  // (padding rows included), so no clearing is needed
  launch_to_tiled(c->K, c->Kpad, c->N, Cem, u, c->st);
  launch_grad(c->N, VT_F64, c->geo, c->refs, c->refs32, u, nullptr, nullptr, z1, z2, c->st);
  if (c->mf) {
    launch_div(c->N, VT_F64, BT_F64, c->geo, c->refs, nullptr, u, z1, z2, c->alpha, dt,
               c->opt.eta, w, c->st, nullptr);
    launch_mf_blocks(c->N, VT_F64, c->geo, c->D, c->mf64, u, z1, z2, dt, w, nullptr, c->st);
  } else {
    launch_div(c->N, VT_F64, BT_F64, c->geo, c->refs, c->blocks, u, z1, z2, c->alpha, dt,
               c->opt.eta, w, c->st, nullptr);
  }
  launch_from_tiled(c->K, c->N, w, y, c->st);
  return check_launch(c);
}

ldg_status ldg_apply_full(ldg_ctx* c, double dt, const double* Y, double* out) {
  if (!c || !Y || !out || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  if (!c->blocks_ready) return fail(c, LDG_EINVAL, "no blocks assembled");
  const int64_t KN = c->K * c->N;
  launch_to_tiled(c->K, c->Kpad, c->N, Y, c->z, c->st);            // Z1
  launch_to_tiled(c->K, c->Kpad, c->N, Y + KN, c->r, c->st);       // Z2
  launch_to_tiled(c->K, c->Kpad, c->N, Y + 2 * KN, c->u, c->st);   // C
  launch_grad(c->N, VT_F64, c->geo, c->refs, c->refs32, c->u, nullptr, nullptr, c->tZ1, c->tZ2, c->st);
  launch_zrows(c->geo, c->N, c->z, c->tZ1, dt, c->w, c->st);
  launch_from_tiled(c->K, c->N, c->w, out, c->st);
  launch_zrows(c->geo, c->N, c->r, c->tZ2, dt, c->w, c->st);
  launch_from_tiled(c->K, c->N, c->w, out + KN, c->st);
  launch_div(c->N, VT_F64, BT_F64, c->geo, c->refs, c->blocks, c->u, c->z, c->r, 1.0, dt,
             c->opt.eta, c->w, c->st);
  launch_from_tiled(c->K, c->N, c->w, out + 2 * KN, c->st);
  return check_launch(c);
}

ldg_status ldg_bj_setup(ldg_ctx* c, double dt) {
  if (!c || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  if (!c->blocks_ready) return fail(c, LDG_EINVAL, "no blocks assembled");
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(int), c->st));
  {
    const double NN = (double)c->NN;
    Timed tm(c, LDG_K_BJ_SETUP, 8.0 * NN * (3.0 * c->K + 2.0 * c->Eint),
             2.0 * NN * c->N * (11.0 * c->K + 2.0 * c->Eint));
    launch_bj_setup(c->N, c->geo, c->refs, c->blocks, c->alpha, dt, c->opt.eta, c->bj, c->status,
                    c->st);
  }
  TRY(check_launch(c));
  int st = 0;
  HIPCHK(c, hipMemcpyAsync(c->host_buf, c->status, sizeof(int), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  std::memcpy(&st, c->host_buf, sizeof(int));
  if (st) return fail(c, LDG_ENOCONV, "zero pivot in a block-Jacobi block");
  return LDG_OK;
}

ldg_status ldg_get_bj(ldg_ctx* c, double* out) {
  if (!c || !out) return fail(c, LDG_EINVAL, "bad arguments");
  launch_export_blocks(c->K, c->N, 1, c->bj, out, c->st);
  return check_launch(c);
}

}  // extern "C"

namespace {

// One linear system of the method at sampled data, solved for C into X from X0:
//   alpha M C + tau (eta S' C + sum_m B^m Z^m(C)) = alpha M Chist + tau (K_D,N + M F)
//                                                   + tau sum_m B^m M^{-1} J^m,
// alpha = 1: an implicit Euler or BDF2 step (Chist its history); alpha = 0,
// tau = 1: the stationary system A Y = V (no history, Chist unused).
ldg_status solve_sampled(ldg_ctx* c, double alpha, double tau, const double* Chist,
                         const double* X0, const double* d, const double* f, const double* cD,
                         const double* gN, ldg_step_info* info) {
  struct Scope {   // the mass coefficient holds for this system only
    ldg_ctx* c;
    ~Scope() { c->alpha = 1.0; }
  } scope{c};
  c->alpha = alpha;
  const int64_t n = c->nvec;
  // a1: projections and boundary data
  {
    Timed tm(c, LDG_K_PROJECT, 2.0 * 8.0 * (c->R + c->N) * c->K,
             2.0 * 2.0 * c->R * c->N * (double)c->K);
    launch_project(c->N, c->K, c->Kpad, c->R, d, c->Wvol, c->D, c->st);
    launch_project(c->N, c->K, c->Kpad, c->R, f, c->Wvol, c->F, c->st);
    launch_boundary(c->N, c->geo, c->nbe, c->belem, c->R1, c->Wb, c->ws, cD, gN, c->nbnd, c->D,
                    c->opt.eta, c->J1, c->J2, c->KDN, c->st);
  }
  if (c->opt.precond == LDG_PC_GNN) {
    if (!c->gnn_params_set) return fail(c, LDG_EINVAL, "learned preconditioner without parameters");
    launch_gnn_features(c->N, c->geo, c->D, tau, c->opt.eta, c->meanA, c->gnode, c->gedge, c->st);
  }
  // a2, a3: D-dependent blocks
  {
    const double NN = (double)c->NN;
    Timed tm(c, LDG_K_ASSEMBLE, 8.0 * NN * (2.0 * c->K + 2.0 * c->Eint) + 8.0 * c->N * c->K,
             2.0 * NN * c->N * (5.0 * c->K + 2.0 * c->Eint));
    launch_assemble_mfma(c->N, BT_F64, c->geo, c->D, c->Tm64, c->blocks, c->st);
  }
  c->blocks_ready = true;
  TRY(check_launch(c));
  // a4: preconditioner
  TRY(ldg_bj_setup(c, tau));
  // right-hand side and its full-system norm
  launch_rhs(c->geo, c->N, alpha != 0.0 ? Chist : nullptr, c->KDN, c->F, tau, c->b3, c->st);
  double nb3 = 0.0, nj1 = 0.0, nj2 = 0.0;
  TRY(norm2(c, level64(c), c->b3, &nb3));
  TRY(norm2(c, level64(c), c->J1, &nj1));
  TRY(norm2(c, level64(c), c->J2, &nj2));
  const double bnorm = std::sqrt(nb3 + tau * tau * (nj1 + nj2));
  // the inner solves of the mixed modes: blocks contracted at FP32 or BF16 on
  // the matrix cores, FP32 copy of the block-Jacobi inverses
  if (c->opt.precision != LDG_FP64) TRY(assemble_lowp(c));
  // a6, a7: Krylov solve (with FP64 refinement)
  bool use_cg = c->opt.krylov == LDG_KRYLOV_CG;
  if (c->opt.krylov == LDG_KRYLOV_AUTO) TRY(coefficient_is_elementwise_constant(c, &use_cg));
  // the factored learned preconditioner of this system (SPD case only)
  c->fac_on = false;
  if (c->opt.precond == LDG_PC_GNN && c->gmode == LDG_GNN_FACTOR) {
    if (use_cg) {
      TRY(fac_build(c, tau));
      TRY(fac_omega(c));
      c->fac_on = true;
    } else if (fac_build(c, tau, true) == LDG_OK) {
      // nonsymmetric step: the factored preconditioner of the operator's
      // symmetric part, a fixed SPD right preconditioner for GMRES
      TRY(fac_omega(c));
      c->fac_on = true;
    } else {
      c->err.clear();   // no Cholesky factor of the symmetric part: block-Jacobi GMRES
    }
  }
  if (X0)
    HIPCHK(c, hipMemcpyAsync(c->X, X0, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  else
    HIPCHK(c, hipMemsetAsync(c->X, 0, n * sizeof(double), c->st));
  c->col_taken = 0;
  ldg_status s = solve_step(c, tau, bnorm > 0.0 ? bnorm : 1.0, use_cg, info);
  info->t = c->t;
  if (s != LDG_OK) {
    c->col_n = 0;
    return s;
  }
  if (c->col_n > 0) TRY(finish_collect(c, tau));
  return LDG_OK;
}

// accept X as the state; Z from the last residual evaluation of X
ldg_status accept_solution(ldg_ctx* c) {
  const int64_t n = c->nvec;
  HIPCHK(c, hipMemcpyAsync(c->C, c->X, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->Z1, c->tZ1, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->Z2, c->tZ2, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  return LDG_OK;
}

}  // namespace

extern "C" {

ldg_status ldg_step_sampled(ldg_ctx* c, double dt, const double* d, const double* f,
                            const double* cD, const double* gN, ldg_step_info* info) {
  if (!c || !d || !f || !info || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  std::memset(info, 0, sizeof(*info));
  TRY(hist_alloc(c));
  // BDF2 needs the previous state at the same step size; else implicit Euler
  const bool bdf2 = c->tscheme == LDG_TIME_BDF2 && c->have_prev &&
                    std::fabs(dt - c->dt_prev) <= 1e-12 * dt;
  const double tau = bdf2 ? 2.0 * dt / 3.0 : dt;
  info->bdf_order = bdf2 ? 2 : 1;
  const int64_t n = c->nvec;
  // the history the step starts from: C^n, or (4 C^n - C^{n-1}) / 3 for BDF2
  const double* Chist = c->C;
  if (bdf2) {
    launch_axpby(VT_F64, n, 4.0 / 3.0, c->C, 0.0, c->Cstar, c->st);
    launch_axpby(VT_F64, n, -1.0 / 3.0, c->Cprev, 1.0, c->Cstar, c->st);
    Chist = c->Cstar;
  }
  // the Krylov solve starts from C^n
  TRY(solve_sampled(c, 1.0, tau, Chist, c->C, d, f, cD, gN, info));
  // a10: accept; C^n becomes the history
  HIPCHK(c, hipMemcpyAsync(c->Cprev, c->C, n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  c->have_prev = true;
  c->dt_prev = dt;
  TRY(accept_solution(c));
  c->t += dt;
  info->t = c->t;
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_solve_stationary_sampled(ldg_ctx* c, const double* d, const double* f,
                                        const double* cD, const double* gN,
                                        ldg_step_info* info) {
  if (!c || !d || !f || !info) return fail(c, LDG_EINVAL, "bad arguments");
  std::memset(info, 0, sizeof(*info));
  // without a Dirichlet edge the stationary operator has the constants in its kernel
  if (3 * c->K - c->n_nd == 0)
    return fail(c, LDG_EINVAL, "stationary solve needs at least one Dirichlet edge");
  TRY(solve_sampled(c, 0.0, 1.0, nullptr, nullptr, d, f, cD, gN, info));
  TRY(accept_solution(c));
  // the stationary state has no previous step: a following BDF2 step starts with Euler
  c->have_prev = false;
  info->bdf_order = 0;
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_gnn_num_params(ldg_ctx* c, int64_t* n) {
  TRY(gnn_order_ok(c));
  if (!c || !n) return LDG_EINVAL;
  *n = gnn_count(c);
  return LDG_OK;
}

ldg_status ldg_gnn_set_params(ldg_ctx* c, const float* w, int64_t n) {
  TRY(gnn_order_ok(c));
  if (!c || !w || n != gnn_count(c)) return fail(c, LDG_EINVAL, "parameter count");
  TRY(gnn_alloc(c, false));
  HIPCHK(c, hipMemcpyAsync(c->gP, w, n * sizeof(float), hipMemcpyHostToDevice, c->st));
  if (c->gnn_alloc_train) {
    HIPCHK(c, hipMemsetAsync(c->gM, 0, n * sizeof(float), c->st));
    HIPCHK(c, hipMemsetAsync(c->gV, 0, n * sizeof(float), c->st));
  }
  c->gstep = 0;
  c->gnn_params_set = true;
  return sync(c);
}

ldg_status ldg_gnn_get_params(ldg_ctx* c, float* w, int64_t n) {
  TRY(gnn_order_ok(c));
  if (!c || !w || n != gnn_count(c) || !c->gnn_params_set)
    return fail(c, LDG_EINVAL, "parameter count or no parameters");
  HIPCHK(c, hipMemcpyAsync(w, c->gP, n * sizeof(float), hipMemcpyDeviceToHost, c->st));
  return sync(c);
}

ldg_status ldg_gnn_set_context(ldg_ctx* c, const double* Dem, double dt) {
  TRY(gnn_order_ok(c));
  if (!c || !(dt > 0.0)) return fail(c, LDG_EINVAL, "bad arguments");
  TRY(gnn_alloc(c, false));
  if (Dem) launch_to_tiled(c->K, c->Kpad, c->N, Dem, c->D, c->st);
  launch_gnn_features(c->N, c->geo, c->D, dt, c->opt.eta, c->meanA, c->gnode, c->gedge, c->st);
  if (c->gmode == LDG_GNN_FACTOR) {
    // the factored preconditioner of this system: blocks, block-Jacobi, W and O
    bool sym = false;
    TRY(coefficient_is_elementwise_constant(c, &sym));
    if (!sym) return fail(c, LDG_EINVAL, "the factored preconditioner needs a coefficient "
                                         "constant per triangle");
    launch_assemble_mfma(c->N, BT_F64, c->geo, c->D, c->Tm64, c->blocks, c->st);
    c->blocks_ready = true;
    TRY(ldg_bj_setup(c, dt));
    TRY(fac_build(c, dt));
    c->gtau = dt;
    c->g_energy_ready = true;
  } else if (c->gloss == LDG_GNN_LOSS_ENERGY) {
    // the energy gradient 2 S (g - t) / (t^T S t) needs S symmetric: d constant per triangle
    bool sym = false;
    TRY(coefficient_is_elementwise_constant(c, &sym));
    if (!sym) return fail(c, LDG_EINVAL, "energy loss needs a coefficient constant per triangle");
    launch_assemble_mfma(c->N, BT_F64, c->geo, c->D, c->Tm64, c->blocks, c->st);
    c->blocks_ready = true;
    c->gtau = dt;
    c->g_energy_ready = true;
  }
  return check_launch(c);
}

ldg_status ldg_gnn_set_mode(ldg_ctx* c, int mode) {
  TRY(gnn_order_ok(c));
  if (!c || (mode != LDG_GNN_CORRECTION && mode != LDG_GNN_FACTOR))
    return fail(c, LDG_EINVAL, "unknown network mode");
  if (mode != c->gmode) {
    c->gmode = mode;
    c->gnn_params_set = false;
    c->g_energy_ready = false;
    c->gnP = gnn_count(c);
  }
  return LDG_OK;
}

ldg_status ldg_gnn_factor_storage(ldg_ctx* c, int bt) {
  TRY(gnn_order_ok(c));
  if (!c || (bt != LDG_FAC_F32 && bt != LDG_FAC_BF16 && bt != LDG_FAC_FP8 && bt != LDG_FAC_FP8W))
    return fail(c, LDG_EINVAL,
                "factor storage is LDG_FAC_F32, LDG_FAC_BF16, LDG_FAC_FP8 or LDG_FAC_FP8W");
  c->fac.wt = bt == LDG_FAC_F32 ? BT_F32 : (bt == LDG_FAC_FP8W ? BT_FP8 : BT_BF16);
  c->fac.ot = bt == LDG_FAC_F32 ? BT_F32 : (bt == LDG_FAC_BF16 ? BT_BF16 : BT_FP8);
  c->g_energy_ready = false;   // blocks of the old storage are stale
  c->fac_built = false;
  return LDG_OK;
}

ldg_status ldg_gnn_factor_omega(ldg_ctx* c, float* om) {
  if (!c || !om || c->gmode != LDG_GNN_FACTOR || !c->gnn_params_set || !c->fac_built)
    return fail(c, LDG_EINVAL, "factor mode, parameters and built factor blocks are needed");
  TRY(fac_omega(c));
  for (int n = 0; n < 3; ++n)
    HIPCHK(c, hipMemcpy2DAsync(om + n, 3 * sizeof(float), c->fac_om + n * c->Kpad, sizeof(float),
                               sizeof(float), c->K, hipMemcpyDeviceToDevice, c->st));
  return sync(c);
}

ldg_status ldg_gnn_factor_export(ldg_ctx* c, double* blocks, float* lognorm) {
  if (!c || c->gmode != LDG_GNN_FACTOR || !c->fac_built)
    return fail(c, LDG_EINVAL, "factor mode and built factor blocks are needed");
  if (blocks) launch_fac_export(c->K, c->N, c->fac, blocks, c->st);
  if (lognorm)
    for (int n = 0; n < 3; ++n)
      HIPCHK(c, hipMemcpy2DAsync(lognorm + n, 3 * sizeof(float), c->fac_lognorm + n * c->Kpad,
                                 sizeof(float), sizeof(float), c->K, hipMemcpyDeviceToDevice,
                                 c->st));
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_gnn_factor_export_rows(ldg_ctx* c, const int32_t* elems, int64_t n, double* blocks,
                                      float* lognorm) {
  if (!c || !elems || n < 0 || !blocks || c->gmode != LDG_GNN_FACTOR || !c->fac_built)
    return fail(c, LDG_EINVAL, "factor mode with built factor blocks and a row list are needed");
  if (n == 0) return LDG_OK;
  // indices come to the host and are checked against K before a launch reads through them
  std::vector<int32_t> h(n);
  HIPCHK(c, hipMemcpyAsync(h.data(), elems, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  for (int32_t k : h)
    if (k < 0 || k >= c->K) return fail(c, LDG_EINVAL, "row index out of range");
  launch_fac_export_rows(n, elems, c->N, c->fac, c->Kpad, c->fac_lognorm, blocks, lognorm, c->st);
  TRY(check_launch(c));
  return sync(c);
}

ldg_status ldg_gnn_set_loss(ldg_ctx* c, int loss) {
  TRY(gnn_order_ok(c));
  if (!c || (loss != LDG_GNN_LOSS_MSE && loss != LDG_GNN_LOSS_ENERGY &&
             loss != LDG_GNN_LOSS_FROBENIUS && loss != LDG_GNN_LOSS_OPTSTEP))
    return fail(c, LDG_EINVAL, "unknown loss");
  if (loss == LDG_GNN_LOSS_OPTSTEP && c->gmode != LDG_GNN_FACTOR)
    return fail(c, LDG_EINVAL, "the optimal-step loss is defined for the factored network");
  c->gloss = loss;
  c->g_energy_ready = false;
  return LDG_OK;
}

ldg_status ldg_gnn_forward(ldg_ctx* c, const float* rhat, float* out) {
  TRY(gnn_order_ok(c));
  if (!c || !rhat || !out || !c->gnn_params_set) return fail(c, LDG_EINVAL, "bad arguments");
  if (c->gmode != LDG_GNN_CORRECTION)
    return fail(c, LDG_EINVAL, "the factored network maps no residual: ldg_gnn_factor_omega");
  launch_to_tiled_f(c->K, c->Kpad, c->N, rhat, c->g_rhat, c->st);
  {
    Timed tm(c, LDG_K_GNN, 0.0, 0.0);
    launch_gnn_forward(c->N, c->geo, c->gP, c->gnode, c->gedge, c->g_rhat, c->gA, c->g_out, c->st);
  }
  launch_from_tiled_f(c->K, c->N, c->g_out, out, c->st);
  return check_launch(c);
}

namespace {
// Energy loss  L = (g - t)^T S (g - t) / (t^T S t)  with S the eliminated
// operator of the context (symmetric in the case the learned preconditioner
// serves), so dL/dg = 2 S (g - t) / (t^T S t).  FP64 vectors r, z, w, u are free
// outside a step.
ldg_status gnn_energy_dout(ldg_ctx* c, double* loss) {
  if (!c->g_energy_ready)
    return fail(c, LDG_EINVAL, "energy loss needs ldg_gnn_set_context after ldg_gnn_set_loss");
  const Level L = level64(c);
  const int64_t n = c->nvec;
  launch_cast(VT_F32, VT_F64, n, 1.0, c->g_out, c->r, c->st);
  launch_axpy_into64(VT_F32, n, -1.0, c->g_tgt, c->r, c->st);
  launch_cast(VT_F32, VT_F64, n, 1.0, c->g_tgt, c->z, c->st);
  apply_op(c, L, c->gtau, c->r, false, L.tz1, L.tz2, c->w);
  apply_op(c, L, c->gtau, c->z, false, L.tz1, L.tz2, c->u);
  double num = 0.0, den = 0.0;
  kdots(c, L, 1, c->r, c->w);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  num = c->host_buf[0];
  kdots(c, L, 1, c->z, c->u);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  den = c->host_buf[0];
  if (!(den > 0.0) || !std::isfinite(num))
    return fail(c, LDG_ENOCONV, "energy loss: target has no positive energy");
  launch_cast(VT_F64, VT_F32, n, 2.0 / den, c->w, c->g_dout, c->st);
  *loss = num / den;
  return LDG_OK;
}

// Factored preconditioner, energy loss of one pair: e = target + rhat, r = S e,
//   d = P r - e,  d0 = BJ^{-1} r - e,  loss = d^T S d / d0^T S d0,
// and d loss / d omega from y = W r, a = (I + F) y, beta = W (2 S d / den),
// alpha = (I + F) beta.
ldg_status gnn_factor_loss_grad(ldg_ctx* c, double* loss) {
  if (!c->g_energy_ready) return fail(c, LDG_EINVAL, "no context set");
  TRY(fac_alloc(c, true));
  const Level L = level64(c);
  const int64_t n = c->nvec;
  const int N = c->N;
  double** v = c->fac_v;
  launch_fac_omega(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT, c->fac_om, c->st);
  launch_cast(VT_F32, VT_F64, n, 1.0, c->g_tgt, v[0], c->st);
  launch_axpy_into64(VT_F32, n, 1.0, c->g_rhat, v[0], c->st);            // e
  apply_op(c, L, c->gtau, v[0], false, L.tz1, L.tz2, v[1]);               // r = S e
  launch_fac_w(N, c->fac, c->geo, v[1], v[2], c->st);                 // y
  launch_fac_f(N, c->fac, c->geo, c->fac_om, false, v[2], v[3], c->st);  // a
  launch_fac_f(N, c->fac, c->geo, c->fac_om, true, v[3], v[4], c->st);   // z = P r
  launch_axpy_into64(VT_F64, n, -1.0, v[0], v[4], c->st);                 // d
  apply_op(c, L, c->gtau, v[4], false, L.tz1, L.tz2, v[5]);               // S d
  kdots(c, L, 1, v[4], v[5]);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  const double num = c->host_buf[0];
  bj_apply(c, L, v[1], v[6], false);
  launch_axpy_into64(VT_F64, n, -1.0, v[0], v[6], c->st);                 // d0
  apply_op(c, L, c->gtau, v[6], false, L.tz1, L.tz2, v[7]);               // S d0
  kdots(c, L, 1, v[6], v[7]);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  const double den = c->host_buf[0];
  if (!(den > 0.0) || !std::isfinite(num))
    return fail(c, LDG_ENOCONV, "energy loss: block-Jacobi error without positive energy");
  launch_cast(VT_F64, VT_F64, n, 2.0 / den, v[5], v[4], c->st);           // dL/dz
  launch_fac_w(N, c->fac, c->geo, v[4], v[6], c->st);                 // beta
  launch_fac_f(N, c->fac, c->geo, c->fac_om, false, v[6], v[7], c->st);  // alpha
  launch_fac_domega(N, c->fac, c->geo, v[3], v[6], v[7], v[2], c->fac_dom, c->st);
  launch_fac_omega_backward(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT,
                            c->fac_om, c->fac_dom, c->gS, c->gGrad, c->st);
  *loss = num / den;
  return check_launch(c);
}

// Factored preconditioner, optimal-step loss of a pair (rhat, target), e = target + rhat:
//   loss = min_t ||e - t P r||_S^2 / ||e||_S^2 = 1 - s^2 / (q c),
//   r = S e, z = P r, s = <r, z>, q = <z, S z>, c = <e, r>;
//   d loss / dz = -2 s / (q c) r + 2 s^2 / (q^2 c) S z, then the chain of the energy loss.
ldg_status gnn_factor_optstep_grad(ldg_ctx* c, double* loss) {
  if (!c->g_energy_ready) return fail(c, LDG_EINVAL, "no context set");
  TRY(fac_alloc(c, true));
  const Level L = level64(c);
  const int64_t n = c->nvec;
  const int N = c->N;
  double** v = c->fac_v;
  double* hb = c->host_buf;
  launch_fac_omega(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT, c->fac_om, c->st);
  launch_cast(VT_F32, VT_F64, n, 1.0, c->g_tgt, v[0], c->st);
  launch_axpy_into64(VT_F32, n, 1.0, c->g_rhat, v[0], c->st);            // e
  apply_op(c, L, c->gtau, v[0], false, L.tz1, L.tz2, v[1]);               // r = S e
  launch_fac_w(N, c->fac, c->geo, v[1], v[2], c->st);                 // y
  launch_fac_f(N, c->fac, c->geo, c->fac_om, false, v[2], v[3], c->st);  // a
  launch_fac_f(N, c->fac, c->geo, c->fac_om, true, v[3], v[4], c->st);   // z = P r
  apply_op(c, L, c->gtau, v[4], false, L.tz1, L.tz2, v[5]);               // S z
  double sv = 0.0, q = 0.0, cv = 0.0;
  kdots(c, L, 1, v[1], v[4]);
  TRY(fetch(c, c->red.result, 1, hb));
  sv = hb[0];
  kdots(c, L, 1, v[4], v[5]);
  TRY(fetch(c, c->red.result, 1, hb));
  q = hb[0];
  kdots(c, L, 1, v[0], v[1]);
  TRY(fetch(c, c->red.result, 1, hb));
  cv = hb[0];
  if (!(q > 0.0) || !(cv > 0.0) || !std::isfinite(sv))
    return fail(c, LDG_ENOCONV, "optimal-step loss: an error or direction without positive energy");
  launch_axpby(VT_F64, n, -2.0 * sv / (q * cv), v[1], 0.0, v[4], c->st);  // dL/dz
  launch_axpby(VT_F64, n, 2.0 * sv * sv / (q * q * cv), v[5], 1.0, v[4], c->st);
  launch_fac_w(N, c->fac, c->geo, v[4], v[6], c->st);                 // beta
  launch_fac_f(N, c->fac, c->geo, c->fac_om, false, v[6], v[7], c->st);  // alpha
  launch_fac_domega(N, c->fac, c->geo, v[3], v[6], v[7], v[2], c->fac_dom, c->st);
  launch_fac_omega_backward(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT,
                            c->fac_om, c->fac_dom, c->gS, c->gGrad, c->st);
  *loss = 1.0 - sv * sv / (q * cv);
  return check_launch(c);
}

// Factored preconditioner, Frobenius loss for a probe w (the rhat input):
//   loss = ||(G S G^T - I) w||^2 / ||(W S W^T - I) w||^2,  G = (I + F) W;
// with u = G^T w, y = W S u, g = 2 ((I + F) y - w) / den and
// beta = W S W^T (I + F)^T g:  d loss / d F_kj = g_k y_j^T + w_k beta_j^T.
ldg_status gnn_factor_frob_grad(ldg_ctx* c, double* loss) {
  if (!c->g_energy_ready) return fail(c, LDG_EINVAL, "no context set");
  TRY(fac_alloc(c, true));
  const Level L = level64(c);
  const int64_t n = c->nvec;
  const int N = c->N;
  double** v = c->fac_v;
  launch_fac_omega(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT, c->fac_om, c->st);
  launch_cast(VT_F32, VT_F64, n, 1.0, c->g_rhat, v[0], c->st);                // w
  launch_fac_f(N, c->fac, c->geo, c->fac_om, true, v[0], v[1], c->st);     // u = G^T w
  apply_op(c, L, c->gtau, v[1], false, L.tz1, L.tz2, v[2]);                    // S u
  launch_fac_w(N, c->fac, c->geo, v[2], v[3], c->st);                      // y
  launch_fac_f(N, c->fac, c->geo, c->fac_om, false, v[3], v[4], c->st);    // (I + F) y
  launch_axpy_into64(VT_F64, n, -1.0, v[0], v[4], c->st);                      // residual
  kdots(c, L, 1, v[4], v[4]);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  const double num = c->host_buf[0];
  launch_fac_wt(N, c->fac, c->geo, v[0], v[5], c->st);                     // W^T w
  apply_op(c, L, c->gtau, v[5], false, L.tz1, L.tz2, v[6]);
  launch_fac_w(N, c->fac, c->geo, v[6], v[5], c->st);
  launch_axpy_into64(VT_F64, n, -1.0, v[0], v[5], c->st);                      // (W S W^T - I) w
  kdots(c, L, 1, v[5], v[5]);
  TRY(fetch(c, c->red.result, 1, c->host_buf));
  const double den = c->host_buf[0];
  if (!(den > 0.0) || !std::isfinite(num))
    return fail(c, LDG_ENOCONV, "Frobenius loss: zero probe or non-finite value");
  launch_cast(VT_F64, VT_F64, n, 2.0 / den, v[4], v[5], c->st);                // g
  launch_fac_f(N, c->fac, c->geo, c->fac_om, true, v[5], v[6], c->st);     // G^T g
  apply_op(c, L, c->gtau, v[6], false, L.tz1, L.tz2, v[7]);
  launch_fac_w(N, c->fac, c->geo, v[7], v[6], c->st);                      // beta
  launch_fac_domega(N, c->fac, c->geo, v[0], v[6], v[5], v[3], c->fac_dom, c->st);
  launch_fac_omega_backward(N, c->geo, c->gP, c->gnode, c->gedge, c->fac_lognorm, c->gT,
                            c->fac_om, c->fac_dom, c->gS, c->gGrad, c->st);
  *loss = num / den;
  return check_launch(c);
}

ldg_status gnn_loss_grad_tiled(ldg_ctx* c, double* loss) {
  if (c->gmode == LDG_GNN_FACTOR) {
    if (c->gloss == LDG_GNN_LOSS_FROBENIUS) return gnn_factor_frob_grad(c, loss);
    if (c->gloss == LDG_GNN_LOSS_OPTSTEP) return gnn_factor_optstep_grad(c, loss);
    return gnn_factor_loss_grad(c, loss);
  }
  Timed tm(c, LDG_K_GNN, 0.0, 0.0);
  launch_gnn_forward(c->N, c->geo, c->gP, c->gnode, c->gedge, c->g_rhat, c->gT, c->g_out, c->st);
  if (c->gloss == LDG_GNN_LOSS_ENERGY) {
    TRY(gnn_energy_dout(c, loss));
    launch_gnn_backward(c->N, c->geo, c->gP, c->gnode, c->gedge, c->g_rhat, c->g_tgt, c->g_dout,
                        c->gT, c->g_out, c->gS, c->gGrad, c->g_loss, c->st);
    return check_launch(c);
  }
  launch_gnn_backward(c->N, c->geo, c->gP, c->gnode, c->gedge, c->g_rhat, c->g_tgt, nullptr, c->gT,
                      c->g_out, c->gS, c->gGrad, c->g_loss, c->st);
  const int nb = (int)((c->Kpad + 255) / 256);
  reduce_partials(nb, c->g_loss, c->g_loss + nb, c->st);
  TRY(check_launch(c));
  TRY(fetch(c, c->g_loss + nb, 1, c->host_buf));
  *loss = c->host_buf[0] / ((double)c->K * c->N);
  return LDG_OK;
}
}  // namespace

ldg_status ldg_gnn_loss_grad(ldg_ctx* c, const float* rhat, const float* target, float* grad,
                             double* loss) {
  TRY(gnn_order_ok(c));
  if (!c || !rhat || !target || !loss || !c->gnn_params_set)
    return fail(c, LDG_EINVAL, "bad arguments");
  TRY(gnn_alloc(c, true));
  launch_to_tiled_f(c->K, c->Kpad, c->N, rhat, c->g_rhat, c->st);
  launch_to_tiled_f(c->K, c->Kpad, c->N, target, c->g_tgt, c->st);
  TRY(gnn_loss_grad_tiled(c, loss));
  if (grad)
    HIPCHK(c, hipMemcpyAsync(grad, c->gGrad, c->gnP * sizeof(float), hipMemcpyDeviceToDevice, c->st));
  return sync(c);
}

ldg_status ldg_gnn_train_step(ldg_ctx* c, const float* rhat, const float* target, double lr,
                              double* loss) {
  TRY(gnn_order_ok(c));
  if (!c || !rhat || !target || !loss || !c->gnn_params_set || !(lr > 0.0))
    return fail(c, LDG_EINVAL, "bad arguments");
  TRY(gnn_alloc(c, true));
  launch_to_tiled_f(c->K, c->Kpad, c->N, rhat, c->g_rhat, c->st);
  launch_to_tiled_f(c->K, c->Kpad, c->N, target, c->g_tgt, c->st);
  TRY(gnn_loss_grad_tiled(c, loss));
  c->gstep += 1;
  launch_adam(c->gnP, c->gP, c->gGrad, c->gM, c->gV, (float)lr, c->gstep, c->st);
  return check_launch(c);
}

ldg_status ldg_gnn_collect(ldg_ctx* c, int nsnap, const int32_t* iters, float* rhat_out,
                           float* target_out) {
  TRY(gnn_order_ok(c));
  if (!c || nsnap < 1 || nsnap > 64 || !iters || !rhat_out || !target_out)
    return fail(c, LDG_EINVAL, "bad arguments");
  for (int s = 0; s < nsnap; ++s)
    if (iters[s] < 0 || (s > 0 && iters[s] <= iters[s - 1]))
      return fail(c, LDG_EINVAL, "snapshot iterations must increase");
  TRY(gnn_alloc(c, false));
  if (c->col_cap < nsnap) {   // snapshot slots are kept until the context is destroyed
    double* p = nullptr;
    TRY(dalloc(c, &p, (size_t)nsnap * c->nvec));
    c->col_snap = p;
    c->col_cap = nsnap;
  }
  c->col_iters.assign(iters, iters + nsnap);
  c->col_n = nsnap;
  c->col_done = 0;
  c->col_rhat = rhat_out;
  c->col_tgt = target_out;
  return LDG_OK;
}

ldg_status ldg_gnn_collected(ldg_ctx* c, int* n) {
  if (!c || !n) return LDG_EINVAL;
  *n = c->col_done;
  return LDG_OK;
}

ldg_status ldg_set_timing(ldg_ctx* c, int on) {
  if (!c) return LDG_EINVAL;
  TRY(sync(c));
  c->timing = on != 0;
  for (auto& s : c->stats) s = ldg_kernel_stat{};
  return LDG_OK;
}

ldg_status ldg_set_matrix_free(ldg_ctx* c, int on) {
  if (!c) return LDG_EINVAL;
  if (on && c->p > kMaxLearnedOrder) return fail(c, LDG_EINVAL, "the matrix-free apply supports p <= 4");
  if (on && !c->mf64) {
    // A-operand tables of the 14 tensors (G1, G2, Rd0..2, Ro(n, n+)), FP64 and FP32
    const RefData& rf = c->ref;
    const double* tens[14] = {rf.G[0].data(), rf.G[1].data(), rf.Rd[0].data(), rf.Rd[1].data(),
                              rf.Rd[2].data()};
    for (int ab = 0; ab < 9; ++ab) tens[5 + ab] = rf.Ro[ab / 3][ab % 3].data();
    std::vector<double> t64((size_t)mf_table_size(c->N));
    mf_build_table(c->N, tens, t64.data());
    std::vector<float> t32(t64.begin(), t64.end());
    double* p64 = nullptr;
    float* p32 = nullptr;
    TRY(dalloc(c, &p64, t64.size()));
    TRY(dalloc(c, &p32, t32.size()));
    TRY(upload(c, p64, t64));
    TRY(upload(c, p32, t32));
    TRY(sync(c));
    c->mf64 = p64;
    c->mf32 = p32;
  }
  c->mf = on != 0;
  return LDG_OK;
}

ldg_status ldg_get_kernel_stat(ldg_ctx* c, int kernel, ldg_kernel_stat* out) {
  if (!c || !out || kernel < 0 || kernel >= LDG_K_COUNT) return fail(c, LDG_EINVAL, "bad arguments");
  TRY(sync(c));
  *out = c->stats[kernel];
  return LDG_OK;
}

ldg_status ldg_lagrange(ldg_ctx* c, const double* C, double* out, int* nL) {
  if (!c || !nL) return c ? fail(c, LDG_EINVAL, "bad arguments") : LDG_EINVAL;
  *nL = c->nL;
  if (!out) return LDG_OK;
  launch_lagrange(c->K, c->N, c->nL, C ? C : c->C, C == nullptr, c->phiL, out, c->st);
  return check_launch(c);
}

ldg_status ldg_write_vtu(ldg_ctx* c, const char* path, const char* name, const double* lagr,
                         int nL, int binary) {
  if (!c || !path || !name || !lagr) return c ? fail(c, LDG_EINVAL, "bad arguments") : LDG_EINVAL;
  if (nL != c->nL) return fail(c, LDG_EINVAL, "Lagrange values per triangle do not match p");
  for (const char* q = name; *q; ++q)
    if (*q == '"' || *q == '<' || *q == '>' || *q == '&')
      return fail(c, LDG_EINVAL, "the variable name holds an XML special character");
  const std::string msg = write_vtu(path, name, c->h_coordV, c->h_V0T, c->K, nL, lagr, binary != 0);
  if (!msg.empty()) return fail(c, LDG_EIO, msg);
  return LDG_OK;
}

ldg_status ldg_mesh_read_medit(const char* path, int64_t* numV, int64_t* K, double* coordV,
                               int32_t* V0T, int32_t* edge_id) {
  if (!path || !numV || !K) return fail_noctx(LDG_EINVAL, "bad arguments");
  std::vector<double> cv;
  std::vector<int32_t> vt, ids;
  const std::string msg = read_medit(path, cv, vt, ids);
  if (!msg.empty()) return fail_noctx(msg.rfind("cannot open", 0) == 0 ? LDG_EIO : LDG_EMESH, msg);
  const bool want = coordV || V0T || edge_id;
  if (want && (*numV != (int64_t)cv.size() / 2 || *K != (int64_t)vt.size() / 3))
    return fail_noctx(LDG_EINVAL, "buffer sizes differ from the file's");
  *numV = (int64_t)cv.size() / 2;
  *K = (int64_t)vt.size() / 3;
  if (coordV) std::memcpy(coordV, cv.data(), cv.size() * sizeof(double));
  if (V0T) std::memcpy(V0T, vt.data(), vt.size() * sizeof(int32_t));
  if (edge_id) std::memcpy(edge_id, ids.data(), ids.size() * sizeof(int32_t));
  return LDG_OK;
}

ldg_status ldg_edge_kinds_from_ids(int64_t K, const int32_t* edge_id, const int32_t* neumann_ids,
                                   int n_neumann, int8_t* edge_kind) {
  if (K < 0 || !edge_id || !edge_kind || n_neumann < 0 || (n_neumann > 0 && !neumann_ids))
    return fail_noctx(LDG_EINVAL, "bad arguments");
  for (int64_t e = 0; e < 3 * K; ++e) {
    const int32_t id = edge_id[e];
    if (id < 0) return fail_noctx(LDG_EMESH, "a boundary edge has no ID");
    int8_t k = id == 0 ? LDG_EDGE_INTERIOR : LDG_EDGE_DIRICHLET;
    for (int q = 0; q < n_neumann && id > 0; ++q)
      if (neumann_ids[q] == id) k = LDG_EDGE_NEUMANN;
    edge_kind[e] = k;
  }
  return LDG_OK;
}

}  // extern "C"

namespace {

// the sample points on the host and the device sample buffers of the callbacks
ldg_status cb_alloc(ldg_ctx* c) {
  if (c->cb_d) return LDG_OK;
  const int64_t nv = (int64_t)c->R * c->K, nb = (int64_t)c->R1 * c->nbnd;
  double *px = nullptr, *py = nullptr;
  TRY(dalloc(c, &px, std::max<int64_t>(nv, nb)));
  TRY(dalloc(c, &py, std::max<int64_t>(nv, nb)));
  auto fetch_pts = [&](int kind, int64_t n, std::vector<double>& hx, std::vector<double>& hy) {
    hx.resize(n);
    hy.resize(n);
    if (n == 0) return LDG_OK;
    ldg_status st = ldg_quad_points(c, kind, px, py);
    if (st != LDG_OK) return st;
    HIPCHK(c, hipMemcpyAsync(hx.data(), px, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(hy.data(), py, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
    return sync(c);
  };
  TRY(fetch_pts(0, nv, c->cb_x, c->cb_y));
  TRY(fetch_pts(1, nb, c->cb_bx, c->cb_by));
  TRY(fetch_pts(2, nb, c->cb_nx, c->cb_ny));
  TRY(dalloc(c, &c->cb_d, std::max<int64_t>(nv, 1)));
  TRY(dalloc(c, &c->cb_f, std::max<int64_t>(nv, 1)));
  TRY(dalloc(c, &c->cb_c0, std::max<int64_t>(nv, 1)));
  TRY(dalloc(c, &c->cb_cD, std::max<int64_t>(nb, 1)));
  TRY(dalloc(c, &c->cb_gN, std::max<int64_t>(nb, 1)));
  return LDG_OK;
}

// evaluate one field on the host and copy it to the device buffer dst
ldg_status cb_eval(ldg_ctx* c, const char* name, ldg_field_fn fn, ldg_flux_fn flux, void* user,
                   double t, bool boundary, double* dst) {
  const std::vector<double>& x = boundary ? c->cb_bx : c->cb_x;
  const std::vector<double>& y = boundary ? c->cb_by : c->cb_y;
  const int64_t n = (int64_t)x.size();
  std::vector<double> out(n, 0.0);
  const int rc = fn ? fn(user, t, x.data(), y.data(), out.data(), n)
                    : flux(user, t, x.data(), y.data(), c->cb_nx.data(), c->cb_ny.data(),
                           out.data(), n);
  if (rc != 0)
    return fail(c, LDG_ECALLBACK, std::string("field callback ") + name + " returned " +
                                      std::to_string(rc));
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(out[i]))
      return fail(c, LDG_ECALLBACK, std::string("field callback ") + name +
                                        " produced a non-finite value");
  if (n > 0)
    HIPCHK(c, hipMemcpyAsync(dst, out.data(), n * sizeof(double), hipMemcpyHostToDevice, c->st));
  return sync(c);   // the host buffer ends here
}

}  // namespace

extern "C" {

ldg_status ldg_set_initial(ldg_ctx* c, ldg_field_fn c0, void* user) {
  if (!c || !c0) return fail(c, LDG_EINVAL, "bad arguments");
  TRY(cb_alloc(c));
  TRY(cb_eval(c, "c0", c0, nullptr, user, 0.0, false, c->cb_c0));
  return ldg_set_initial_samples(c, c->cb_c0, 0.0);
}

ldg_status ldg_step(ldg_ctx* c, double dt, const ldg_problem* pb, ldg_step_info* info) {
  if (!c || !pb || !info || !(dt > 0.0) || !pb->d || !pb->f)
    return fail(c, LDG_EINVAL, "bad arguments");
  const bool has_dir = 3 * c->K - c->n_nd > 0, has_neu = 3 * c->K - c->n_sd > 0;
  if ((has_dir && !pb->c_D) || (has_neu && !pb->g_N))
    return fail(c, LDG_EINVAL, "the mesh has Dirichlet (Neumann) edges but no c_D (g_N)");
  TRY(cb_alloc(c));
  const double t = c->t + dt;   // data at the new time level (Sec. 2.5)
  TRY(cb_eval(c, "d", pb->d, nullptr, pb->user, t, false, c->cb_d));
  TRY(cb_eval(c, "f", pb->f, nullptr, pb->user, t, false, c->cb_f));
  if (has_dir) TRY(cb_eval(c, "c_D", pb->c_D, nullptr, pb->user, t, true, c->cb_cD));
  if (has_neu) TRY(cb_eval(c, "g_N", nullptr, pb->g_N, pb->user, t, true, c->cb_gN));
  return ldg_step_sampled(c, dt, c->cb_d, c->cb_f, has_dir ? c->cb_cD : nullptr,
                          has_neu ? c->cb_gN : nullptr, info);
}

ldg_status ldg_set_initial_dofs(ldg_ctx* c, const double* C, int on_device) {
  return ldg_set_state(c, C, on_device, 0.0);
}

ldg_status ldg_gnn_load(ldg_ctx* c, const float* w, int64_t n) { return ldg_gnn_set_params(c, w, n); }

ldg_status ldg_gnn_save(ldg_ctx* c, float* w, int64_t n) { return ldg_gnn_get_params(c, w, n); }

ldg_status ldg_sample_workload(ldg_ctx* c, int kind, double t, const double* dT, double* d,
                               double* f, double* cD, double* gN, double* c0) {
  if (!c || kind < 1 || kind > 6) return fail(c, LDG_EINVAL, "bad workload kind");
  if ((kind == 3 || kind == 4) && !dT) return fail(c, LDG_EINVAL, "block field needs dT");
  if (d || f || c0)
    launch_sample_vol(c->geo, c->R, c->qvol, kind, t, dT, d, f, c0, nullptr, nullptr, c->st);
  if (cD || gN)
    launch_sample_bnd(c->geo, c->R1, c->sb, c->nbnd, c->bk, c->bn, kind, t, cD, gN, nullptr,
                      nullptr, c->st);
  return check_launch(c);
}

}  // extern "C"
