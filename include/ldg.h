/*
 * ldg.h -- C ABI of the MI355X (gfx950) LDG diffusion hot path.
 *
 * Method: local discontinuous Galerkin discretisation of the 2D diffusion
 * equation  dt c - div(d grad c) = f  with Dirichlet/Neumann data (Sec. 1.3,
 * eq:diffusion:nonmixed) in the mixed form z = -grad c (Sec. 2.2), modal
 * orthonormal bases of order p = 0..6 (Sec. 2.4.1: the paper's functions up
 * to p = 4, beyond that orthonormal collapsed-coordinate polynomials by
 * recursion, the alternative to Gram-Schmidt that Sec. 2.4.1 names), the
 * global block system
 * eq:timeDepSystem and one implicit Euler step per call (eq:fullSystem):
 *     (W + dt A(t+dt)) Y = W Y^n + dt V(t+dt),   Y = [Z1; Z2; C],
 * or a two-step backward differentiation step, or the stationary system
 * A Y = V of Sec. 3.7.  The linear system is solved on the system for C
 * obtained by eliminating Z (M is block diagonal, M_k = 2|T_k| I, eq:hatM):
 * preconditioned CG where that system is symmetric positive definite,
 * right-preconditioned restarted GMRES otherwise, with block-Jacobi or a
 * learned graph-network preconditioner, in FP64 or in FP32/BF16 with FP64
 * iterative refinement, stopping on the relative residual of the full 3KN
 * system.
 *
 * Conventions
 *   - Element k, basis index i (0-based): vectors are "element-major",
 *     value (k, i) at k*N + i, N = (p+1)(p+2)/2.  Outputs keep the caller's
 *     element order.
 *   - Local edge n of triangle k joins its local vertices n+1 and n+2 (mod 3)
 *     (edge n lies opposite vertex n, Fig. 3 and eq:gammaMap).
 *   - Triangles must be counter-clockwise (det B_k = 2|T_k| > 0, Sec. 3.2).
 *   - "device" pointers are HIP device memory on the context's device; "host"
 *     pointers are ordinary CPU memory.  The caller owns every pointer it
 *     passes; the library never keeps or frees caller memory after a call.
 *   - All device work is enqueued on options.stream (a hipStream_t, NULL =
 *     the default stream).  Calls that return numbers to the host
 *     synchronise that stream.
 *   - Every entry point returns an ldg_status; nothing throws or aborts
 *     across the ABI.  ldg_last_error() describes the last failure of a
 *     context.
 */
#ifndef LDG_H
#define LDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldg_ctx ldg_ctx; /* opaque, owned by the library */

typedef enum {
  LDG_OK = 0,
  LDG_EINVAL = -1,    /* bad argument: NULL pointer, p outside 0..6, eta <= 0, dt <= 0, ... */
  LDG_EMESH = -2,     /* orientation, conformity or edge kinds inconsistent */
  LDG_ENOMEM = -3,    /* device allocation failed */
  LDG_EDEVICE = -4,   /* a HIP call failed */
  LDG_ENOCONV = -5,   /* the solver did not reach rtol; the state is not advanced */
  LDG_EUNSUPPORTED = -6,
  LDG_EIO = -7,       /* a file could not be opened, read or written */
  LDG_ECALLBACK = -8  /* a field callback returned non-zero or a non-finite value */
} ldg_status;

/*
 * LDG_FP64: everything in FP64.  Mixed modes: the state, the residual of the
 * full system and the refinement correction stay FP64; each refinement
 * sweep solves A d = r with FP32 vectors (FP64 inner products), the stored
 * blocks in FP32 or BF16 and FP32 arithmetic, and a FP32 block-Jacobi.  A
 * sweep that fails to halve the FP64 residual although the inner solve
 * reported a reduction at least four times larger (the low-precision operator,
 * not the Krylov method, limits progress) moves the inner solve one precision
 * up (BF16 -> FP32 -> FP64), counted in ldg_step_info.fallbacks.  With GMRES
 * one sweep is one restart cycle.
 */
typedef enum { LDG_FP64 = 0, LDG_MIXED_FP32 = 1, LDG_MIXED_BF16 = 2 } ldg_precision;
typedef enum { LDG_PC_BLOCK_JACOBI = 0, LDG_PC_GNN = 1 } ldg_precond;
typedef enum { LDG_EDGE_INTERIOR = 0, LDG_EDGE_DIRICHLET = 1, LDG_EDGE_NEUMANN = 2 } ldg_edge_kind;
/*
 * Krylov method of a step.  With a coefficient that is constant on every
 * triangle (only the first mode of D non-zero) the blocks satisfy
 * B^m = -(A^m)^T diag(d) and the eliminated operator is symmetric positive
 * definite, so LDG_KRYLOV_AUTO uses preconditioned conjugate gradients;
 * otherwise (or if CG breaks down) restarted GMRES.
 */
typedef enum { LDG_KRYLOV_AUTO = 0, LDG_KRYLOV_GMRES = 1, LDG_KRYLOV_CG = 2 } ldg_krylov;
/*
 * Quadrature of the reference tensors (Sec. 3.6).  LDG_QUAD_EXACT: every
 * polynomial integrand integrated exactly (the plain definition of the
 * tensors).  LDG_QUAD_PAPER: the paper's routines' rules, order max(2p, 1) on
 * the triangle and 2p + 1 on the edges, below the degree 3p of the
 * three-factor integrands of G_hat and R_hat for p >= 2 (identical for p <= 1).
 * The projection and boundary-data rules are the paper's in both.
 */
typedef enum { LDG_QUAD_EXACT = 0, LDG_QUAD_PAPER = 1 } ldg_quad_policy;

typedef struct {
  int p;              /* polynomial order 0..6; the paper's routines stop at 4 (assert in
                         the main script), and so do the learned preconditioner and the
                         matrix-free apply (LDG_EINVAL for p = 5, 6 with either) */
  double eta;         /* penalty eta > 0 (prob:semidiscrete), default 1 */
  int precision;      /* ldg_precision, default LDG_FP64 */
  int precond;        /* ldg_precond, default LDG_PC_BLOCK_JACOBI */
  double rtol;        /* relative residual of the full system, default 1e-8; FP64 rounding
                         bounds what is reachable near 1e-16 ||A|| ||Y|| / ||V|| */
  int restart;        /* GMRES restart length m in 1..200, default 30.  A GMRES cycle
                         that runs all m iterations and halves neither its own residual
                         estimate nor the FP64 residual doubles m for the rest of the
                         context's life, while 2m stays within the system size K N and
                         the basis within 2 GiB (indefinite steps, where restarted GMRES
                         stalls; on large meshes the bound keeps m fixed) */
  int max_iters;      /* total Krylov iterations per step, default 5000 */
  void* stream;       /* hipStream_t for all device work */
  int krylov;         /* ldg_krylov, default LDG_KRYLOV_AUTO */
  double inner_rtol;  /* mixed modes: relative tolerance of each inner solve, default 1e-3 */
  int quad;           /* ldg_quad_policy of the reference tensors, default LDG_QUAD_EXACT */
  int cg_keep_direction; /* mixed modes, CG steps.  1 (default): each refinement sweep
                         after the first continues from the last search direction of the
                         sweep before, the FP64 residual replacing the iterated one (as in
                         reliable-update CG); the first new direction is made conjugate to
                         the kept one, and its step length minimises along it.  0: every
                         sweep starts CG afresh from p = P r.  GMRES sweeps always
                         restart, and so does FP64 CG */
  int edge_traces;    /* mixed modes with LDG_QUAD_EXACT.  1 (default): the FP32 apply of
                         the inner solves in quadrature form, with no stored blocks read:
                         the volume terms of B^m (eq:hatG) from d_h at the points of a
                         collapsed Gauss rule exact for their degree 3p-1, its edge terms
                         (eq:hatRdiag, eq:hatRoffdiag) from the traces of d_h nu.Z_h at
                         ceil((3p+1)/2) Gauss points per edge (exact for degree 3p),
                         which the gradient half writes and the neighbours read.  0: the
                         five stored FP32 or BF16 blocks.  Ignored in FP64, with
                         LDG_QUAD_PAPER and in the matrix-free apply */
} ldg_options;

typedef struct {
  int64_t K;          /* triangles */
  int N;              /* local basis functions */
  int R;              /* volume quadrature points per triangle (projection rule, order max(2p,1)) */
  int R1;             /* Gauss points per boundary edge (order 2p+1) */
  int64_t n_bnd;      /* boundary edges */
  int64_t E_int;      /* interior edges */
} ldg_sizes;

typedef struct {
  int iters;           /* Krylov iterations of the step (inner ones in the mixed modes) */
  int restarts;        /* GMRES cycles */
  int ir_steps;        /* outer refinement sweeps (mixed modes), 0 in FP64 */
  int fallbacks;       /* fallbacks taken (CG -> GMRES, learned -> block-Jacobi) */
  int krylov;          /* ldg_krylov actually used by the step */
  double rel_residual; /* ||b - (W + dt A) Y|| / ||b|| of the full system, FP64 */
  double t;            /* time level reached */
  int learned_iters;   /* iterations run with the learned preconditioner */
  int guarded_iters;   /* of those, iterations that took the block-Jacobi direction
                          because <r, P r> < 0.25 <r, BJ^{-1} r> */
  int fallback_reason; /* ldg_fallback of the last fallback taken */
  int bdf_order;       /* 1: implicit Euler step, 2: two-step backward differentiation */
  int gmres_restart;   /* GMRES restart length after the step (see ldg_options.restart) */
} ldg_step_info;

/*
 * Why a step left its first solver: a curvature p^T A p <= 0 (CG, flexible
 * CG), <r, P r> <= 0 with the learned preconditioner, a non-finite residual,
 * no new residual minimum (by 1%) within 200 flexible-CG iterations, a
 * nonsymmetric step the learned preconditioner does not serve (the residual
 * correction network, or a factored preconditioner whose symmetric part has
 * no Cholesky factor), or a mixed
 * sweep that failed to halve the residual while the inner solve reported a
 * four times larger reduction.
 */
typedef enum {
  LDG_FB_NONE = 0, LDG_FB_CURVATURE = 1, LDG_FB_RZ = 2, LDG_FB_NONFINITE = 3,
  LDG_FB_STAGNATION = 4, LDG_FB_NONSYMMETRIC = 5, LDG_FB_PRECISION = 6
} ldg_fallback;

/* Fill *opt with the defaults listed above. */
ldg_status ldg_options_default(ldg_options* opt);

/*
 * Build a context from a triangulation (Sec. 3.1, Table 1).
 *   coordV    host, numV x 2 vertex coordinates
 *   V0T       host, K x 3 counter-clockwise vertex indices, 0-based
 *   edge_kind host, K x 3 ldg_edge_kind per local edge
 * Computes the grid lists and the reference tensors once (convention 1 of
 * Sec. 3: stationary data is computed only once), uploads them and
 * allocates every device buffer the steps need.  The state starts at t = 0
 * with C = 0.  Errors: EINVAL, EMESH (non-positive area, an edge shared by
 * more than two triangles or traversed twice in one direction, a kind that
 * disagrees with the topology), ENOMEM, EDEVICE.
 */
ldg_status ldg_create(const double* coordV, int64_t numV, const int32_t* V0T, int64_t K,
                      const int8_t* edge_kind, const ldg_options* opt, ldg_ctx** out);
void ldg_destroy(ldg_ctx* ctx);
const char* ldg_last_error(const ldg_ctx* ctx);
ldg_status ldg_get_sizes(const ldg_ctx* ctx, ldg_sizes* out);

/*
 * Physical coordinates of the points where the caller samples its data: the
 * points F_k(q_r) of the quadrature rule that the L2 projection of Sec. 3.4
 * applies on every triangle (order max(2p, 1), the rule the main script of
 * Sec. 4 projects with), and the Gauss points of the boundary edges that the
 * boundary integrals of Sec. 3.6.9-3.6.11 use (J_D, K_D, K_N).
 *   kind 0: volume points of the projection rule, layout [R][K]
 *           (point r of triangle k at r*K + k);
 *   kind 1: Gauss points of the boundary edges, layout [R1][n_bnd], the
 *           boundary edges ordered by (triangle, local edge);
 *   kind 2: (boundary only) exterior unit normal at those points.
 * x, y: device, caller-allocated with the sizes above.
 */
ldg_status ldg_quad_points(ldg_ctx* ctx, int kind, double* x, double* y);

/*
 * L2 projection (Sec. 3.4): out = samples * (w o phi_hat) M_hat^{-1}, one
 * N-vector per triangle.  samples: device [R][K] values of a function at
 * the kind-0 points; out: device K x N, element-major.
 */
ldg_status ldg_project(ldg_ctx* ctx, const double* samples, double* out);

/* Set the state: C (K x N, element-major) and the time level t. */
ldg_status ldg_set_state(ldg_ctx* ctx, const double* C, int on_device, double t);
/* Initial state as the L2 projection of c0 sampled at the kind-0 points. */
ldg_status ldg_set_initial_samples(ldg_ctx* ctx, const double* c0_samples, double t0);

/*
 * One implicit Euler step t -> t + dt (eq:fullSystem, data at t + dt):
 *   d, f    device [R][K]     diffusion coefficient and source at the kind-0 points
 *   cD, gN  device [R1][n_bnd] Dirichlet / Neumann data at the kind-1 points
 *           (values on edges of the other kind are ignored; gN may be NULL
 *           when there is no Neumann edge, cD when there is no Dirichlet edge)
 * Runs projection, block assembly, preconditioner setup, the Krylov solve
 * and the recovery of Z on the device.  On LDG_ENOCONV the state is left
 * unchanged and *info describes the failed solve.
 */
ldg_status ldg_step_sampled(ldg_ctx* ctx, double dt, const double* d, const double* f,
                            const double* cD, const double* gN, ldg_step_info* info);

/*
 * The stationary system A Y = V (eq:fullSystem without the W term; the
 * verification setting of Sec. 3.7, Table 2), with the same data arguments
 * as ldg_step_sampled (sampled at whatever time the caller chooses).  Solved
 * through the same eliminated operator with the mass term dropped,
 *   eta S' C + sum_m B^m Z^m(C) = K_D,N + M F + sum_m B^m M^{-1} J^m,
 * by the same Krylov solver, preconditioner and precision options, starting
 * from C = 0.  The solution becomes the state (C, Z1, Z2); the time level is
 * unchanged and the BDF2 history is cleared.  info->bdf_order is 0.  A mesh
 * with no Dirichlet edge (the operator then has the constants in its
 * kernel): LDG_EINVAL before any launch.  On LDG_ENOCONV the state is left
 * unchanged.
 */
ldg_status ldg_solve_stationary_sampled(ldg_ctx* ctx, const double* d, const double* f,
                                        const double* cD, const double* gN, ldg_step_info* info);

/*
 * Time scheme of the steps.  LDG_TIME_EULER (default): the implicit Euler step
 * of Sec. 2.5.  LDG_TIME_BDF2: the second-order two-step backward
 * differentiation formula with the same space discretisation,
 *   W (3/2 Y^{n+1} - 2 Y^n + 1/2 Y^{n-1}) / dt + A^{n+1} Y^{n+1} = V^{n+1},
 * solved as (W + tau A) Y^{n+1} = W Y* + tau V with tau = 2 dt / 3 and
 * C* = (4 C^n - C^{n-1}) / 3 (W has zero Z rows).  It needs the previous state
 * at the same dt: every step keeps its starting state; ldg_set_state and
 * ldg_set_initial_samples clear it, ldg_set_history sets it (device K x N,
 * element-major, with its step size).  Without it, or after a change of dt,
 * a step is implicit Euler (ldg_step_info.bdf_order says which).
 * Unknown schemes: LDG_EINVAL.
 */
typedef enum { LDG_TIME_EULER = 0, LDG_TIME_BDF2 = 1 } ldg_time_scheme;
ldg_status ldg_set_time_scheme(ldg_ctx* ctx, int scheme);
ldg_status ldg_set_history(ldg_ctx* ctx, const double* C_prev, double dt_prev);

/*
 * Current solution: the three blocks of Y = [Z1; Z2; C], the unknown vector
 * of eq:fullSystem (Sec. 2.5), each block ordered as eq:timeDepSystem orders
 * it, degree of freedom j of triangle k at k*N + j (index (k-1)N + j of the
 * paper), in the caller's element order and in the basis of Sec. 2.4.1.
 * C, Z1, Z2: K x N FP64 each, device (on_device = 1) or host, caller-owned;
 * any may be NULL.  LDG_EINVAL for a NULL context.
 */
ldg_status ldg_get_solution(ldg_ctx* ctx, double* C, double* Z1, double* Z2, int on_device);

/*
 * Kernel timing with HIP events recorded around each launch on the
 * context's stream (off by default; the events cost a few microseconds per
 * launch).  Statistics accumulate from the call that switches timing on.
 * bytes: algorithmic HBM bytes of all timed launches (every operand read
 * or written once, stored blocks counted with their N*N values, neighbour
 * gathers not counted); flops likewise.
 */
typedef enum {
  LDG_K_DIV = 0,       /* divergence half of the operator: streams the stored blocks
                          (matrix-free: the terms without blocks) */
  LDG_K_GRAD = 1,      /* gradient half of the operator */
  LDG_K_BJ_APPLY = 2,  /* block-Jacobi application */
  LDG_K_ASSEMBLE = 3,  /* block assembly */
  LDG_K_BJ_SETUP = 4,  /* block-Jacobi setup and inversion */
  LDG_K_KRYLOV = 5,    /* Gram-Schmidt dots, updates, vector updates */
  LDG_K_PROJECT = 6,   /* projections and boundary data */
  LDG_K_GNN = 7,       /* graph-network inference and training */
  LDG_K_FACTOR = 8,    /* factored learned preconditioner: setup and application */
  LDG_K_MF = 9,        /* matrix-free block terms of the divergence half */
  LDG_K_RESIDUAL = 10, /* the operator applies of the FP64 residual of each refinement sweep
                          (counted here, not under LDG_K_DIV / LDG_K_GRAD / LDG_K_MF) */
  LDG_K_COUNT = 11
} ldg_kernel_id;
typedef struct {
  int64_t launches;
  double total_ms;
  double bytes;
  double flops;
} ldg_kernel_stat;
ldg_status ldg_set_timing(ldg_ctx* ctx, int on);

/*
 * Matrix-free operator apply (on = 1; default 0).  The Krylov iterations then
 * do not stream the stored D-dependent blocks: the divergence half applies
 * sum_m B^m Z^m + sum_n U_kn (nu^1 Z^1_k+ + nu^2 Z^2_k+) by contracting the
 * projected coefficient D (FP64) with the reference tensors G_hat, R_hat_diag
 * and R_hat_off (Sec. 3.6.3, 3.6.6, 3.6.7) on the matrix cores inside the
 * apply: one GEMM over the pairs (l, j) per triangle group, with the tensor
 * as the shared operand and D_kl u_j as the per-triangle one.  FP64 vectors
 * use FP64 matrix instructions; the FP32 inner solves of the mixed modes use
 * FP32 ones (FP32 operands and sums, more accurate than BF16 blocks).  The
 * stored blocks are still assembled once per step for the block-Jacobi and
 * learned preconditioners.  Takes effect at the next apply.  p <= 4 only
 * (LDG_EINVAL otherwise).
 */
ldg_status ldg_set_matrix_free(ldg_ctx* ctx, int on);
ldg_status ldg_get_kernel_stat(ldg_ctx* ctx, int kernel, ldg_kernel_stat* out);

/* ---- entry points of the individual steps of the path (used by the tests) ---- */

/*
 * Assemble the D-dependent blocks (Sec. 3.6.3, 3.6.6, 3.6.7) from a
 * projected coefficient D (device, K x N):
 *   slot 0, 1: B^m_kk = -G^m_k + R^{m,diag}_k + R^m_{D,k}        (m = 1, 2)
 *   slot 2+n : U_kn = 1/2 |E_kn| sum_l D_{k+ l} R_hat_off(:,:,l,n,n+),
 *              so that R^m_{k k+} = nu^m_kn U_kn (eq:globR:offdiag);
 *              zero for boundary edges.
 * The blocks stay in the context; ldg_get_blocks copies them out as
 * device K x 5 x N x N (element, slot, row i, column j).
 */
ldg_status ldg_assemble(ldg_ctx* ctx, const double* D);
ldg_status ldg_get_blocks(ldg_ctx* ctx, double* out);
/*
 * Mixed-precision contexts also contract the blocks at the inner-solve
 * precision (FP32, or BF16 operands with FP32 accumulation) on the matrix
 * cores; ldg_get_blocks_lowp copies those out widened to FP64, same layout.
 */
ldg_status ldg_get_blocks_lowp(ldg_ctx* ctx, double* out);
/*
 * The FP64 blocks (n x 5 x N x N) or block-Jacobi inverses (n x N x N) of
 * the n triangles listed in elems (device, 0-based, each < K; not checked
 * on the device), for sampled checks of large meshes.  out: device.
 */
ldg_status ldg_get_blocks_rows(ldg_ctx* ctx, const int32_t* elems, int64_t n, double* out);
ldg_status ldg_get_bj_rows(ldg_ctx* ctx, const int32_t* elems, int64_t n, double* out);

/*
 * Operator of the eliminated system with the blocks of the last
 * ldg_assemble: y = M C + dt (eta (S + S_D) C - sum_m B^m M^{-1} A^m C),
 * A^m = -H^m + Q^m + Q^m_N, B^m = -G^m + R^m + R^m_D (eq:timeDepSystem).
 * C, y: device K x N.
 */
ldg_status ldg_apply_schur(ldg_ctx* ctx, double dt, const double* C, double* y);

/*
 * The same operator evaluated as the inner solves of the mixed modes do:
 * C rounded to FP32, both halves in FP32 arithmetic, y widened to FP64.  The
 * block terms come from the coefficient of the last ldg_assemble: in the
 * quadrature form of ldg_options.edge_traces (the default with
 * LDG_QUAD_EXACT), else from the context's FP32 or BF16 copies of its blocks.
 * C, y: device K x N, element-major.  LDG_EINVAL in an FP64 context.
 */
ldg_status ldg_apply_schur_lowp(ldg_ctx* ctx, double dt, const double* C, double* y);

/*
 * ldg_apply_schur without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same operator, same kernels, same result bit for bit.
 * Its four temporary vectors live in a fixed 64 MiB device workspace that the
 * library holds on every device it runs on until the process ends, so the
 * mesh must satisfy 4 * Kpad * N * 8 <= 64 MiB, i.e. Kpad * N <= 2,097,152
 * (Kpad = K rounded up to a multiple of 64): larger meshes get LDG_EINVAL
 * before any launch.  The call allocates nothing and frees nothing.  All
 * contexts on one device share the workspace: calls that can overlap on one
 * device (other streams, other threads) race and must be serialised by the
 * caller.  C, y: device K x N, element-major, caller-owned.
 */
ldg_status ldg_apply_schur_noalloc(ldg_ctx* ctx, double dt, const double* C, double* y);

/*
 * Full operator of eq:fullSystem: out = (W + dt A) Y for Y = [Z1; Z2; C]
 * (device, 3 K N, each part element-major), blocks of the last ldg_assemble.
 */
ldg_status ldg_apply_full(ldg_ctx* ctx, double dt, const double* Y, double* out);

/*
 * Block-Jacobi preconditioner: inverses of the K diagonal N x N blocks of
 * the eliminated operator above (device, K x N x N), for step size dt.
 */
ldg_status ldg_bj_setup(ldg_ctx* ctx, double dt);
ldg_status ldg_get_bj(ldg_ctx* ctx, double* out);

/*
 * Synthetic benchmark data: samples of the analytic fields of a workload at
 * the kind-0 / kind-1 points at time t (not part of the method; it stands in
 * for a caller's coefficient functions).
 *   kind   1: d = 1 + sin(pi x) cos(pi y) exp(-t)/2
 *          2: d = exp(sin(2 pi x) sin(2 pi y)/2) (1 + t/10)
 *          3: d = dT[k] on triangle k          (piecewise constant)
 *          4: d = dT[k] (1 + sin(t)/10)
 *          5: d = exp(x + y), stationary c
 *   c = cos(7x) cos(7y) exp(-t) (kind 5: without exp(-t)),
 *   f = dt c - div(d grad c) (inside each triangle for kinds 3, 4),
 *   c_D = c, g_N = -grad c . nu, c0 = c at t = 0.
 *   kind   6: the problem of the paper's main script (Sec. 4): d = 1.01 on the
 *             open square (1/4, 3/4)^2 and 0.01 elsewhere, f = t/10,
 *             c_D = sin(2 pi y + t), g_N = y, c0 = sin(x) cos(y) (no
 *             closed-form solution; its Neumann edges lie at y = 0 and 1).
 *   dT: device, K values (kinds 3, 4 only, else NULL).  Any output may be NULL;
 *   layouts as in ldg_quad_points.
 */
ldg_status ldg_sample_workload(ldg_ctx* ctx, int kind, double t, const double* dT, double* d,
                               double* f, double* cD, double* gN, double* c0);

/*
 * Learned preconditioner (options.precond = LDG_PC_GNN; p <= 4, every
 * ldg_gnn_* call returns LDG_EINVAL for p = 5, 6).  A graph network on
 * the element graph (nodes: triangles; edges: interior edges, both
 * directions), FP32, width 32: an encoder, three message-passing layers
 * (message relu(h_j W_m + e_kj W_e + b_m) summed over neighbours, residual
 * update h_k += relu([h_k, a_k] W_u + b_u)) and a linear decoder.  Inputs:
 * r_hat = BJ^{-1} r / rho (rho = RMS of BJ^{-1} r), log mean d, relative
 * higher modes of D, log area, log(dt d / |T|), eta per triangle; normal,
 * log edge length, one-hot (n, n+) and log coefficient ratio per edge.  The
 * preconditioner is P(r) = BJ^{-1} r + rho g(r_hat), used inside flexible
 * CG; a breakdown returns the step to block-Jacobi CG (fallbacks), and the
 * FP64 residual of the full system decides convergence as always.  For
 * nonsymmetric steps (GMRES) block-Jacobi is used and one fallback counted.
 * Parameters are a flat FP32 vector: W_enc [(2N+3) x 32], b_enc [32], then
 * per layer W_m [32 x 32], W_e [13 x 32], b_m [32], W_u [64 x 32], b_u [32],
 * then W_dec [32 x N], b_dec [N] (row-major).
 */
/*
 * Network mode.  LDG_GNN_CORRECTION (default): the residual-correction
 * network above, applied at every iteration inside flexible CG.
 * LDG_GNN_FACTOR: a linear, symmetric positive definite preconditioner built
 * once per system,
 *   P = W^T (I + F)^T (I + F) W,  W = blockdiag(W_k), W_k^T W_k = BJ_k^{-1}
 *   (W_k the transposed lower Cholesky factor of the block-Jacobi inverse),
 *   F_kj = -omega_kn O_kn for j = k+ across edge n,  O_kn = W_k S_kj W_j^T,
 * with S_kj the blocks of the eliminated operator between triangles sharing
 * an edge and omega_kn = 0.95 sigmoid(h_k w_hk + h_j w_hj + e_kn w_e
 * + w_o log ||O_kn||_F + b_o) from the same encoder and three layers fed the
 * node features only (N + 3 inputs).  Plain preconditioned CG keeps its
 * optimality with it; a breakdown returns the step to block-Jacobi CG.
 * Nonsymmetric steps (d varying inside triangles) build the same operator
 * from the symmetric part: W_k from the Cholesky factor of (BJ_k^{-1} +
 * BJ_k^{-T}) / 2 and O_kn = W_k (S_kj + S_jk^T) / 2 W_j^T, SPD again, and apply
 * it as a fixed right preconditioner of GMRES (where that Cholesky factor
 * does not exist the step runs block-Jacobi GMRES and counts a fallback).
 * Parameters: the trunk as above with W_enc [(N+3) x 32], then w_hk [32],
 * w_hj [32], w_e [13], w_o, b_o.  Training uses the energy loss of
 * ldg_gnn_set_loss on the collected pairs, with the error e = target + rhat:
 * (P r - e)^T S (P r - e) / (BJ^{-1} r - e)^T S (BJ^{-1} r - e), r = S e,
 * or, with LDG_GNN_LOSS_FROBENIUS, the factorised-sparse-approximate-inverse
 * objective for a probe vector w passed as rhat (target unused):
 * ||(G S G^T - I) w||^2 / ||(W S W^T - I) w||^2, G = (I + F) W; Gaussian
 * probes make it a Hutchinson estimate of ||G S G^T - I||_F^2 (relative).
 * The energy loss favours smooth modes alone and can drive omega to its cap;
 * the Frobenius loss weighs every mode alike.
 * Changing the mode drops the parameters.  Unknown modes: LDG_EINVAL.
 */
typedef enum { LDG_GNN_CORRECTION = 0, LDG_GNN_FACTOR = 1 } ldg_gnn_mode;
ldg_status ldg_gnn_set_mode(ldg_ctx* ctx, int mode);
/* parameter count of the current mode */
ldg_status ldg_gnn_num_params(ldg_ctx* ctx, int64_t* n);
/* host parameter vector in/out; setting resets the Adam moments */
ldg_status ldg_gnn_set_params(ldg_ctx* ctx, const float* w, int64_t n);
ldg_status ldg_gnn_get_params(ldg_ctx* ctx, float* w, int64_t n);
/*
 * Training loss.  LDG_GNN_LOSS_MSE (default): mean over (k, i) of
 * (g_ki - target_ki)^2.  LDG_GNN_LOSS_ENERGY: (g - t)^T S (g - t) / (t^T S t)
 * with S the eliminated operator of the context (coefficient D, step dt), i.e.
 * the energy-norm error of the corrected step relative to that of the plain
 * block-Jacobi step; it needs ldg_gnn_set_context after this call, which then
 * also assembles the FP64 blocks of D (overwriting the solver's) and returns
 * LDG_EINVAL unless D is constant on every triangle (S symmetric, the case
 * the learned preconditioner serves).  LDG_GNN_LOSS_OPTSTEP (factored network
 * only): the energy left after one preconditioned step with the best step
 * length, min_t ||e - t P r||_S^2 / ||e||_S^2 = 1 - (r^T P r)^2 /
 * ((P r)^T S (P r) e^T r) with r = S e, e = target + rhat; it does not change
 * when e or P is scaled (as CG's iterates do not), and on smooth errors (the
 * late errors of the method's own CG solves) its minimum sits where CG's
 * iteration count has its own.  Unknown values: LDG_EINVAL.
 */
typedef enum {
  LDG_GNN_LOSS_MSE = 0, LDG_GNN_LOSS_ENERGY = 1, LDG_GNN_LOSS_FROBENIUS = 2,
  LDG_GNN_LOSS_OPTSTEP = 3
} ldg_gnn_loss;
ldg_status ldg_gnn_set_loss(ldg_ctx* ctx, int loss);
/* per-triangle and per-edge features from D (device K x N, NULL: last projected) and dt */
ldg_status ldg_gnn_set_context(ldg_ctx* ctx, const double* D, double dt);
/* g = network(r_hat): r_hat, g device K x N FP32 (correction mode) */
ldg_status ldg_gnn_forward(ldg_ctx* ctx, const float* rhat, float* g);
/*
 * Factor mode, after a factor build (ldg_gnn_set_context, or a step with the
 * learned preconditioner; omega from the features of that system): omega (device K x 3 FP32, 0 on
 * boundary edges) from the current parameters, and the factor blocks
 * (device K x 4 x N x N FP64: W_k, O_k0, O_k1, O_k2 row-major, O on boundary
 * edges undefined; may be NULL) with log ||O_kn||_F (device K x 3 FP32,
 * undefined on boundary edges; may be NULL), as stored (see below).
 */
ldg_status ldg_gnn_factor_omega(ldg_ctx* ctx, float* omega);
/*
 * Storage of the factor blocks: LDG_FAC_FP8 (default; W_k in BF16, O_kn in OCP
 * E4M3 FP8, round to nearest even; the entries of O_kn, blocks of a symmetric
 * positive definite matrix with identity diagonal blocks, lie in [-1, 1]),
 * LDG_FAC_FP8W (both in E4M3; W_k stored as s_k W8_k with the power of two
 * s_k = 2^round(log2(max |W_k| / 256)) per triangle, which keeps the block
 * inside the E4M3 range), LDG_FAC_BF16 (both in BF16) or LDG_FAC_F32.  Only
 * the upper triangle of W_k is stored.  P stays exactly symmetric positive definite in each, the same rounded blocks
 * forming G and G^T; the solution's accuracy is set by the FP64 residual as
 * always.  Takes effect at the next factor build (step or
 * ldg_gnn_set_context).
 */
typedef enum {
  LDG_FAC_F32 = 0, LDG_FAC_BF16 = 1, LDG_FAC_FP8 = 2, LDG_FAC_FP8W = 3
} ldg_fac_storage;
ldg_status ldg_gnn_factor_storage(ldg_ctx* ctx, int storage);
ldg_status ldg_gnn_factor_export(ldg_ctx* ctx, double* blocks, float* lognorm);
/*
 * The same for the triangles elems[0..n) only (device int32, each in [0, K),
 * else LDG_EINVAL before any launch): blocks device n x 4 x N x N FP64,
 * lognorm device n x 3 FP32 (may be NULL).  Valid after a factor build (a
 * step with the learned preconditioner or ldg_gnn_set_context).
 */
ldg_status ldg_gnn_factor_export_rows(ldg_ctx* ctx, const int32_t* elems, int64_t n,
                                      double* blocks, float* lognorm);
/*
 * loss (as selected by ldg_gnn_set_loss) and its gradient (device, n_params
 * floats, may be NULL); the weight gradients are fixed-order FP64
 * reductions.  ldg_gnn_train_step does the same and one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr.
 */
ldg_status ldg_gnn_loss_grad(ldg_ctx* ctx, const float* rhat, const float* target, float* grad,
                             double* loss);
ldg_status ldg_gnn_train_step(ldg_ctx* ctx, const float* rhat, const float* target, double lr,
                              double* loss);
/*
 * Training data from the method's own solves: arm the next ldg_step_sampled
 * (FP64 block-Jacobi CG) to keep its iterates x_s at the CG iterations
 * iters[0] < iters[1] < ... (host, nsnap <= 64).  When the step converges to
 * x*, pair s is e = x* - x_s, r = A e, z = BJ^{-1} r, rho = RMS(z):
 * rhat_out[s] = z / rho, target_out[s] = (e - z) / rho (device, nsnap x K x N
 * FP32, element-major).  ldg_gnn_collected reports how many were taken.
 */
ldg_status ldg_gnn_collect(ldg_ctx* ctx, int nsnap, const int32_t* iters, float* rhat_out,
                           float* target_out);
ldg_status ldg_gnn_collected(ldg_ctx* ctx, int* n);

/* ---- Host field callbacks ---------------------------------------------- */

/*
 * Fields given as host functions instead of samples.  A field callback fills
 * out[i] = value at (x[i], y[i]) for i < n, at time t, and returns 0 (non-zero:
 * the call fails with LDG_ECALLBACK and the state is unchanged).  The Neumann
 * flux also receives the exterior unit normal (nx[i], ny[i]) of the boundary
 * edge the point lies on (the Neumann data of Sec. 1.3 is a normal flux).  All
 * arrays are host memory owned by the library for the duration of the call.
 * The points are the library's: the volume points of ldg_quad_points kind 0
 * for d, f, c0; the boundary Gauss points of kind 1 for c_D and g_N.
 */
typedef int (*ldg_field_fn)(void* user, double t, const double* x, const double* y, double* out,
                            int64_t n);
typedef int (*ldg_flux_fn)(void* user, double t, const double* x, const double* y,
                           const double* nx, const double* ny, double* out, int64_t n);
typedef struct {
  ldg_field_fn d;     /* diffusion coefficient */
  ldg_field_fn f;     /* source */
  ldg_field_fn c_D;   /* Dirichlet data (may be NULL without Dirichlet edges) */
  ldg_flux_fn g_N;    /* Neumann data (may be NULL without Neumann edges) */
  void* user;         /* passed to every callback */
} ldg_problem;

/* Initial state: the L2 projection (Sec. 3.4) of c0(x, y) = c0_fn at t = 0; t is set to 0. */
ldg_status ldg_set_initial(ldg_ctx* ctx, ldg_field_fn c0, void* user);
/*
 * One step t -> t + dt as ldg_step_sampled (same scheme, options and error
 * behaviour), with d, f, c_D, g_N evaluated on the host at t + dt (Sec. 2.5)
 * by the problem's callbacks.
 */
ldg_status ldg_step(ldg_ctx* ctx, double dt, const ldg_problem* problem, ldg_step_info* info);
/*
 * Initial state from its coefficients: C^0 given directly in the basis of
 * Sec. 2.4.1 (K x N FP64, element-major as in ldg_get_solution; device
 * pointer if on_device, else host), instead of the projection of c0 that
 * the main script of Sec. 4 starts from.  Z1 and Z2 are left as they are
 * until the next step recomputes them: W has zero Z rows in the step of
 * Sec. 2.5, so the flux of the initial state never enters a step.  t = 0;
 * the BDF2 history is cleared.  LDG_EINVAL for NULL arguments.
 */
ldg_status ldg_set_initial_dofs(ldg_ctx* ctx, const double* C, int on_device);
/* Network parameters in and out (the same as ldg_gnn_set_params / ldg_gnn_get_params). */
ldg_status ldg_gnn_load(ldg_ctx* ctx, const float* w, int64_t n);
ldg_status ldg_gnn_save(ldg_ctx* ctx, float* w, int64_t n);

/* ---- Input and output -------------------------------------------------- */

/*
 * Read a triangulation from an ASCII MEDIT ".mesh" file, the format Gmsh
 * writes and the paper's circle-domain generator reads (Sec. 4,
 * domainCircle): sections Vertices (x y [z] ref, the count of coordinates
 * set by a Dimension 2 / 3 keyword, default 3), Edges (v1 v2 ID: the boundary
 * ID of a boundary edge) and Triangles (v1 v2 v3 ref), 1-based vertex
 * numbers, "#" comments.  Two calls: with coordV, V0T and edge_id NULL it
 * sets *numV and *K; then, with those values in *numV and *K, it fills
 *   coordV   host numV x 2
 *   V0T      host K x 3, 0-based, reordered counter-clockwise where needed
 *   edge_id  host K x 3, per local edge n (opposite local vertex n): 0 for an
 *            edge shared by two triangles, the listed ID (> 0) of a boundary
 *            edge, -1 for a boundary edge the file lists no ID for.
 * Errors: EIO (the file cannot be opened), EMESH (malformed file, a vertex
 * number out of range, an edge in more than two triangles, a boundary ID
 * <= 0), EINVAL (NULL pointers, sizes that differ from the file's).  No
 * context: ldg_last_error(NULL) gives the text.
 */
ldg_status ldg_mesh_read_medit(const char* path, int64_t* numV, int64_t* K, double* coordV,
                               int32_t* V0T, int32_t* edge_id);

/*
 * Edge kinds from boundary IDs (the paper's main script marks the edges with
 * IDs 1 and 3 Neumann, all other boundary edges Dirichlet): ID 0 interior, an
 * ID in neumann_ids[0..n_neumann) Neumann, any other positive ID Dirichlet;
 * host arrays of K x 3.  A negative ID: EMESH.
 */
ldg_status ldg_edge_kinds_from_ids(int64_t K, const int32_t* edge_id, const int32_t* neumann_ids,
                                   int n_neumann, int8_t* edge_kind);

/*
 * Values of a discrete function at the Lagrange points of every triangle
 * (Sec. 3.8): nL = 1 (p = 0: the barycentre), 3 (p = 1: the vertices) or 6
 * (p >= 2: the vertices, then the midpoints of the edges opposite vertices
 * 1, 2, 3; for p > 2 these are point values of the order-p function, the
 * output holding at most quadratics).  C: device K x N element-major, or NULL
 * for the current state.  out: device K x nL element-major, or NULL to query
 * *nL only.
 */
ldg_status ldg_lagrange(ldg_ctx* ctx, const double* C, double* out, int* nL);

/*
 * Write Lagrange values (host K x nL, as ldg_lagrange returns them) as an XML
 * VTK unstructured-grid file (.vtu) for visualization (Sec. 3.8): every
 * triangle carries its own points (the function is discontinuous); linear
 * triangles (VTK type 5) for nL = 1 (the value at all three vertices) and
 * nL = 3, quadratic triangles (type 22) for nL = 6; Float32 point data named
 * `name` (no XML special characters).  binary = 0: ASCII with 9 significant
 * digits; else base64 "binary" arrays (UInt32 byte-count header).  Errors:
 * EINVAL (nL other than ldg_lagrange's), EIO.
 */
ldg_status ldg_write_vtu(ldg_ctx* ctx, const char* path, const char* name, const double* lagr,
                         int nL, int binary);

#ifdef __cplusplus
}
#endif
#endif /* LDG_H */
