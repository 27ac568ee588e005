"""LDG discretisation of the diffusion equation, written from the paper.

Everything is plain FP64 numpy/scipy.  Vectors are element-major,
index (k-1)N+i of the paper being k*N + i here; the full solution vector is
Y = [Z1; Z2; C] (eq:fullSystem).

Sources:
  projection          Sec. 3.4 (L2 projection), M_hat = identity
  blocks              Sec. 2.4.3 / 2.4.4 (component-wise definitions), transformed
                      to the reference triangle as in Sec. 3.6 (eq:hatM ... eq:hatRoffdiag)
  system              eq:timeDepSystem, eq:fullSystem and its implicit Euler step
  error               Sec. 3.5 (computeL2Error)

Readings where the paper is silent or inconsistent (all listed in the design
notes of the repository):
  * the penalty uses 1/|E| (eq:globS), not 1/h_T;
  * the diagonal blocks of R^m use nu^m for both m (eq:globR:diag);
  * G^m = sum_l D_kl (b1 G_hat(:,:,l,1) + b2 G_hat(:,:,l,2)) with
    (b1, b2) = (B22, -B21) for m = 1 and (-B12, B11) for m = 2 (eq:hatG);
  * data d, f, c_D, g_N are taken at the new time level t^{n+1}.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .mesh import DIRICHLET, INTERIOR, NEUMANN, Grid
from .quadrature import boundary_order, collapsed_rule, projection_order, rule_1d, triangle_rule
from .refelem import RefTensors, gamma


# --------------------------------------------------------------------------
# L2 projection (Sec. 3.4)
# --------------------------------------------------------------------------
def volume_points(grid, p, order=None, elems=None):
    """Physical quadrature points [K x R] of the projection rule and its weights."""
    q1, q2, w = triangle_rule(projection_order(p) if order is None else order)
    X1, X2 = grid.map_to_physical(q1, q2, elems)
    return X1, X2, (q1, q2, w)


def project_samples(samples, rule, hatM):
    """D hatM = sum_r w_r d(F_k(q_r)) phi(q_r)  ->  D   (samples: [K x R])."""
    q1, q2, w = rule
    N = hatM.shape[0]
    rhs = samples @ (w[:, None] * basis.phi_all(N, q1, q2))
    return np.linalg.solve(hatM.T, rhs.T).T


def project(grid, p, func, hatM, order=None, elems=None):
    """L2 projection of func(x1, x2) onto P_p(T_h) (rows: all triangles or `elems`)."""
    X1, X2, rule = volume_points(grid, p, order, elems)
    return project_samples(func(X1, X2), rule, hatM)


def l2_error(grid, C, func, order=None):
    """||c_h - c||_{L2(Omega)} with a triangle rule (Sec. 3.5)."""
    N = C.shape[1]
    p = basis.order_of(N)
    if order is None:
        q1, q2, w = collapsed_rule(p + 6)
    else:
        q1, q2, w = triangle_rule(order)
    X1, X2 = grid.map_to_physical(q1, q2)
    ch = C @ basis.phi_all(N, q1, q2).T
    return np.sqrt(2 * np.dot(((ch - func(X1, X2)) ** 2) @ w, grid.areaT))


# --------------------------------------------------------------------------
# Boundary data vectors (Sec. 3.6.9-3.6.11): J_D^m, K_D, K_N
# --------------------------------------------------------------------------
def boundary_points(grid, p):
    """Physical edge quadrature points [K x 3 x R1] of the order-(2p+1) rule."""
    s, ws = rule_1d(boundary_order(p))
    X1 = np.zeros((grid.numT, 3, len(s)))
    X2 = np.zeros_like(X1)
    for n in range(3):
        g1, g2 = gamma(n, s)
        X1[:, n], X2[:, n] = grid.map_to_physical(g1, g2)
    return X1, X2, (s, ws)


def boundary_vectors(grid, p, cD, gN, D):
    """J1_D, J2_D, K_D, K_N as [K x N] arrays.

    cD(x1, x2) and gN(x1, x2, nu1, nu2) are the boundary data at the new time."""
    N = basis.num_basis(p)
    K = grid.numT
    X1, X2, (s, ws) = boundary_points(grid, p)
    J = np.zeros((2, K, N))
    KD = np.zeros((K, N))
    KN = np.zeros((K, N))
    for n in range(3):
        g1, g2 = gamma(n, s)
        Pn = basis.phi_all(N, g1, g2)                    # [R1 x N]
        dir_ = grid.kind[:, n] == DIRICHLET
        if np.any(dir_):
            cv = cD(X1[dir_, n], X2[dir_, n])            # [Kd x R1]
            integral = cv @ (ws[:, None] * Pn)           # int_0^1 phi_i(g_n) c_D ds
            for m in range(2):
                J[m, dir_] += (grid.nuE0T[dir_, n, m] * grid.areaE0T[dir_, n])[:, None] * integral
            KD[dir_] += integral
        neu = grid.kind[:, n] == NEUMANN
        if np.any(neu):
            gv = gN(X1[neu, n], X2[neu, n], grid.nuE0T[neu, n, 0:1], grid.nuE0T[neu, n, 1:2])
            # int_0^1 phi_i phi_l g_N ds, then contracted with D_kl
            integral = np.einsum("kr,r,ri,rl->kil", gv, ws, Pn, Pn)
            KN[neu] += grid.areaE0T[neu, n][:, None] * np.einsum("kil,kl->ki", integral, D[neu])
    return J[0], J[1], KD, KN


# --------------------------------------------------------------------------
# Block rows of the global matrices (Sec. 2.4.3, 2.4.4 and Sec. 3.6)
# --------------------------------------------------------------------------
def _coo(rows, cols, blocks, nrow_blocks, K, N):
    """Sparse [nrow_blocks*N x K*N] matrix from N x N blocks at block (rows, cols)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    if len(rows) == 0:
        return sp.csr_matrix((nrow_blocks * N, K * N))
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    R = (rows[:, None, None] * N + ii).reshape(-1)
    Cc = (cols[:, None, None] * N + jj).reshape(-1)
    return sp.csr_matrix((blocks.reshape(-1), (R, Cc)), shape=(nrow_blocks * N, K * N))


class Blocks:
    """Rows of M, H^m, Q^m, Q^m_N, S, S_D, G^m, R^m, R^m_D for the elements `elems`.

    Each attribute is a sparse matrix with len(elems)*N rows and K*N columns;
    with elems = all elements these are the global matrices of the paper."""

    def __init__(self, grid, refs, D=None, elems=None):
        K, N = grid.numT, refs.N
        el = np.arange(K) if elems is None else np.asarray(elems)
        ne = len(el)
        pos = np.arange(ne)
        B = grid.B[el]
        B11, B12, B21, B22 = B[:, 0, 0], B[:, 0, 1], B[:, 1, 0], B[:, 1, 1]
        hH, hG = refs.hatH, refs.hatG
        Sd, So, Rd, Ro = refs.hatSdiag, refs.hatSoff, refs.hatRdiag, refs.hatRoff
        nu = grid.nuE0T[el]
        aE = grid.areaE0T[el]
        kind = grid.kind[el]
        kp, npl = grid.kp[el], grid.np_[el]
        blk = lambda a, M: a[:, None, None] * M[None]
        # mass (eq:globMlocM, eq:hatM): M_k = 2|T_k| M_hat
        self.M = _coo(pos, el, blk(2 * grid.areaT[el], refs.hatM), ne, K, N)
        # H^m (Sec. 3.6.2)
        H1 = blk(B22, hH[:, :, 0]) - blk(B21, hH[:, :, 1])
        H2 = -blk(B12, hH[:, :, 0]) + blk(B11, hH[:, :, 1])
        self.H = [_coo(pos, el, H1, ne, K, N), _coo(pos, el, H2, ne, K, N)]
        # Q^m, S (eq:globQ, eq:globS), Q^m_N (eq:globQm:N), S_D (eq:globS:D)
        Qd = [np.zeros((ne, N, N)), np.zeros((ne, N, N))]
        QNd = [np.zeros((ne, N, N)), np.zeros((ne, N, N))]
        Sdg = np.zeros((ne, N, N))
        SDd = np.zeros((ne, N, N))
        Qo_r, Qo_c, Qo_b, So_b = [], [], [[], []], []
        for n in range(3):
            it = kind[:, n] == INTERIOR
            di = kind[:, n] == DIRICHLET
            ne_ = kind[:, n] == NEUMANN
            for m in range(2):
                Qd[m] += blk(0.5 * it * nu[:, n, m] * aE[:, n], Sd[:, :, n])
                QNd[m] += blk(ne_ * nu[:, n, m] * aE[:, n], Sd[:, :, n])
            Sdg += blk(it * 1.0, Sd[:, :, n])            # (1/|E|) |E| S_hat_diag
            SDd += blk(di * 1.0, Sd[:, :, n])
            idx = np.nonzero(it)[0]
            Qo_r.append(pos[idx])
            Qo_c.append(kp[idx, n])
            Soff = So[:, :, n, npl[idx, n]].transpose(2, 0, 1)   # [E x N x N]
            for m in range(2):
                Qo_b[m].append(blk(0.5 * nu[idx, n, m] * aE[idx, n], np.ones((N, N))) * Soff)
            So_b.append(-Soff)
        orow, ocol = np.concatenate(Qo_r), np.concatenate(Qo_c)
        self.Q = [_coo(pos, el, Qd[m], ne, K, N) + _coo(orow, ocol, np.concatenate(Qo_b[m]), ne, K, N)
                  for m in range(2)]
        self.QN = [_coo(pos, el, QNd[m], ne, K, N) for m in range(2)]
        self.S = _coo(pos, el, Sdg, ne, K, N) + _coo(orow, ocol, np.concatenate(So_b), ne, K, N)
        self.SD = _coo(pos, el, SDd, ne, K, N)
        if D is None:
            return
        # G^m (eq:locGm with eq:hatG)
        De = D[el]
        Gl1 = np.einsum("kl,ijl->kij", De, hG[:, :, :, 0])
        Gl2 = np.einsum("kl,ijl->kij", De, hG[:, :, :, 1])
        G1 = blk(B22, np.ones((N, N))) * Gl1 - blk(B21, np.ones((N, N))) * Gl2
        G2 = -blk(B12, np.ones((N, N))) * Gl1 + blk(B11, np.ones((N, N))) * Gl2
        self.G = [_coo(pos, el, G1, ne, K, N), _coo(pos, el, G2, ne, K, N)]
        # R^m (eq:globR with eq:hatRdiag / eq:hatRoffdiag), R^m_D (eq:globR:D)
        Rdg = [np.zeros((ne, N, N)), np.zeros((ne, N, N))]
        RDd = [np.zeros((ne, N, N)), np.zeros((ne, N, N))]
        Ro_b = [[], []]
        for n in range(3):
            it = kind[:, n] == INTERIOR
            di = kind[:, n] == DIRICHLET
            RE = np.einsum("kl,ijl->kij", De, Rd[:, :, :, n])   # R_E / |E|
            for m in range(2):
                Rdg[m] += blk(0.5 * it * nu[:, n, m] * aE[:, n], np.ones((N, N))) * RE
                RDd[m] += blk(di * nu[:, n, m] * aE[:, n], np.ones((N, N))) * RE
            idx = np.nonzero(it)[0]
            Dp = D[kp[idx, n]]                                  # D of the neighbour
            Roff = np.einsum("el,ijle->eij", Dp, Ro[:, :, :, n, npl[idx, n]])
            for m in range(2):
                Ro_b[m].append(blk(0.5 * nu[idx, n, m] * aE[idx, n], np.ones((N, N))) * Roff)
        self.R = [_coo(pos, el, Rdg[m], ne, K, N) + _coo(orow, ocol, np.concatenate(Ro_b[m]), ne, K, N)
                  for m in range(2)]
        self.RD = [_coo(pos, el, RDd[m], ne, K, N) for m in range(2)]


# --------------------------------------------------------------------------
# Global system (eq:timeDepSystem, eq:fullSystem) and implicit Euler
# --------------------------------------------------------------------------
def system(blocks, eta):
    """A(t) as a 3KN x 3KN sparse matrix, Y = [Z1; Z2; C]."""
    b = blocks
    A13 = -b.H[0] + b.Q[0] + b.QN[0]
    A23 = -b.H[1] + b.Q[1] + b.QN[1]
    A31 = -b.G[0] + b.R[0] + b.RD[0]
    A32 = -b.G[1] + b.R[1] + b.RD[1]
    A33 = eta * (b.S + b.SD)
    return sp.bmat([[b.M, None, A13], [None, b.M, A23], [A31, A32, A33]], format="csr")


def rhs_vector(blocks, eta, J1, J2, KD, KN, F):
    """V(t) = [-J1_D; -J2_D; eta K_D - K_N + L] with L = M F."""
    L = blocks.M @ F.reshape(-1)
    return np.concatenate([-J1.reshape(-1), -J2.reshape(-1),
                           eta * KD.reshape(-1) - KN.reshape(-1) + L])


def mass_W(blocks):
    KN = blocks.M.shape[0]
    Z = sp.csr_matrix((KN, KN))
    return sp.bmat([[Z, None, None], [None, Z, None], [None, None, blocks.M]], format="csr")


class Problem:
    """Mesh + order + penalty + data: the inputs of one LDG run."""

    def __init__(self, coordV, V0T, kind, p, eta=1.0, policy="exact"):
        self.grid = Grid(coordV, V0T, kind)
        self.p = p
        self.N = basis.num_basis(p)
        self.eta = eta
        self.refs = RefTensors(p, policy)
        self.static = Blocks(self.grid, self.refs)

    # data at one time level ------------------------------------------------
    def data(self, workload, t):
        g = self.grid
        hatM = self.refs.hatM
        D = project(g, self.p, lambda x, y: workload.d(t, x, y), hatM)
        F = project(g, self.p, lambda x, y: workload.f(t, x, y), hatM)
        J1, J2, KD, KN = boundary_vectors(
            g, self.p, lambda x, y: workload.c_D(t, x, y),
            lambda x, y, n1, n2: workload.g_N(t, x, y, n1, n2), D)
        return dict(D=D, F=F, J1=J1, J2=J2, KD=KD, KN=KN)

    def assemble(self, data):
        b = Blocks(self.grid, self.refs, data["D"])
        A = system(b, self.eta)
        V = rhs_vector(b, self.eta, data["J1"], data["J2"], data["KD"], data["KN"], data["F"])
        return b, A, V

    def initial(self, workload):
        return project(self.grid, self.p, workload.c0, self.refs.hatM)

    # one implicit Euler step ------------------------------------------------
    def step(self, C, t_new, tau, workload, data=None):
        """Solve (W + tau A^{n+1}) Y^{n+1} = W Y^n + tau V^{n+1} directly.

        Returns (C, Z1, Z2, info) with info holding the system pieces."""
        if data is None:
            data = self.data(workload, t_new)
        b, A, V = self.assemble(data)
        W = mass_W(b)
        KN = self.grid.numT * self.N
        Yn = np.concatenate([np.zeros(2 * KN), C.reshape(-1)])
        rhs = W @ Yn + tau * V
        lhs = (W + tau * A).tocsc()
        Y = spla.spsolve(lhs, rhs)
        res = np.linalg.norm(rhs - lhs @ Y) / np.linalg.norm(rhs)
        sh = (self.grid.numT, self.N)
        return (Y[2 * KN:].reshape(sh), Y[:KN].reshape(sh), Y[KN:2 * KN].reshape(sh),
                dict(rhs=rhs, lhs=lhs, rel_residual=res, data=data, blocks=b))

    def step_bdf2(self, C, C_prev, t_new, dt, workload, data=None):
        """Two-step backward differentiation in time (second order), with the
        space discretisation of the paper's implicit Euler step (Sec. 2.5):
            W (3/2 Y^{n+1} - 2 Y^n + 1/2 Y^{n-1}) / dt + A^{n+1} Y^{n+1} = V^{n+1},
        i.e. (W + tau A^{n+1}) Y^{n+1} = W Y* + tau V^{n+1} with tau = 2 dt / 3 and
        Y* = (4 Y^n - Y^{n-1}) / 3.  W has zero Z rows, so only the C parts of the
        history enter.  Equal steps dt are assumed."""
        return self.step((4.0 * C - C_prev) / 3.0, t_new, 2.0 * dt / 3.0, workload, data)

    def solve_stationary(self, workload):
        """Solve A Y = V at t = 0 (the verification setting of Sec. 3.7)."""
        data = self.data(workload, 0.0)
        b, A, V = self.assemble(data)
        Y = spla.spsolve(A.tocsc(), V)
        KN = self.grid.numT * self.N
        sh = (self.grid.numT, self.N)
        return Y[2 * KN:].reshape(sh), Y[:KN].reshape(sh), Y[KN:2 * KN].reshape(sh)


# --------------------------------------------------------------------------
# Block elimination of Z (used to check the GPU's Schur-form operator)
# --------------------------------------------------------------------------
def minv_blocks(grid, refs):
    """M^{-1} as a sparse block-diagonal matrix: (2|T_k| M_hat)^{-1}."""
    K, N = grid.numT, refs.N
    inv = np.linalg.inv(refs.hatM)
    return _coo(np.arange(K), np.arange(K),
                (1.0 / (2 * grid.areaT))[:, None, None] * inv[None], K, K, N)


def schur_pieces(blocks, grid, refs, eta):
    """(A^m, B^m, M, M^{-1}, S') of the full matrix, A^m = -H^m + Q^m + Q^m_N,
    B^m = -G^m + R^m + R^m_D, S' = eta (S + S_D)."""
    b = blocks
    A = [-b.H[m] + b.Q[m] + b.QN[m] for m in range(2)]
    Bm = [-b.G[m] + b.R[m] + b.RD[m] for m in range(2)]
    return A, Bm, b.M, minv_blocks(grid, refs), eta * (b.S + b.SD)


def schur_matrix(blocks, grid, refs, eta, tau):
    """Schur complement of (W + tau A) with respect to the Z rows:
    M + tau (eta (S + S_D) - sum_m B^m M^{-1} A^m)."""
    A, Bm, M, Mi, Sp = schur_pieces(blocks, grid, refs, eta)
    return (M + tau * (Sp - Bm[0] @ Mi @ A[0] - Bm[1] @ Mi @ A[1])).tocsr()


def schur_rhs(blocks, grid, refs, eta, tau, Cn, data):
    """Right-hand side of the eliminated system for C^{n+1}."""
    A, Bm, M, Mi, Sp = schur_pieces(blocks, grid, refs, eta)
    L = M @ data["F"].reshape(-1)
    b3 = M @ Cn.reshape(-1) + tau * (eta * data["KD"].reshape(-1) - data["KN"].reshape(-1) + L)
    for m, J in enumerate((data["J1"], data["J2"])):
        b3 = b3 + tau * (Bm[m] @ (Mi @ J.reshape(-1)))
    return b3


def recover_z(blocks, grid, refs, eta, C, data):
    """Z^m = -M^{-1}(A^m C + J^m_D) from the first two block rows."""
    A, _, _, Mi, _ = schur_pieces(blocks, grid, refs, eta)
    sh = C.shape
    return [(-(Mi @ (A[m] @ C.reshape(-1) + J.reshape(-1)))).reshape(sh)
            for m, J in enumerate((data["J1"], data["J2"]))]


def step_schur(problem, C, t_new, tau, workload, data=None):
    """Implicit Euler step solved on the eliminated system (sparse direct)."""
    pr = problem
    if data is None:
        data = pr.data(workload, t_new)
    b = Blocks(pr.grid, pr.refs, data["D"])
    Sm = schur_matrix(b, pr.grid, pr.refs, pr.eta, tau)
    rhs = schur_rhs(b, pr.grid, pr.refs, pr.eta, tau, C, data)
    Cn = spla.spsolve(Sm.tocsc(), rhs).reshape(C.shape)
    Z1, Z2 = recover_z(b, pr.grid, pr.refs, pr.eta, Cn, data)
    return Cn, Z1, Z2, dict(data=data, blocks=b)


def step_schur_cg(problem, C, t_new, tau, workload, rtol=1e-13, maxiter=200000, data=None):
    """Implicit Euler step on the eliminated system by preconditioned CG, for
    meshes too large for the sparse direct solve.

    Valid where the eliminated matrix is symmetric positive definite: d
    constant on every triangle (then B^m = -(A^m)^T diag(d)).  Block-Jacobi
    preconditioner (inverses of the N x N diagonal blocks), start from C^n,
    stop at ||rhs - S C|| <= rtol ||rhs|| in the true residual.
    Returns (C, Z1, Z2, info) with the CG iteration count in info."""
    pr = problem
    if data is None:
        data = pr.data(workload, t_new)
    b = Blocks(pr.grid, pr.refs, data["D"])
    Sm = schur_matrix(b, pr.grid, pr.refs, pr.eta, tau)
    rhs = schur_rhs(b, pr.grid, pr.refs, pr.eta, tau, C, data)
    K, N = C.shape
    diag = np.zeros((K, N, N))
    Sc = Sm.tocsr()
    for i in range(N):
        for j in range(N):
            diag[:, i, j] = Sc[np.arange(K) * N + i, np.arange(K) * N + j].A1
    inv = np.linalg.inv(diag)
    prec = spla.LinearOperator(Sm.shape, matvec=lambda v: np.einsum(
        "kij,kj->ki", inv, v.reshape(K, N)).reshape(-1), dtype=np.float64)
    its = [0]

    def count(_):
        its[0] += 1

    x, flag = spla.cg(Sc, rhs, x0=C.reshape(-1).copy(), rtol=rtol, atol=0.0, maxiter=maxiter,
                      M=prec, callback=count)
    res = np.linalg.norm(rhs - Sc @ x) / np.linalg.norm(rhs)
    Cn = x.reshape(C.shape)
    Z1, Z2 = recover_z(b, pr.grid, pr.refs, pr.eta, Cn, data)
    return Cn, Z1, Z2, dict(data=data, blocks=b, iters=its[0], rel_residual=res, flag=flag)

def full_residual(problem, blocks, data, tau, Cn, C, Z1, Z2):
    """||W Y^n + tau V - (W + tau A) Y|| / ||W Y^n + tau V|| of the full 3KN system."""
    A = system(blocks, problem.eta)
    V = rhs_vector(blocks, problem.eta, data["J1"], data["J2"], data["KD"], data["KN"], data["F"])
    W = mass_W(blocks)
    KN = Cn.size
    Yn = np.concatenate([np.zeros(2 * KN), Cn.reshape(-1)])
    Y = np.concatenate([Z1.reshape(-1), Z2.reshape(-1), C.reshape(-1)])
    rhs = W @ Yn + tau * V
    return np.linalg.norm(rhs - (W + tau * A) @ Y) / np.linalg.norm(rhs)


def schur_apply_rows(grid, refs, D, C, tau, eta, elems, J=None):
    """Rows `elems` of M C + tau(eta S' C + sum_m B^m Z^m),  Z^m = -M^{-1}(A^m C [+ J^m]).

    Only the block rows these rows touch are built: B^m, M, S' on `elems`,
    A^m on `elems` and their neighbours.  Returns (y [len x N], Z [2][len x N])
    with Z on `elems`."""
    K, N = grid.numT, refs.N
    elems = np.asarray(elems)
    nbr = grid.kp[elems]
    patch = np.unique(np.concatenate([elems, nbr[nbr >= 0]]))
    bp = Blocks(grid, refs, None, elems=patch)
    be = Blocks(grid, refs, D, elems=elems)
    c = C.reshape(-1)
    inv = np.linalg.inv(refs.hatM)
    Zfull = []
    for m in range(2):
        AC = ((-bp.H[m] + bp.Q[m] + bp.QN[m]) @ c).reshape(len(patch), N)
        if J is not None:
            AC = AC + J[m][patch]
        Zp = -(AC @ inv.T) / (2 * grid.areaT[patch])[:, None]
        z = np.zeros((K, N))
        z[patch] = Zp
        Zfull.append(z)
    y = be.M @ c + tau * (eta * ((be.S + be.SD) @ c)
                          + sum((-be.G[m] + be.R[m] + be.RD[m]) @ Zfull[m].reshape(-1)
                                for m in range(2)))
    return y.reshape(len(elems), N), [Zfull[m][elems] for m in range(2)]
