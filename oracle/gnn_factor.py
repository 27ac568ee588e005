"""FP64 reference of the learned factored preconditioner (linear, SPD).

Test infrastructure, like the rest of the oracle; the device implementation in
the library is independent of it.

For a step whose eliminated operator S is symmetric positive definite (a
coefficient constant on every triangle), let BJ_k = S_kk be its diagonal
blocks and W_k = R_k^T with R_k the lower Cholesky factor of BJ_k^{-1}, so that
W_k^T W_k = BJ_k^{-1}.  The scaled operator W S W^T has identity diagonal
blocks; its blocks between neighbours k and j = k+ (across local edge n of k)
are O_kn = W_k S_kj W_j^T, with O_kn^T = O_{j n+} by the symmetry of S.  The
preconditioner is

    P = W^T (I + F)^T (I + F) W,     F_kj = -omega_kn O_kn,

symmetric positive definite whenever I + F is nonsingular, and equal to the
block-Jacobi inverse for omega = 0.  omega_kn in (0, OMEGA_MAX) comes from a
graph network over the element graph that sees the coefficient and the
geometry but not the residual: the encoder and the three message-passing
layers of oracle.gnn (node input without r_hat, N + 3 features), then per
directed interior edge

    omega_kn = OMEGA_MAX * sigmoid(h_k . w_hk + h_j . w_hj + e_kn . w_e
                                   + w_o log ||O_kn||_F + b_o).

The network runs once per system; every Krylov iteration applies the fixed
linear P, so preconditioned CG keeps its optimality.

Nonsymmetric steps (a coefficient that varies inside triangles) use the same
construction on the symmetric part of the operator: W_k from the Cholesky
factor of (BJ_k^{-1} + BJ_k^{-T}) / 2 and O_kn = W_k (S_kj + S_jk^T) / 2 W_j^T.
P is then SPD again (where those diagonal factors exist) and serves as a fixed
right preconditioner of GMRES.

Training losses, both 1 at omega = 0:

  Frobenius (the factorised-sparse-approximate-inverse objective): with
  G = (I + F) W and a probe vector w (Gaussian: a Hutchinson estimate of
  ||G S G^T - I||_F^2),
      loss = ||(G S G^T - I) w||^2 / ||(W S W^T - I) w||^2.

  Energy (on pairs from the method's own CG solves): for an error e (scaled
  by the RMS of BJ^{-1} r) and r = S e,
      loss = (P r - e)^T S (P r - e) / (BJ^{-1} r - e)^T S (BJ^{-1} r - e),
  the energy-norm error after one preconditioned step relative to
  block-Jacobi's.  Late CG errors are smooth, so this loss rewards amplifying
  smooth modes and drives omega towards its cap, where I + F comes close to
  singular on other modes; the Frobenius loss weighs every mode alike.
"""
import numpy as np
import scipy.sparse as sp

from oracle import gnn

OMEGA_MAX = 0.95
HEAD = [("w_hk", (gnn.WIDTH,)), ("w_hj", (gnn.WIDTH,)), ("w_e", (gnn.E_IN,)), ("w_o", ()),
        ("b_o", ())]


def param_shapes(N):
    """Trunk on node features only (N + 3 inputs), then the edge head."""
    return gnn.trunk_shapes(N + 3) + HEAD


def n_params(N):
    return gnn.n_params(N, param_shapes(N))


def init_params(N, seed, omega0=0.6):
    """Glorot-uniform weights from numpy's default_rng(seed), zero biases except
    b_o, set so that omega = omega0 where the other head terms vanish."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in param_shapes(N):
        if name.startswith("b_") or shp == ():
            d[name] = np.zeros(shp)
        elif len(shp) == 1:
            lim = np.sqrt(6.0 / (shp[0] + 1))
            d[name] = 0.1 * rng.uniform(-lim, lim, shp)
        else:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            d[name] = rng.uniform(-lim, lim, shp)
    q = omega0 / OMEGA_MAX
    d["b_o"] = np.array(np.log(q / (1.0 - q)))
    return gnn.pack(d, N, param_shapes(N))


class System:
    """The pieces of one system the preconditioner is built from."""

    def __init__(self, grid, S, symmetric_part=False):
        S = sp.csr_matrix(S)
        K = grid.numT
        N = S.shape[0] // K
        self.K, self.N, self.S = K, N, S
        Sb = sp.csr_matrix((S + S.T) * 0.5) if symmetric_part else S
        blk = lambda a, b: Sb[a * N:(a + 1) * N, b * N:(b + 1) * N].toarray()
        sblk = lambda a: S[a * N:(a + 1) * N, a * N:(a + 1) * N].toarray()
        self.BJinv = np.stack([np.linalg.inv(sblk(k)) for k in range(K)])
        chol_of = (lambda B: 0.5 * (B + B.T)) if symmetric_part else (lambda B: B)
        self.Wk = np.stack([np.linalg.cholesky(chol_of(B)).T for B in self.BJinv])   # W_k = R_k^T
        self.O = np.zeros((K, 3, N, N))
        self.mask = grid.kp >= 0
        for k in range(K):
            for n in range(3):
                j = grid.kp[k, n]
                if j >= 0:
                    self.O[k, n] = self.Wk[k] @ blk(k, j) @ self.Wk[j].T
        self.kp = grid.kp
        self.lognorm = np.where(self.mask, np.log(np.maximum(
            np.sqrt((self.O ** 2).sum(axis=(2, 3))), 1e-300)), 0.0)
        self.Wg = sp.block_diag(list(self.Wk)).tocsr()
        self.BJg = sp.block_diag(list(self.BJinv)).tocsr()

    def F(self, omega):
        """The global matrix F (blocks -omega_kn O_kn at (k, k+))."""
        K, N = self.K, self.N
        rows, cols, vals = [], [], []
        ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        for k in range(K):
            for n in range(3):
                j = self.kp[k, n]
                if j >= 0:
                    rows.append((k * N + ii).ravel())
                    cols.append((j * N + jj).ravel())
                    vals.append((-omega[k, n] * self.O[k, n]).ravel())
        if not rows:
            return sp.csr_matrix((K * N, K * N))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(K * N, K * N))

    def P(self, omega):
        """The preconditioner as a global sparse matrix."""
        G = (sp.eye(self.K * self.N) + self.F(omega)) @ self.Wg
        return (G.T @ G).tocsr()


def head_preactivation(P, hk, hj, e, lognorm):
    """h_k . w_hk + h_j . w_hj + e_kn . w_e + w_o log ||O_kn||_F + b_o (rows of edges)."""
    return hk @ P["w_hk"] + hj @ P["w_hj"] + e @ P["w_e"] + P["w_o"] * lognorm + P["b_o"]


def omega(theta, grid, node, edge, sysm, keep=False):
    """omega [K x 3] (0 on boundary edges) from the network."""
    N = sysm.N
    P = gnn.unpack(theta, N, param_shapes(N))
    h, acts = gnn.trunk_forward(P, grid, node, edge)
    kp = sysm.kp
    m = sysm.mask
    a = np.zeros((grid.numT, 3))
    for n in range(3):
        j = np.where(m[:, n], kp[:, n], 0)
        a[:, n] = head_preactivation(P, h, h[j], edge[:, n], sysm.lognorm[:, n])
    sig = 1.0 / (1.0 + np.exp(-a))
    om = np.where(m, OMEGA_MAX * sig, 0.0)
    if keep:
        return om, (P, h, acts, sig)
    return om


def energy_loss(theta, grid, node, edge, sysm, rhat, target):
    """Loss of one pair (rhat, target) as collected: e = target + rhat (scaled)."""
    e = (target + rhat).reshape(-1)
    r = sysm.S @ e
    d = sysm.P(omega(theta, grid, node, edge, sysm)) @ r - e
    d0 = sysm.BJg @ r - e
    return (d @ (sysm.S @ d)) / (d0 @ (sysm.S @ d0))


def _grad_through_z(theta, grid, node, edge, sysm, r, loss_of_z):
    """(loss, d loss / d theta) for a loss of z = P r: loss_of_z(z) gives (loss,
    d loss / dz); the chain rule runs through z = W^T (I + F)^T a, a = (I + F) y,
    y = W r."""
    N = sysm.N
    om, (P, h, acts, sig) = omega(theta, grid, node, edge, sysm, keep=True)
    Fm = sysm.F(om)
    I = sp.eye(sysm.K * N)
    y = sysm.Wg @ r
    a = (I + Fm) @ y
    z = sysm.Wg.T @ ((I + Fm).T @ a)
    L, v = loss_of_z(z)                        # v = dL/dz
    beta = sysm.Wg @ v                         # dL/db,  b = (I + F)^T a
    alpha = beta + Fm @ beta                   # dL/da
    # dL/dF_kj = a_k beta_j^T + alpha_k y_j^T ;  dL/domega_kn = -<dL/dF_kj, O_kn>
    K = sysm.K
    A_ = a.reshape(K, N)
    B_ = beta.reshape(K, N)
    Al = alpha.reshape(K, N)
    Y = y.reshape(K, N)
    dom = np.zeros((K, 3))
    for n in range(3):
        j = np.where(sysm.mask[:, n], sysm.kp[:, n], 0)
        Ob = sysm.O[:, n]
        dom[:, n] = -(np.einsum("ki,kij,kj->k", A_, Ob, B_[j])
                      + np.einsum("ki,kij,kj->k", Al, Ob, Y[j]))
    return L, _head_backward(theta, grid, edge, sysm, P, h, acts, sig, dom)


def energy_loss_grad(theta, grid, node, edge, sysm, rhat, target):
    """(loss, d loss / d theta) by the chain rule."""
    S = sysm.S
    e = (target + rhat).reshape(-1)
    r = S @ e
    d0 = sysm.BJg @ r - e
    den = d0 @ (S @ d0)

    def f(z):
        d = z - e
        Sd = S @ d
        return (d @ Sd) / den, 2.0 * Sd / den
    return _grad_through_z(theta, grid, node, edge, sysm, r, f)


def optstep_loss(theta, grid, node, edge, sysm, rhat, target):
    """Energy left after one preconditioned step with the best step length,
    relative to the error's energy:  min_t ||e - t P r||_S^2 / ||e||_S^2
    = 1 - (r^T P r)^2 / ((P r)^T S (P r) e^T r),  r = S e, e = target + rhat.
    Scaling e or P leaves it unchanged, as it leaves CG's iterates."""
    e = (target + rhat).reshape(-1)
    r = sysm.S @ e
    z = sysm.P(omega(theta, grid, node, edge, sysm)) @ r
    return 1.0 - (r @ z) ** 2 / ((z @ (sysm.S @ z)) * (e @ r))


def optstep_loss_grad(theta, grid, node, edge, sysm, rhat, target):
    """(loss, d loss / d theta): with s = r^T z, q = z^T S z, c = e^T r,
    d loss / dz = -2 s / (q c) r + 2 s^2 / (q^2 c) S z."""
    S = sysm.S
    e = (target + rhat).reshape(-1)
    r = S @ e
    c = e @ r

    def f(z):
        Sz = S @ z
        s_, q = r @ z, z @ Sz
        return 1.0 - s_ * s_ / (q * c), -2.0 * s_ / (q * c) * r + 2.0 * s_ * s_ / (q * q * c) * Sz
    return _grad_through_z(theta, grid, node, edge, sysm, r, f)


def _head_backward(theta, grid, edge, sysm, P, h, acts, sig, dom):
    """Gradient of the loss from d loss / d omega (K x 3) through head and trunk."""
    N = sysm.N
    da = np.where(sysm.mask, dom, 0.0) * OMEGA_MAX * sig * (1.0 - sig)
    G = {k: np.zeros_like(v_) for k, v_ in P.items()}
    dh = np.zeros_like(h)
    for n in range(3):
        m = sysm.mask[:, n]
        j = sysm.kp[m, n]
        dn = da[m, n]
        G["w_hk"] = G["w_hk"] + h[m].T @ dn
        G["w_hj"] = G["w_hj"] + h[j].T @ dn
        G["w_e"] = G["w_e"] + edge[m, n].T @ dn
        G["w_o"] = G["w_o"] + sysm.lognorm[m, n] @ dn
        G["b_o"] = G["b_o"] + dn.sum()
        dh[m] += dn[:, None] * P["w_hk"][None, :]
        np.add.at(dh, j, dn[:, None] * P["w_hj"][None, :])
    gnn.trunk_backward(P, grid, edge, acts, dh, G)
    return gnn.pack(G, N, param_shapes(N))


def frobenius_loss(theta, grid, node, edge, sysm, w):
    """||(G S G^T - I) w||^2 / ||(W S W^T - I) w||^2 for a probe w (K x N)."""
    w = w.reshape(-1)
    om = omega(theta, grid, node, edge, sysm)
    G = (sp.eye(sysm.K * sysm.N) + sysm.F(om)) @ sysm.Wg
    r = G @ (sysm.S @ (G.T @ w)) - w
    r0 = sysm.Wg @ (sysm.S @ (sysm.Wg.T @ w)) - w
    return (r @ r) / (r0 @ r0)


def frobenius_loss_grad(theta, grid, node, edge, sysm, w):
    """(loss, d loss / d theta): with u = G^T w, y = W S u, v = (I + F) y,
    g = 2 (v - w) / den and beta = W S W^T (I + F)^T g,
    d loss / d F_kj = g_k y_j^T + w_k beta_j^T."""
    K, N = sysm.K, sysm.N
    w = w.reshape(-1)
    om, (P, h, acts, sig) = omega(theta, grid, node, edge, sysm, keep=True)
    Fm = sysm.F(om)
    I = sp.eye(K * N)
    Wg, S = sysm.Wg, sysm.S
    u = Wg.T @ ((I + Fm).T @ w)
    y = Wg @ (S @ u)
    v = (I + Fm) @ y
    r0 = Wg @ (S @ (Wg.T @ w)) - w
    den = r0 @ r0
    L = ((v - w) @ (v - w)) / den
    g = 2.0 * (v - w) / den
    beta = Wg @ (S @ (Wg.T @ ((I + Fm).T @ g)))
    Wv, Y, Gv, Bv = (x.reshape(K, N) for x in (w, y, g, beta))
    dom = np.zeros((K, 3))
    for n in range(3):
        j = np.where(sysm.mask[:, n], sysm.kp[:, n], 0)
        Ob = sysm.O[:, n]
        dom[:, n] = -(np.einsum("ki,kij,kj->k", Gv, Ob, Y[j])
                      + np.einsum("ki,kij,kj->k", Wv, Ob, Bv[j]))
    return L, _head_backward(theta, grid, edge, sysm, P, h, acts, sig, dom)
