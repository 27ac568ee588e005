"""FP64 reference of the graph-network preconditioner (forward and backward).

The network acts on the element graph of the mesh: nodes are triangles,
directed edges join a triangle to each neighbour across an interior edge.
It maps a normalised block-Jacobi-preconditioned residual to a correction
of the block-Jacobi step:  P(r) = BJ^{-1} r + rho g(BJ^{-1} r / rho),  rho the
RMS of BJ^{-1} r.  Widths are 32; all activations are ReLU.

  node input  x_k = [ r_hat_k (N), log dbar_k, D_k[1:] / D_k0 (N-1),
                      log(|T_k| / mean|T|), log(dt dbar_k / |T_k|), eta ]     (2N+3)
  edge input  e_kj = [ nu_kn (2), log(|E_kn| / sqrt(mean|T|)),
                       one-hot(3 n + n+) (9), log(dbar_j / dbar_k) ]           (13)
  h0  = relu(x W_enc + b_enc)
  layer l = 1..3:  p_{j->k} = h_j W_m + e_kj W_e + b_m,   a_k = sum_j relu(p_{j->k})
                   u_k = [h_k, a_k] W_u + b_u,             h_k <- h_k + relu(u_k)
  g   = h3 W_dec + b_dec
  loss = mean over (k, i) of (g_ki - target_ki)^2

dbar_k = sqrt(2) D_k0 is the mean of d_h on T_k (phi_1 = sqrt(2)).

This module is test infrastructure like the rest of the oracle; the device
implementation in the library is independent of it.
"""
import numpy as np

WIDTH = 32
E_IN = 13
LAYERS = 3


def n_in(N):
    return 2 * N + 3


def trunk_shapes(n_input):
    """(name, shape) list of the encoder and the message-passing layers."""
    W = WIDTH
    shapes = [("W_enc", (n_input, W)), ("b_enc", (W,))]
    for l in range(LAYERS):
        shapes += [("W_m%d" % l, (W, W)), ("W_e%d" % l, (E_IN, W)), ("b_m%d" % l, (W,)),
                   ("W_u%d" % l, (2 * W, W)), ("b_u%d" % l, (W,))]
    return shapes


def param_shapes(N):
    """Ordered (name, shape) list of the flat parameter vector."""
    return trunk_shapes(n_in(N)) + [("W_dec", (WIDTH, N)), ("b_dec", (N,))]


def n_params(N, shapes=None):
    return sum(int(np.prod(s)) for _, s in (shapes or param_shapes(N)))


def unpack(theta, N, shapes=None):
    out, o = {}, 0
    for name, shp in (shapes or param_shapes(N)):
        sz = int(np.prod(shp))
        out[name] = theta[o:o + sz].reshape(shp)
        o += sz
    return out


def pack(d, N, shapes=None):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1)
                           for name, _ in (shapes or param_shapes(N))])


def init_params(N, seed):
    """Glorot-uniform weights, zero biases, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in param_shapes(N):
        if name.startswith("b_"):
            d[name] = np.zeros(shp)
        else:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            d[name] = rng.uniform(-lim, lim, shp)
    return pack(d, N)


def features(grid, D, dt, eta):
    """Node context features [K x (N+3)] (everything but r_hat) and edge features
    [K x 3 x 13] (zero rows for boundary edges)."""
    K, N = D.shape
    dbar = np.sqrt(2.0) * D[:, 0]
    meanA = grid.areaT.mean()
    rel = D[:, 1:] / D[:, :1]
    node = np.concatenate([np.log(np.abs(dbar))[:, None], rel,
                           np.log(grid.areaT / meanA)[:, None],
                           np.log(dt * np.abs(dbar) / grid.areaT)[:, None],
                           np.full((K, 1), eta)], axis=1)
    edge = np.zeros((K, 3, E_IN))
    for n in range(3):
        kp = grid.kp[:, n]
        m = kp >= 0
        edge[m, n, 0:2] = grid.nuE0T[m, n]
        edge[m, n, 2] = np.log(grid.areaE0T[m, n] / np.sqrt(meanA))
        edge[m, n, 3 + 3 * n + grid.np_[m, n]] = 1.0
        edge[m, n, 12] = np.log(np.abs(dbar[kp[m]]) / np.abs(dbar[m]))
    return node, edge


def forward(theta, grid, node, edge, rhat, keep=False):
    """g [K x N]; with keep=True also the activations backward() needs."""
    K, N = rhat.shape
    P = unpack(theta, N)
    h, acts = trunk_forward(P, grid, np.concatenate([rhat, node], axis=1), edge)
    g = h @ P["W_dec"] + P["b_dec"]
    return (g, acts) if keep else g


def trunk_forward(P, grid, x, edge):
    """Node states h [K x 32] after the encoder and the layers, and the activations."""
    K = x.shape[0]
    relu = lambda z: np.maximum(z, 0.0)
    z0 = x @ P["W_enc"] + P["b_enc"]
    h = relu(z0)
    acts = {"x": x, "z0": z0, "h": [h], "p": [], "a": [], "u": []}
    for l in range(LAYERS):
        a = np.zeros((K, WIDTH))
        ps = []
        for n in range(3):
            kp = grid.kp[:, n]
            m = kp >= 0
            p = np.zeros((K, WIDTH))
            p[m] = h[kp[m]] @ P["W_m%d" % l] + edge[m, n] @ P["W_e%d" % l] + P["b_m%d" % l]
            a[m] += relu(p[m])
            ps.append(p)
        u = np.concatenate([h, a], axis=1) @ P["W_u%d" % l] + P["b_u%d" % l]
        h = h + relu(u)
        acts["p"].append(ps)
        acts["a"].append(a)
        acts["u"].append(u)
        acts["h"].append(h)
    return h, acts


def loss(theta, grid, node, edge, rhat, target):
    g = forward(theta, grid, node, edge, rhat)
    return np.mean((g - target) ** 2)


def energy_loss(theta, grid, node, edge, rhat, target, S):
    """(g - t)^T S (g - t) / (t^T S t): the A-norm error of the corrected step
    relative to the block-Jacobi step (S the eliminated operator)."""
    d = (forward(theta, grid, node, edge, rhat) - target).reshape(-1)
    t = target.reshape(-1)
    return (d @ (S @ d)) / (t @ (S @ t))


def energy_loss_grad(theta, grid, node, edge, rhat, target, S):
    g = forward(theta, grid, node, edge, rhat)
    d = (g - target).reshape(-1)
    t = target.reshape(-1)
    den = t @ (S @ t)
    Sd = S @ d
    dg = (2.0 * Sd / den).reshape(g.shape)      # S symmetric
    return (d @ Sd) / den, backward(theta, grid, node, edge, rhat, dg)


def loss_grad(theta, grid, node, edge, rhat, target):
    """(loss, d loss / d theta) by the chain rule through forward()."""
    g = forward(theta, grid, node, edge, rhat)
    L = np.mean((g - target) ** 2)
    return L, backward(theta, grid, node, edge, rhat, 2.0 * (g - target) / g.size)


def backward(theta, grid, node, edge, rhat, dg):
    """d (loss) / d theta given d loss / d g, by the chain rule through forward()."""
    K, N = rhat.shape
    P = unpack(theta, N)
    g, A = forward(theta, grid, node, edge, rhat, keep=True)
    G = {k: np.zeros_like(v) for k, v in P.items()}
    h3 = A["h"][LAYERS]
    G["W_dec"] = h3.T @ dg
    G["b_dec"] = dg.sum(0)
    trunk_backward(P, grid, edge, A, dg @ P["W_dec"].T, G)
    return pack(G, N)


def trunk_backward(P, grid, edge, A, dh, G):
    """Accumulate the trunk parameters' gradients into G given d loss / d h3."""
    K = dh.shape[0]
    for l in reversed(range(LAYERS)):
        h = A["h"][l]
        a = A["a"][l]
        u = A["u"][l]
        du = dh * (u > 0)
        G["W_u%d" % l] = np.concatenate([h, a], axis=1).T @ du
        G["b_u%d" % l] = du.sum(0)
        dcat = du @ P["W_u%d" % l].T
        dh_prev = dh + dcat[:, :WIDTH]
        da = dcat[:, WIDTH:]
        for n in range(3):
            kp = grid.kp[:, n]
            m = kp >= 0
            p = A["p"][l][n]
            dp = np.zeros((K, WIDTH))
            dp[m] = da[m] * (p[m] > 0)
            G["W_m%d" % l] += h[kp[m]].T @ dp[m]
            G["W_e%d" % l] += edge[m, n].T @ dp[m]
            G["b_m%d" % l] += dp[m].sum(0)
            np.add.at(dh_prev, kp[m], dp[m] @ P["W_m%d" % l].T)
        dh = dh_prev
    dz0 = dh * (A["z0"] > 0)
    G["W_enc"] = A["x"].T @ dz0
    G["b_enc"] = dz0.sum(0)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
