"""Analytic data of the benchmark problems (coefficients, sources, exact solutions).

Every field is a function of (t, x, y) on numpy arrays.  The same formulas
are evaluated on the GPU by the library's synthetic-workload sampler; the
two implementations are independent and agree to rounding.

Problem (Sec. 1.3, eq:diffusion:nonmixed): dt c - div(d grad c) = f with
Dirichlet data c_D = c and Neumann data g_N = -grad c . nu.  The
manufactured solution of the benchmark configurations is
c = cos(7x) cos(7y) exp(-t); f is derived from it exactly where d is smooth,
and inside each constant block where d is piecewise constant.

MAIN is the problem of the paper's main script (the template of Sec. 4): a
discontinuous coefficient (1.01 on the open square (1/4, 3/4)^2, 0.01
outside), f = 0.1 t, c_D = sin(2 pi y + t), g_N = y, c0 = sin(x) cos(y), with
Neumann edges at y = 0 and y = 1; it has no closed-form solution.
"""
import numpy as np

SMOOTH1, SMOOTH2, LOGNORMAL, LOGNORMAL_T, TABLE2, MAIN = 1, 2, 3, 4, 5, 6


def lognormal_blocks(n_cells, seed, sigma, block=8, contrast=1e3):
    """Block values exp(sigma*clip(xi, +-a)), a = ln(contrast)/(2 sigma), one per
    block x block cells of the n_cells x n_cells grid, indexed [bx, by]."""
    nb = -(-n_cells // block)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((nb, nb))
    a = np.log(contrast) / (2.0 * sigma)
    return np.exp(sigma * np.clip(xi, -a, a))       # [bx, by]


def triangle_values(blocks, n_cells, block=8):
    """Value of the block field on every triangle of the n_cells x n_cells
    Friedrichs-Keller mesh: a triangle takes the value of the block of cells
    its cell belongs to, so the field jumps only across mesh edges."""
    from .meshes import fk_cells
    ix, iy = fk_cells(n_cells)
    return np.ascontiguousarray(blocks[ix // block, iy // block], np.float64)


def position_values(blocks, n_cells, x, y, block=8):
    """The block field sampled by position: the value of the block of cells of
    the unjittered n_cells x n_cells grid that contains (x, y).  On a jittered
    mesh, triangles then straddle block boundaries and the field jumps inside
    them (the other reading of the block field)."""
    nb = blocks.shape[0]
    h = block / float(n_cells)
    bx = np.clip(np.floor(np.asarray(x) / h).astype(np.int64), 0, nb - 1)
    by = np.clip(np.floor(np.asarray(y) / h).astype(np.int64), 0, nb - 1)
    return np.ascontiguousarray(blocks[bx, by], np.float64)


class Workload:
    """Coefficient d, source f, boundary data c_D, g_N and exact c of one problem.

    Block-field kinds (LOGNORMAL, LOGNORMAL_T) are constant on each triangle:
    d(t, x, y) is then called with point arrays whose rows are the triangles
    of the mesh in order ([K x R])."""

    def __init__(self, kind, n_cells=1, blocks=None, block=8):
        self.kind = kind
        self.n_cells = n_cells
        self.blocks = None if blocks is None else np.ascontiguousarray(blocks, np.float64)
        self.block = block
        self.dT = None if blocks is None else triangle_values(self.blocks, n_cells, block)
        self.stationary = kind == TABLE2

    def restrict(self, elems):
        """The same workload seen on the triangles `elems` only (rows of point arrays)."""
        w = Workload(self.kind)
        w.n_cells, w.block, w.blocks = self.n_cells, self.block, self.blocks
        w.dT = None if self.dT is None else self.dT[np.asarray(elems)]
        return w

    # --- exact solution and its derivatives -------------------------------
    def c(self, t, x, y):
        if self.kind == MAIN:
            raise ValueError("the main-script problem has no closed-form solution")
        c = np.cos(7 * x) * np.cos(7 * y)
        return c if self.stationary else c * np.exp(-t)

    def grad_c(self, t, x, y):
        e = 1.0 if self.stationary else np.exp(-t)
        return (-7 * np.sin(7 * x) * np.cos(7 * y) * e,
                -7 * np.cos(7 * x) * np.sin(7 * y) * e)

    # --- diffusion coefficient and its gradient ----------------------------
    def _block_value(self, x, y):
        x = np.asarray(x)
        if x.ndim == 0 or x.shape[0] != self.dT.shape[0]:
            raise ValueError("block fields are sampled triangle by triangle: rows must be the K triangles")
        return self.dT.reshape((-1,) + (1,) * (x.ndim - 1)) * np.ones_like(x)

    def d(self, t, x, y):
        if self.kind == SMOOTH1:
            return 1 + 0.5 * np.sin(np.pi * x) * np.cos(np.pi * y) * np.exp(-t)
        if self.kind == SMOOTH2:
            return np.exp(0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)) * (1 + 0.1 * t)
        if self.kind == LOGNORMAL:
            return self._block_value(x, y)
        if self.kind == LOGNORMAL_T:
            return self._block_value(x, y) * (1 + 0.1 * np.sin(t))
        if self.kind == TABLE2:
            return np.exp(x + y)
        if self.kind == MAIN:
            inside = (x < 0.75) & (x > 0.25) & (y < 0.75) & (y > 0.25)
            return inside.astype(np.float64) + 0.01
        raise ValueError(self.kind)

    def grad_d(self, t, x, y):
        if self.kind == SMOOTH1:
            e = 0.5 * np.exp(-t) * np.pi
            return (e * np.cos(np.pi * x) * np.cos(np.pi * y),
                    -e * np.sin(np.pi * x) * np.sin(np.pi * y))
        if self.kind == SMOOTH2:
            dd = self.d(t, x, y) * np.pi
            return (dd * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y),
                    dd * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y))
        if self.kind in (LOGNORMAL, LOGNORMAL_T):
            z = np.zeros_like(x)
            return z, z
        if self.kind == TABLE2:
            e = np.exp(x + y)
            return e, e
        raise ValueError(self.kind)

    # --- derived data -------------------------------------------------------
    def f(self, t, x, y):
        if self.kind == MAIN:
            return 0.1 * t * np.ones_like(np.asarray(x, dtype=np.float64))
        c = self.c(t, x, y)
        dtc = 0.0 * c if self.stationary else -c
        lap = -98.0 * c
        gx, gy = self.grad_c(t, x, y)
        dx, dy = self.grad_d(t, x, y)
        return dtc - (dx * gx + dy * gy) - self.d(t, x, y) * lap

    def c_D(self, t, x, y):
        if self.kind == MAIN:
            return np.sin(2 * np.pi * y + t)
        return self.c(t, x, y)

    def g_N(self, t, x, y, nu1, nu2):
        if self.kind == MAIN:
            return np.asarray(y, dtype=np.float64) + 0.0 * nu1
        gx, gy = self.grad_c(t, x, y)
        return -(gx * nu1 + gy * nu2)

    def c0(self, x, y):
        if self.kind == MAIN:
            return np.sin(x) * np.cos(y)
        return self.c(0.0, x, y)
