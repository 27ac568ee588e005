"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

from inputs.fields import LOGNORMAL, LOGNORMAL_T, SMOOTH1, SMOOTH2, TABLE2, Workload, lognormal_blocks
from inputs.meshes import square_mesh


def rel_l2(area, A, B):
    """sqrt(sum_k |T_k| ||A_k - B_k||^2) / sqrt(sum_k |T_k| ||B_k||^2) (M_k = 2|T_k| I)."""
    A = np.asarray(A).reshape(len(area), -1)
    B = np.asarray(B).reshape(len(area), -1)
    num = np.sqrt(np.sum(area[:, None] * (A - B) ** 2))
    den = np.sqrt(np.sum(area[:, None] * B ** 2))
    return num / max(den, 1e-300)


def workload(kind, n_cells, seed=None, sigma=1.0, block=8):
    if kind in (LOGNORMAL, LOGNORMAL_T):
        blk = lognormal_blocks(n_cells, seed, sigma, block=block)
        return Workload(kind, n_cells=n_cells, blocks=blk, block=block)
    return Workload(kind)


def to_np(t):
    return t.detach().cpu().numpy()


def l2_sketch(area, X, rows=64, seed=0):
    """Gaussian sketch of the L2 norm of a discrete function: S v / sqrt(rows),
    with v_(k,i) = sqrt(2|T_k|) X_ki (so ||v|| = ||x_h||_L2 in an orthonormal
    basis) and S a [rows x K*N] matrix of independent standard normals drawn
    row by row from numpy default_rng([seed, row]).  ||sketch(X)|| estimates
    ||x_h||; for rows = 64 the ratio lies in [0.75, 1.25] with probability
    above 0.99 (chi-square with 64 degrees of freedom), and sketches are
    linear, so sketch(A) - sketch(B) estimates ||a_h - b_h||."""
    v = (np.sqrt(2.0 * np.asarray(area))[:, None] * np.asarray(X).reshape(len(area), -1)).reshape(-1)
    out = np.empty(rows)
    for j in range(rows):
        out[j] = np.random.default_rng([seed, j]).standard_normal(v.size) @ v
    return out / np.sqrt(rows)
