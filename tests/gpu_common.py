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
