"""Write the oracle's first two steps of the 256 x 256-cell, p = 3 workload.

Workload: the Friedrichs-Keller square of 256 x 256 cells (K = 131,072) with
interior vertices jittered (seed 1004); log-normal coefficient, one value per
8 x 8-cell block (sigma 1.5, field seed 4100), constant on every triangle;
forcing and Dirichlet data of c = cos 7x cos 7y e^-t; two implicit Euler steps
of dt = 1e-4 (eq:fullSystem of Sec. 2.5) from the projection of c(0).  The
eliminated system is symmetric positive definite here, and the oracle solves
it by block-Jacobi CG to a true relative residual of 1e-14 (the mesh is too
large for its sparse direct solve).

Stored (learned_p3_256.npz), per step:
  C, Z1, Z2 on 2048 triangles drawn with numpy default_rng(256);
  the L2 norms of c_h and of z_h;
  64-row Gaussian sketches of C, Z1 and Z2 (tests/gpu_common.l2_sketch).

Calls only oracle/, inputs/ and the sketch helper.  About 20 minutes:
  python tests/golden/make_learned_p3_256.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs.fields import LOGNORMAL, Workload, lognormal_blocks  # noqa: E402
from inputs.meshes import square_mesh  # noqa: E402
from oracle.ldg import Problem, step_schur_cg  # noqa: E402
from tests.gpu_common import l2_sketch  # noqa: E402

N_CELLS, P, JITTER, SIGMA, FIELD, DT, STEPS = 256, 3, 1004, 1.5, 4100, 1e-4, 2
N_SAMPLE = 2048


def main():
    t0 = time.perf_counter()
    coordV, V0T, kind = square_mesh(N_CELLS, seed=JITTER)
    pr = Problem(coordV, V0T, kind, P)
    w = Workload(LOGNORMAL, n_cells=N_CELLS,
                 blocks=lognormal_blocks(N_CELLS, FIELD, SIGMA, block=8), block=8)
    K = pr.grid.numT
    a = pr.grid.areaT
    sample = np.sort(np.random.default_rng(256).choice(K, N_SAMPLE, replace=False))
    C = pr.initial(w)
    out = {"sample": sample, "dt": DT, "steps": np.arange(1, STEPS + 1)}
    rec = {k: [] for k in ("C_s", "Z1_s", "Z2_s", "norm_c", "norm_z", "sk_C", "sk_Z1", "sk_Z2",
                           "iters", "rel_residual")}
    t = 0.0
    for n in range(1, STEPS + 1):
        t += DT
        C, Z1, Z2, info = step_schur_cg(pr, C, t, DT, w, rtol=1e-14)
        assert info["flag"] == 0, info["flag"]
        rec["C_s"].append(C[sample]); rec["Z1_s"].append(Z1[sample]); rec["Z2_s"].append(Z2[sample])
        rec["norm_c"].append(np.sqrt(np.sum(2 * a[:, None] * C ** 2)))
        rec["norm_z"].append(np.sqrt(np.sum(2 * a[:, None] * (Z1 ** 2 + Z2 ** 2))))
        for name, X in (("sk_C", C), ("sk_Z1", Z1), ("sk_Z2", Z2)):
            rec[name].append(l2_sketch(a, X))
        rec["iters"].append(info["iters"]); rec["rel_residual"].append(info["rel_residual"])
        print("step %d: %d CG iterations, residual %.2e, %.0f s" %
              (n, info["iters"], info["rel_residual"], time.perf_counter() - t0), flush=True)
    out.update({k: np.array(v) for k, v in rec.items()})
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "learned_p3_256.npz"), **out)


if __name__ == "__main__":
    main()
