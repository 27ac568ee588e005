"""Write the oracle trajectory of the 64 x 64-cell, p = 2 workload.

Workload: the Friedrichs-Keller square of 64 x 64 cells with interior vertices
jittered (seed 1002), smooth coefficient d = exp(sin(2 pi x) sin(2 pi y) / 2)
(1 + t / 10), manufactured solution c = cos 7x cos 7y e^-t with Dirichlet data
on every side, 100 implicit Euler steps of dt = 1e-3 (eq:fullSystem of
Sec. 2.5).  Every step is solved by the oracle's sparse direct solve of the
system with Z eliminated (an exact reduction of the full 3KN system).

Stored (plain_p2_64.npz):
  C, Z1, Z2 at steps 1 and 100 in full (K x N);
  C, Z1, Z2 at every step on 128 triangles drawn with numpy default_rng(64);
  the L2 norms of c_h and of (z1, z2) at every step.

Calls only oracle/ and inputs/.  About 15 minutes on one core:
  python tests/golden/make_plain_p2_64.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs.fields import SMOOTH2, Workload  # noqa: E402
from inputs.meshes import square_mesh  # noqa: E402
from oracle.ldg import Problem, step_schur  # noqa: E402

N_CELLS, P, JITTER, DT, STEPS = 64, 2, 1002, 1e-3, 100
FULL_STEPS = (1, 100)
N_SAMPLE = 128


def main():
    coordV, V0T, kind = square_mesh(N_CELLS, seed=JITTER)
    pr = Problem(coordV, V0T, kind, P)
    w = Workload(SMOOTH2)
    K = pr.grid.numT
    sample = np.sort(np.random.default_rng(64).choice(K, N_SAMPLE, replace=False))
    a = pr.grid.areaT
    C = pr.initial(w)
    out = {"sample": sample, "steps": np.arange(1, STEPS + 1), "dt": DT}
    Cs, Z1s, Z2s, nc, nz = [], [], [], [], []
    t = 0.0
    t0 = time.perf_counter()
    for n in range(1, STEPS + 1):
        t += DT
        C, Z1, Z2, _ = step_schur(pr, C, t, DT, w)
        Cs.append(C[sample]); Z1s.append(Z1[sample]); Z2s.append(Z2[sample])
        nc.append(np.sqrt(np.sum(2 * a[:, None] * C ** 2)))
        nz.append(np.sqrt(np.sum(2 * a[:, None] * (Z1 ** 2 + Z2 ** 2))))
        if n in FULL_STEPS:
            out["C_%d" % n], out["Z1_%d" % n], out["Z2_%d" % n] = C, Z1, Z2
        print("step %d  t=%.3f  %.1f s" % (n, t, time.perf_counter() - t0), flush=True)
    out.update(C_s=np.array(Cs), Z1_s=np.array(Z1s), Z2_s=np.array(Z2s),
               norm_c=np.array(nc), norm_z=np.array(nz))
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "plain_p2_64.npz"), **out)


if __name__ == "__main__":
    main()
