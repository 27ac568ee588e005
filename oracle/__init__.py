"""Plain, slow FP64 CPU oracle of the LDG diffusion hot path (Frank, Reuter,
Aizinger, Knabner: "FESTUNG ... Part I: Diffusion operator", arXiv 1408.3877).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the GPU path: its inputs come from the separate
``inputs`` package, and every formula here is written from the paper:

* basis.py       modal orthonormal basis (Sec. 2.4.1)
* quadrature.py  Gauss rules on [0,1] and on the reference triangle (Sec. 3.3)
* refelem.py     edge maps gamma/theta and reference tensors (Sec. 3.6)
* mesh.py        grid lists of Table 1 (Sec. 3.1)
* ldg.py         L2 projection, global blocks, implicit Euler step (Sec. 2, 3)

Every function is pinned by the "not gpu" tests to values or properties the
paper or the mathematics fix (see tests/test_oracle_*.py).
"""
