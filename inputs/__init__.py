"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds no arithmetic of the LDG method itself: it only builds
meshes (vertex coordinates, triangle vertex lists, boundary kinds) and the
analytic coefficient / solution fields of the benchmark problems, plus the
seeded random numbers those fields draw.  Both the oracle and the HIP path
take their inputs from here and from nowhere else.
"""
