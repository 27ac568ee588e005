"""MI355X-native LDG diffusion hot path (arXiv 1408.3877): C-ABI library + thin binding.

The computation runs in the HIP library ``libldg.so`` built from ``csrc/``
(``python -m paper_1408_3877_amd.build``); this package only marshals
arguments.  Importing the binding fails loudly when the library is missing.
"""
from .ldg import (LDG_FP64, LDG_MIXED_BF16, LDG_MIXED_FP32, LdgError, Solver, edge_kinds_from_ids,
                  library_path, load_library, read_mesh_medit)

__all__ = ["Solver", "LdgError", "load_library", "library_path", "read_mesh_medit",
           "edge_kinds_from_ids", "LDG_FP64", "LDG_MIXED_FP32", "LDG_MIXED_BF16"]
