"""The C-ABI library loads and exports every entry point include/ldg.h declares."""
import os
import re
import ctypes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ldg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1408_3877_amd import build
    from paper_1408_3877_amd.ldg import library_path
    if not os.path.exists(library_path()):
        build.build()
    lib = ctypes.CDLL(library_path())
    names = _declared()
    assert "ldg_step_sampled" in names and "ldg_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1408_3877_amd import ldg
    bound = set(ldg._SIGS) | {"ldg_destroy", "ldg_last_error"}
    assert set(_declared()) <= bound


def test_sampled_inputs_are_checked_before_any_library_call():
    # the sampled-data entry points take raw device pointers: the binding must
    # reject a wrong length or dtype itself (host-only: a bare binding object
    # with no context and the CPU as its device)
    import numpy as np
    import pytest
    import torch

    from paper_1408_3877_amd.ldg import Solver
    s = object.__new__(Solver)
    s.torch, s.device = torch, torch.device("cpu")
    s.K, s.N, s.R, s.R1, s.n_bnd = 10, 3, 3, 2, 4
    good_v, good_b = np.zeros(30), np.zeros(8)
    d, f, cD, gN = s._sampled_inputs(good_v, torch.zeros(30, dtype=torch.float32), good_b, None)
    assert d.dtype == f.dtype == cD.dtype == torch.float64 and gN is None
    with pytest.raises(ValueError):
        s._sampled_inputs(np.zeros(29), good_v, good_b, good_b)
    with pytest.raises(ValueError):
        s._sampled_inputs(good_v, good_v, np.zeros(9), good_b)
    with pytest.raises(ValueError):
        s._sampled_inputs(good_v, good_v, None, np.zeros((2, 4)))
    with pytest.raises(TypeError):
        s._sampled_inputs(torch.zeros(30, dtype=torch.int64), good_v, None, None)
