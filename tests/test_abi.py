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
