"""The allocation-free operator apply (library workspace, no allocation)
against ldg_apply_schur, which uses the context's own buffers: the same kernels
in the same order, so the results must agree bit for bit.  Two calls in a row
on one device, the second with a smaller mesh (the workspace keeps the first
call's contents), and a mesh beyond the workspace's limit, rejected before
any launch."""
import numpy as np
import pytest

from inputs.meshes import NORTH, square_mesh

pytestmark = pytest.mark.gpu


def _ctx(n, p, seed, matrix_free=False):
    from paper_1408_3877_amd import Solver
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(NORTH,))
    s = Solver(cV, V0T, kind, p)
    rng = np.random.default_rng(seed)
    s.assemble(1.0 + 0.3 * rng.standard_normal((s.K, s.N)))
    if matrix_free:
        s.set_matrix_free(True)
    return s, rng.standard_normal((s.K, s.N))


@pytest.mark.parametrize("matrix_free", [False, True])
def test_noalloc_apply_matches_the_allocating_apply(matrix_free):
    import torch
    assert torch.cuda.is_available()
    for n, p, seed in ((40, 4, 901), (7, 2, 902)):     # second call smaller
        s, C = _ctx(n, p, seed, matrix_free)
        want = s.apply_schur(0.013, C)
        y = torch.full((s.K, s.N), float("nan"), dtype=torch.float64, device="cuda")
        s.apply_schur_noalloc(0.013, C, y)
        torch.cuda.synchronize()
        assert torch.equal(y, want), (n, p, float((y - want).abs().max()))


def test_noalloc_apply_rejects_meshes_beyond_the_workspace():
    import torch
    s, C = _ctx(265, 4, 903)
    kpad = (s.K + 63) // 64 * 64
    assert kpad * s.N > 2 ** 21                    # 140480 * 15 values per vector
    y = torch.zeros((s.K, s.N), dtype=torch.float64, device="cuda")
    from paper_1408_3877_amd.ldg import LdgError
    with pytest.raises(LdgError, match="allocation-free") as e:
        s.apply_schur_noalloc(0.01, C, y)
    assert e.value.code == -1                      # LDG_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(y) == 0
