"""The entry point that allocates no device memory (tsk_rsvd_solve_noalloc):
through the C ABI its results equal those of tsk_rsvd_solve (same kernels,
scratch from the library's static per-GPU buffer instead of a workspace), on
two calls in a row whose second input is smaller, and a shape whose scratch
exceeds the buffer is refused before any work."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import paper_2104_01101_amd as t
    t.lib()  # fail loudly if the library is missing
    return t


def _case(m, r, s, R, k, seed, dtype=torch.float64):
    rs = np.random.default_rng(seed)
    Z = torch.from_numpy(rs.standard_normal((m, r))).to(DEV).to(dtype)
    Y = torch.from_numpy(rs.standard_normal((m, r)) @ rs.standard_normal((r, s))
                         + 0.1 * rs.standard_normal((m, s))).to(DEV).to(dtype)
    Om = torch.from_numpy(rs.standard_normal((s, k))).to(DEV)
    return Z, Y, R, Om


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_equals_workspace_solve_twice(tsk, dtype):
    """r = 256 (block-swept Gram, products with Y in the O(m s k) order), then
    r = 100 (the fused one-workgroup chain) on the same static buffer."""
    for shape, seed in (((2048, 256, 1500, 16, 26), 1), ((300, 100, 400, 10, 20), 2)):
        Z, Y, R, Om = _case(*shape, seed, dtype)
        A0, W0 = tsk.rsvd_solve(Z, Y, R, Om)
        A1, W1 = tsk.rsvd_solve_noalloc(Z, Y, R, Om)
        torch.cuda.synchronize()
        assert torch.equal(A0, A1) and torch.equal(W0, W1), shape


def test_noalloc_refuses_oversized_shape(tsk):
    """r = 1200 needs more than the 32 MiB buffer (the Gram, its inverse and
    the sweep partner alone are 3 r^2 doubles): ENOMEM, nothing written."""
    from paper_2104_01101_amd import _lib as L
    Z, Y, R, Om = _case(2400, 1200, 50, 4, 12, 3)
    with pytest.raises(L.TskError) as e:
        tsk.rsvd_solve_noalloc(Z, Y, R, Om)
    assert e.value.status == L.ENOMEM and "static buffer" in str(e.value)
