"""GPU checks of the 64x64 diagonal-block factorisation of the blocked
FP64 Cholesky (factor and inverse of the factor, the critical path of
the gain), in both forms: the pivot sweep and the hierarchical form
(16-pivot sweeps in one wave, panels, trailing updates and the inverse's
off-diagonal blocks on FP64 MFMA).  Reference: LAPACK's Cholesky factor
and the explicit inverse (numpy), and the first non-positive pivot of the
unblocked elimination."""

import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _run(which, a):
    import paper_2012_10091_amd as m
    lib = m.load_library()
    ad = torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    L = torch.full((64, 64), 7.0, dtype=torch.float64, device="cuda")
    Li = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.menkf_test_chol_diag(which, ctypes.c_void_p(ad.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                                    ctypes.c_void_p(Li.data_ptr()), ctypes.c_void_p(info.data_ptr()), None, s) == 0
    torch.cuda.synchronize()
    return L.cpu().numpy(), Li.cpu().numpy(), int(info.item())


def _spd(seed, cond=1.0):
    rs = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rs.standard_normal((64, 64)))
    ev = np.geomspace(1.0, 1.0 / cond, 64)
    return (q * ev) @ q.T


@pytest.mark.parametrize("which", [0, 1], ids=["sweep", "hierarchical"])
@pytest.mark.parametrize("seed,cond", [(1, 1.0), (2, 1e3), (3, 1e7)])
def test_factor_and_inverse(which, seed, cond):
    a = _spd(seed, cond)
    say(f"diag block which={which} seed={seed} cond={cond:g}")
    L, Li, info = _run(which, a)
    assert info == 0
    Lr = np.linalg.cholesky(a)
    tril = np.tril(np.ones((64, 64), dtype=bool))
    # the factor (lower triangle written; the upper one untouched)
    assert np.abs(L[tril] - Lr[tril]).max() <= 1e-13 * cond ** 0.5 * np.abs(Lr).max()
    assert np.all(L[~tril] == 7.0)
    # the inverse of the factor, zeros above the diagonal
    Lir = np.linalg.inv(Lr)
    assert np.all(Li[~tril] == 0.0)
    assert np.abs(Li - Lir).max() <= 1e-13 * cond * np.abs(Lir).max()


@pytest.mark.parametrize("which", [0, 1], ids=["sweep", "hierarchical"])
@pytest.mark.parametrize("j", [0, 1, 5, 14, 16, 37, 63])
def test_first_nonpositive_pivot_is_reported(which, j):
    """A block whose pivot j (0-based) of the elimination is negative: the
    status is j + 1 and the outputs are left untouched."""
    a = _spd(11)
    Lr = np.linalg.cholesky(a)
    a[j, j] -= Lr[j, j] ** 2 + 0.5    # the j-th Schur pivot becomes -0.5
    say(f"non-SPD diag block which={which} pivot {j}")
    L, Li, info = _run(which, a)
    assert info == j + 1
    assert np.all(L == 7.0) and np.all(Li == 0.0)
