"""GPU parity of spin_invert_lu (inversion through a block LU factorisation
without pivoting, the paper's comparison method) against O4, through the C ABI.

Tolerances as for spin_invert: forward error against the oracle
<= max(1e-13, 100 kappa u) and rho <= 1e-12; exact cases bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).T)).cuda().t()


def _host(t):
    return t.detach().cpu().numpy()


CASES = [("dd", 256, 64), ("spd", 200, 32), ("dd", 300, 64), ("spdk", 512, 64), ("dd", 128, 128),
         ("dd", 1000, 128), ("dd", 1, 1), ("spd", 640, 16)]


@pytest.mark.parametrize("kind,n,leaf", CASES)
def test_invert_lu_parity(torch_cuda, kind, n, leaf):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = {"dd": lambda: W.diag_dominant(n, n), "spd": lambda: W.spd_gram(n, n),
         "spdk": lambda: W.spd_spectrum(n, n, kappa=1e4)}[kind]()
    X = _host(S.invert_lu(_dev(torch, A), leaf=leaf))
    assert S.info() == 0
    ref, info = oracle.lu_inv(A, leaf)
    assert info == 0
    kap = np.linalg.cond(A)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * kap * U), (err, kap)
    assert oracle.residual(A, X) <= 1e-12


@pytest.mark.parametrize("n,leaf", [(32, 8), (64, 16), (130, 64)])
def test_invert_lu_exact_unimodular(torch_cuda, n, leaf):
    """L U with unit bidiagonal factors: integers throughout, so the exact
    rational inverse whatever the summation order."""
    import paper_1801_04723_amd as S
    from oracle.exact import exact_inverse, to_float
    torch = torch_cuda
    A = W.unimodular_bidiag(n, seed=n + leaf)
    X = _host(S.invert_lu(_dev(torch, A), leaf=leaf))
    assert S.info() == 0
    assert np.array_equal(X, to_float(exact_inverse(A)))


def test_invert_lu_reports_breakdown(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(256, seed=3)
    A[:, 200] = 0.0
    A[200, :] = 0.0
    S.invert_lu(_dev(torch, A), leaf=64)
    assert S.info() == 201


def test_invert_lu_full_size_8192(torch_cuda):
    """n = 8192, leaf 128, U(-1,1) + n I: residual and sampled columns, and
    agreement with spin_invert."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 8192
    dA = W.torch_diag_dominant(n, seed=3)
    X1 = S.invert_lu(dA, leaf=128)
    assert S.info() == 0
    assert S.residual(dA, X1) <= 1e-12
    X2 = S.invert(dA, leaf=128)
    assert float((X1 - X2).norm() / X2.norm()) <= 1e-13
    cols = torch.from_numpy(np.sort(np.random.default_rng(2).choice(n, 8, replace=False))).cuda()
    Xs = X1[:, cols].contiguous()
    E = torch.zeros_like(Xs)
    E[cols, torch.arange(len(cols), device="cuda")] = 1.0
    R = dA @ Xs - E
    assert float((R.norm(dim=0) / (dA.norm() * Xs.norm(dim=0))).max()) <= 1e-14
    del dA, X1, X2, Xs, E, R
    S.release()
    torch.cuda.empty_cache()
