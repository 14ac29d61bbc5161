"""GPU parity of spin_invert_spd (per node: II, the lower halves of S and C11
with their mirrors, C21 and the transpose C12 = C21^T) against O3, the
oracle's symmetric specialisation of Alg. 1, through the C ABI.

Tolerances as for spin_invert: forward error against the oracle
<= max(1e-13, 100 kappa u) and rho <= 1e-12 (<= 1e-14 at kappa = 1e4, where
an asymmetric S or C11 passed on would leave about 2e-13).  Exact cases bit
for bit; the result exactly symmetric outside the leaf blocks.
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


def _gen(kind, n):
    if kind == "spd":
        return W.spd_gram(n, seed=n)
    if kind == "spdk":
        return W.spd_spectrum(n, seed=n, kappa=1e4)
    raise ValueError(kind)


CASES = [
    ("spd", 256, 64),
    ("spd", 200, 32),     # ragged split
    ("spd", 513, 64),     # ragged, odd order
    ("spd", 1024, 256),   # blocked-leaf tier
    ("spdk", 512, 64),    # kappa = 1e4 spectrum
    ("spd", 2048, 512),
    ("spd", 640, 16),     # deep recursion, tiny leaves
    ("spd", 96, 96),      # a single leaf
    ("spd", 1, 1),
]


@pytest.mark.parametrize("kind,n,leaf", CASES)
def test_invert_spd_parity(torch_cuda, kind, n, leaf):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = _gen(kind, n)
    dA = _dev(torch, A)
    X = _host(S.invert_spd(dA, leaf=leaf))
    assert S.info() == 0
    ref, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    kap = np.linalg.cond(A)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * kap * U), (err, kap)
    rho = oracle.residual(A, X)
    assert rho <= (1e-14 if kind == "spdk" else 1e-12), rho
    if n > leaf:
        n1 = oracle.split(n)
        assert np.array_equal(X[:n1, n1:], X[n1:, :n1].T)
        if n1 > leaf:  # C11 of an internal node: lower half mirrored
            assert np.array_equal(X[:n1, :n1], X[:n1, :n1].T)


@pytest.mark.parametrize("n,leaf", [(32, 8), (64, 16), (130, 64)])
def test_invert_spd_exact_unimodular(torch_cuda, n, leaf):
    """L L^T with unit bidiagonal L: small integers throughout, so the result
    is the exact rational inverse whatever the summation order."""
    import paper_1801_04723_amd as S
    from oracle.exact import exact_inverse, to_float
    torch = torch_cuda
    A = W.spd_unimodular(n, seed=n + leaf)
    X = _host(S.invert_spd(_dev(torch, A), leaf=leaf))
    assert S.info() == 0
    assert np.array_equal(X, to_float(exact_inverse(A)))


def test_invert_spd_agrees_with_general_path(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(1024, seed=11)
    dA = _dev(torch, A)
    X1 = _host(S.invert(dA, leaf=128))
    X2 = _host(S.invert_spd(dA, leaf=128))
    assert np.linalg.norm(X2 - X1) / np.linalg.norm(X1) <= 100 * np.linalg.cond(A) * U


def test_invert_spd_reports_breakdown(torch_cuda):
    """A zero row and column in the second leaf: status = its global column."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(256, seed=3)
    A[:, 200] = 0.0
    A[200, :] = 0.0
    S.invert_spd(_dev(torch, A), leaf=64)
    assert S.info() == 201


def test_invert_spd_replay_and_padded_ld(torch_cuda):
    """Graph replay gives the first call's bits; padded leading dimensions
    leave the padding untouched."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n, lda, leaf = 600, 640, 128
    A = W.spd_gram(n, seed=9)
    Ap = np.full((lda, n), 7.0)
    Ap[:n] = A
    dA = _dev(torch, Ap)[:n]
    buf = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
    dX = buf.t()[:n]  # column-major, ld = lda
    S.invert_spd(dA, leaf=leaf, out=dX)
    first = _host(dX).copy()
    for _ in range(3):
        S.invert_spd(dA, leaf=leaf, out=dX)
    torch.cuda.synchronize()
    assert np.array_equal(_host(dX), first)
    assert torch.isnan(buf.t()[n:]).all()
    ref, _ = oracle.strassen_inv_spd(A, leaf)
    assert np.linalg.norm(first - ref) / np.linalg.norm(ref) <= 100 * np.linalg.cond(A) * U


def test_invert_spd_full_size_8192(torch_cuda):
    """The bench matrix B B^T/n + I at n = 8192, leaf 256: residual, sampled
    columns of A X = I with torch's own product, exact C12 = C21^T."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n, leaf = 8192, 256
    dA = _dev(torch, W.spd_gram(n, 2))
    dX = S.invert_spd(dA, leaf=leaf)
    assert S.info() == 0
    assert S.residual(dA, dX) <= 1e-12
    cols = torch.from_numpy(np.sort(np.random.default_rng(1).choice(n, 8, replace=False))).cuda()
    Xs = dX[:, cols].contiguous()
    E = torch.zeros_like(Xs)
    E[cols, torch.arange(len(cols), device="cuda")] = 1.0
    R = dA @ Xs - E
    assert float((R.norm(dim=0) / (dA.norm() * Xs.norm(dim=0))).max()) <= 1e-14
    h = n // 2
    assert torch.equal(dX[:h, h:], dX[h:, :h].t())
    assert torch.equal(dX[:h, :h], dX[:h, :h].t())
    del dA, dX, Xs, E, R
    S.release()
    torch.cuda.empty_cache()
