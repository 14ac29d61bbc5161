"""GPU parity of the FP64-accurate product on INT8 matrix cores (spin_gemm_int8)
against its definition in oracle.ozaki, bit for bit, through the C ABI, and
the Newton refinement built on it (mixed modes with SPIN_REFINE_INT8).

The emulated product is a deterministic function of its operands: the
integers each row and column round to, their exact product, one rounding and
the epilogue's one rounding.  The GPU forms the exact product from INT8
residue products and Chinese remaindering, so any slip in a residue, a
fragment layout, a carry or the final rounding changes bits."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import ozaki as OZ

pytestmark = pytest.mark.gpu

MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197]


def _log2M(count):
    return sum(math.log2(m) for m in MODULI[:count])


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401
    return torch


def _dev(torch, a, pad=0):
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    buf = torch.full((n, m + pad), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(a.T)).cuda()
    return buf.t()[:m, :] if pad else buf.t()


def _ld(t):
    return max(t.stride(1), 1)


def _run(torch, A, B, epi, C0=None, moduli=14, beta=0, pad=0):
    import paper_1801_04723_amd as S
    m, k = A.shape
    n = B.shape[1]
    dA, dB = _dev(torch, A, pad), _dev(torch, B, pad)
    dC = _dev(torch, C0, pad) if C0 is not None else None
    dD = _dev(torch, np.zeros((m, n)), pad + 3)
    S.gemm_int8(m, n, k, dA, _ld(dA), dB, _ld(dB), epi, dC, _ld(dC) if dC is not None else 1, dD,
                _ld(dD), moduli=moduli, beta_a=beta, beta_b=beta)
    torch.cuda.synchronize()
    return dD.cpu().numpy()


def _want(A, B, epi, C0, moduli, beta):
    k = A.shape[1]
    if beta <= 0:
        beta = min(53, OZ.beta_for(k, _log2M(moduli)))
    D = OZ.emulated_product(A, B, beta, beta)
    if epi == 1:
        return np.eye(D.shape[0]) - D
    if epi == 2:
        return C0 + D
    return D


def _same(x, y):
    return np.array_equal(x.view(np.int64), y.view(np.int64)) or \
        (np.array_equal(np.isnan(x), np.isnan(y)) and np.array_equal(x[~np.isnan(x)], y[~np.isnan(y)]))


SHAPES = [(1, 1, 1), (17, 33, 5), (64, 64, 64), (128, 128, 64), (130, 250, 70), (300, 257, 513),
          (256, 256, 1000)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_emulated_product_bitwise(torch_cuda, m, n, k, epi):
    if epi == 1 and m != n:
        n = m
    g = np.random.default_rng(m * 7 + n + k)
    A = g.standard_normal((m, k)) * np.exp2(g.integers(-20, 20, size=(m, 1)))
    B = g.standard_normal((k, n)) * np.exp2(g.integers(-20, 20, size=(1, n)))
    C0 = g.standard_normal((m, n)) if epi == 2 else None
    got = _run(torch_cuda, A, B, epi, C0, pad=2 if m > 100 else 0)
    assert _same(got, _want(A, B, epi, C0, 14, 0))


@pytest.mark.parametrize("moduli,beta", [(2, 0), (5, 0), (9, 20), (15, 0), (15, 53)])
def test_moduli_and_budgets(torch_cuda, moduli, beta):
    import paper_1801_04723_amd as S
    g = np.random.default_rng(moduli)
    m, n, k = 70, 90, 150
    A = g.standard_normal((m, k))
    B = g.standard_normal((k, n))
    if beta and 1 + math.log2(k) + 2 * beta >= _log2M(moduli):
        with pytest.raises(S.SpinError):
            _run(torch_cuda, A, B, 0, moduli=moduli, beta=beta)
        return
    assert _same(_run(torch_cuda, A, B, 0, moduli=moduli, beta=beta), _want(A, B, 0, None, moduli, beta))


def test_integer_data_exact_and_nonfinite(torch_cuda):
    g = np.random.default_rng(2)
    A = g.integers(-3000, 3000, size=(96, 200)).astype(float)
    B = g.integers(-3000, 3000, size=(200, 80)).astype(float)
    assert np.array_equal(_run(torch_cuda, A, B, 0), A @ B)
    A[5, 7] = np.nan
    B[3, 11] = np.inf
    got = _run(torch_cuda, A, B, 0)
    assert np.isnan(got[5]).all() and np.isnan(got[:, 11]).all()
    mask = np.ones_like(got, bool)
    mask[5] = False
    mask[:, 11] = False
    assert np.array_equal(got[mask], (np.nan_to_num(A) @ np.nan_to_num(B, posinf=0))[mask])


@pytest.mark.parametrize("m,n,k,epi", [(1030, 1290, 333, 0), (1100, 1100, 700, 1), (1024, 1536, 64, 2),
                                         (1023, 2049, 129, 0)])
def test_large_tile_ragged_sampled_rows(torch_cuda, m, n, k, epi):
    """Products with both sides of at least 1024 run on the 256 x 256 tile:
    ragged edges in m, n and k, sampled rows (every tile boundary and the
    last row) bit for bit against the definition."""
    g = np.random.default_rng(m + 3 * n + 7 * k)
    A = g.standard_normal((m, k)) * np.exp2(g.integers(-20, 20, size=(m, 1)))
    B = g.standard_normal((k, n)) * np.exp2(g.integers(-20, 20, size=(1, n)))
    C0 = g.standard_normal((m, n)) if epi == 2 else None
    got = _run(torch_cuda, A, B, epi, C0, pad=1)
    rows = np.unique(np.concatenate([[0, 127, 128, 255, 256, 511, 512, m - 1],
                                     g.choice(m, 4, replace=False)]))
    beta = min(53, OZ.beta_for(k, _log2M(14)))
    D = OZ.emulated_product(A[rows], B, beta, beta)
    if epi == 1:
        want = np.eye(m, n)[rows] - D
    elif epi == 2:
        want = C0[rows] + D
    else:
        want = D
    assert _same(got[rows], want)


def test_full_size_sampled_rows(torch_cuda):
    """Order 4096, the refinement's residual shape: sampled rows bit for bit
    (a row's shift depends only on that row, a column's on that column)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 4096
    A = W.diag_dominant(n, seed=41)
    X = np.linalg.inv(A)
    dA, dX = _dev(torch, A), _dev(torch, X)
    dR = torch.empty_like(dA)
    S.gemm_int8(n, n, n, dA, n, dX, n, 1, None, 1, dR, n)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(0).choice(n, 3, replace=False))
    R = dR[rows, :].cpu().numpy()
    beta = min(53, OZ.beta_for(n, _log2M(14)))
    want = np.eye(n)[rows] - OZ.emulated_product(A[rows], X, beta, beta)
    assert _same(R, want)


@pytest.mark.parametrize("mode,steps", [("fp32_int8", 2), ("bf16x3_int8", 3)])
def test_refinement_on_int8(torch_cuda, mode, steps):
    """Mixed inversion refined with emulated products reaches rho <= 1e-12
    (checked on the device and by the oracle's residual) and agrees with the
    FP64-refined result."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(1024, seed=12, kappa=1e4)
    dA = _dev(torch, A)
    X, rep = S.invert_mixed(dA, leaf=128, mode=mode, ns_steps=steps, report=True)
    assert rep["status"] == 0, rep
    Xh = X.cpu().numpy()
    assert oracle.residual(A, Xh) <= 1e-12
    ref, info = oracle.strassen_inv(A, 128)
    assert info == 0
    assert np.linalg.norm(Xh - ref) / np.linalg.norm(ref) <= 100 * np.linalg.cond(A) * 2.0 ** -53
