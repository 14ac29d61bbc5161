"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Tolerances (IEEE binary64, u = 2^-53; float32 u32 = 2^-24):
* block products: |D - D_ref| <= 4 (k + 2) u (|A| |B| + |C0|) elementwise,
  the standard bound for a length-k dot product plus the epilogue's roundings;
* inverses: relative residual rho <= 1e-12 and forward error against the
  oracle <= max(1e-13, 100 kappa u);
* exact cases (powers-of-two diagonal, permutation, block-diagonal zeros)
  bit for bit.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch


def _dev_f(torch, a, dtype=None):
    """Column-major device copy of a numpy matrix (returned as a transposed view)."""
    a = np.asarray(a)
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.t()  # shape (m, n), strides (1, m)


def _host(t):
    return t.detach().cpu().numpy()


def _kappa(a):
    return float(np.linalg.cond(a))


# ---------------------------------------------------------------- products
GEMM_CASES = [
    # m, n, k, alpha, beta, add_identity, pad (extra leading-dimension rows)
    (1, 1, 1, 1.0, 0.0, False, 0),
    (17, 33, 5, 1.0, 0.0, False, 1),
    (64, 64, 64, -1.0, 1.0, False, 0),
    (128, 128, 128, -1.0, 0.0, False, 3),
    (130, 250, 70, 1.0, 1.0, False, 0),
    (300, 257, 513, -1.0, 1.0, False, 5),
    (512, 512, 512, -1.0, 0.0, True, 0),
    (1000, 24, 700, 1.0, 0.0, False, 2),
    # 128-tile kernel: 16 x 16 tiles take the XCD block order, 16 x 12 the plain order
    (2048, 2048, 64, -1.0, 1.0, False, 0),
    (2048, 1536, 100, 1.0, 1.0, False, 3),
    # eight waves per workgroup: 128-tile with 240 tiles and a ragged n; 64-tile
    # with ragged m and n
    (1920, 2040, 96, -1.0, 1.0, False, 2),
    (1000, 1100, 64, 1.0, 1.0, False, 4),
    # 32-tile products with several K slabs: a ragged m and n, and a k that
    # is a multiple of 64 but not of 128
    (96, 130, 256, -1.0, 1.0, False, 2),
    (200, 64, 192, 1.0, 0.0, False, 0),
    (40, 40, 0, -1.0, 1.0, True, 0),
]


@pytest.mark.parametrize("case", GEMM_CASES)
def test_gemm_f64_parity(torch_cuda, case):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    m, n, k, alpha, beta, add_i, pad = case
    g = np.random.default_rng(m * 7 + n * 3 + k)
    A = g.uniform(-1, 1, size=(m + pad, k))
    B = g.uniform(-1, 1, size=(k + pad, n))
    C = g.uniform(-1, 1, size=(m + pad, n))
    dA, dB, dC = _dev_f(torch, A), _dev_f(torch, B), _dev_f(torch, C)
    dD = _dev_f(torch, np.full((m + pad, n), np.nan))
    S.gemm_cm(m, n, k, alpha, dA, m + pad, dB, k + pad, beta, dC if beta else None, m + pad,
              dD, m + pad, add_i, S.FP64)
    torch.cuda.synchronize()
    D = _host(dD)
    ref = alpha * oracle.gemm(A[:m], B[:k]) + beta * C[:m]
    if add_i:
        ref[np.arange(min(m, n)), np.arange(min(m, n))] += 1.0
    bound = 4 * (k + 2) * U * (np.abs(A[:m]) @ np.abs(B[:k]) + np.abs(C[:m]) + 1.0)
    assert np.all(np.abs(D[:m] - ref) <= bound)
    assert np.all(np.isnan(D[m:]))  # padding rows untouched


def test_gemm_in_place_c0_equals_d(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    m, n, k = 192, 320, 256
    g = np.random.default_rng(5)
    A, B, C = g.uniform(-1, 1, (m, k)), g.uniform(-1, 1, (k, n)), g.uniform(-1, 1, (m, n))
    dA, dB, dC = _dev_f(torch, A), _dev_f(torch, B), _dev_f(torch, C)
    S.gemm_cm(m, n, k, -1.0, dA, m, dB, k, 1.0, dC, m, dC, m, False, S.FP64)
    torch.cuda.synchronize()
    ref = C - oracle.gemm(A, B)
    bound = 4 * (k + 2) * U * (np.abs(A) @ np.abs(B) + np.abs(C))
    assert np.all(np.abs(_host(dC) - ref) <= bound)


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (200, 136, 300), (512, 512, 512), (1024, 1000, 96),
                                   (2048, 1920, 64)])
def test_gemm_f32_parity(torch_cuda, m, n, k):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    g = np.random.default_rng(m + n + k)
    A = g.uniform(-1, 1, (m, k)).astype(np.float32)
    B = g.uniform(-1, 1, (k, n)).astype(np.float32)
    C = g.uniform(-1, 1, (m, n)).astype(np.float32)
    dA, dB, dC = _dev_f(torch, A), _dev_f(torch, B), _dev_f(torch, C)
    dD = _dev_f(torch, np.zeros((m, n), np.float32))
    S.gemm_cm(m, n, k, -1.0, dA, m, dB, k, 1.0, dC, m, dD, m, False, S.MIXED_FP32)
    torch.cuda.synchronize()
    ref = C.astype(np.float64) - oracle.gemm(A.astype(np.float64), B.astype(np.float64))
    bound = 4 * (k + 2) * U32 * (np.abs(A) @ np.abs(B) + np.abs(C))
    assert np.all(np.abs(_host(dD).astype(np.float64) - ref) <= bound)


# ------------------------------------------------------------------- leaves
LEAF_SIZES = [1, 2, 3, 16, 17, 31, 64, 100, 128, 129, 200, 256, 300, 512, 777, 1024, 1536, 2048]


@pytest.mark.parametrize("L", LEAF_SIZES)
def test_leaf_gj_parity(torch_cuda, L):
    """A single leaf (leaf >= n) is the Gauss-Jordan kernel alone."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(L, seed=L) - 0.9 * L * np.eye(L)  # pivoting is active
    dA = _dev_f(torch, A)
    X = _host(S.invert(dA, leaf=max(L, 1)))
    assert S.info() == 0
    ref, info = oracle.gj_inv(A)
    assert info == 0
    kap = _kappa(A)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * kap * U), (err, kap)
    assert oracle.residual(A, X) <= 1e-13


@pytest.mark.parametrize("L", [5, 64, 128, 256, 640])
def test_leaf_exact_cases(torch_cuda, L):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    D = W.pow2_diagonal(L, seed=L)
    X = _host(S.invert(_dev_f(torch, D), leaf=L))
    assert np.array_equal(X, np.diag(1.0 / np.diag(D)))
    P = W.permutation(L, seed=L)
    X = _host(S.invert(_dev_f(torch, P), leaf=L))
    assert np.array_equal(X, P.T)


def test_leaf_mixed_f32_io_is_fp64_inside(torch_cuda):
    """Mixed mode with no recursion and no refinement: the leaf reads the
    FP32 copy, eliminates in FP64 and stores FP32 (one rounding at the end)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 96
    A = W.diag_dominant(n, 4)
    X, rep = S.invert_mixed(_dev_f(torch, A), leaf=n, ns_steps=0, report=True)
    A32 = A.astype(np.float32).astype(np.float64)
    ref, _ = oracle.gj_inv(A32)
    X = _host(X)
    assert np.max(np.abs(X - ref) / np.maximum(np.abs(ref), 1e-300)) <= 2 * U32 * (1 + 1e-3)
    assert rep["steps"] == 0 and rep["status"] == 0


# --------------------------------------------------------------- recursion
INV_CASES = [
    # generator, n, leaf
    ("dd", 256, 64),     # diag-dominant parity case (depth 2)
    ("dd", 300, 64),     # ragged split
    ("spd", 512, 128),
    ("spd", 1024, 256),  # blocked-leaf tier
    ("dd", 640, 16),     # deep recursion, tiny leaves
    ("spdk", 512, 64),   # kappa = 1e4 spectrum
    ("hh", 256, 32),     # Householder: self-inverse
    ("dd", 1000, 200),
    ("spd", 2048, 512),
]


def _gen(kind, n):
    if kind == "dd":
        return W.diag_dominant(n, seed=n)
    if kind == "spd":
        return W.spd_gram(n, seed=n)
    if kind == "spdk":
        return W.spd_spectrum(n, seed=n, kappa=1e4)
    if kind == "hh":
        return W.householder(n, seed=n)
    raise ValueError(kind)


@pytest.mark.parametrize("kind,n,leaf", INV_CASES)
def test_invert_fp64_parity(torch_cuda, kind, n, leaf):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = _gen(kind, n)
    dA = _dev_f(torch, A)
    X = _host(S.invert(dA, leaf=leaf))
    assert S.info() == 0
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    kap = _kappa(A)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * kap * U), (err, kap)
    rho = oracle.residual(A, X)
    assert rho <= 1e-12, rho
    # the library's own residual reaches the same verdict (both values sit at
    # the rounding floor here; tight agreement is tested on a perturbed inverse)
    assert S.residual(dA, _dev_f(torch, X)) <= 1e-12


@pytest.mark.parametrize("n,lda,leaf", [(600, 611, 300), (1000, 1003, 512), (515, 520, 515)])
def test_invert_fp64_panel_leaves_padded_lda(torch_cuda, n, lda, leaf):
    """FP64 leaves above order 128 are read in place from the input (the
    first panel and its update use the input's leading dimension): padded
    input and output, NaN in the input padding, the output padding kept."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(n, seed=n + 5)
    bufA = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
    bufA[:, :n] = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dA = bufA.t()[:n, :]                      # column-major view with ld lda
    bufX = torch.full((n, lda + 2), 7.0, dtype=torch.float64, device="cuda")
    dX = bufX.t()[:n, :]
    S.invert(dA, leaf=leaf, out=dX)
    assert S.info() == 0
    X = _host(dX)
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * _kappa(A) * U), err
    assert oracle.residual(A, X) <= 1e-12
    assert bool(torch.all(bufX[:, n:] == 7.0))
    assert bool(torch.all(torch.isnan(bufA[:, n:])))   # the input is never written


@pytest.mark.parametrize("n,eps", [(300, 1e-6), (1024, 1e-9)])
def test_device_residual_matches_host(torch_cuda, n, eps):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(n, seed=n)
    X = np.linalg.inv(A)
    X = X * (1.0 + eps * np.random.default_rng(1).standard_normal(X.shape))
    rho_host = oracle.residual(A, X)
    rho_dev = S.residual(_dev_f(torch, A), _dev_f(torch, X))
    assert abs(rho_dev - rho_host) <= 1e-3 * rho_host


def test_invert_matches_gj_oracle_too(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(256, seed=1)
    X = _host(S.invert(_dev_f(torch, A), leaf=64))
    ref, _ = oracle.gj_inv(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= 1e-14


def test_row_major_input_gives_row_major_inverse(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 384
    A = W.diag_dominant(n, seed=3) + np.triu(np.ones((n, n)))  # not symmetric
    dA = torch.from_numpy(np.ascontiguousarray(A)).to("cuda")  # row-major
    X = _host(S.invert(dA, leaf=128))
    assert oracle.residual(A, X) <= 1e-13
    assert abs(S.residual(dA, torch.from_numpy(np.ascontiguousarray(X)).cuda()) - oracle.residual(A, X)) < 1e-14


def test_block_diagonal_exact_zeros(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n, leaf = 512, 128
    n1 = oracle.split(n)
    A = W.block_diagonal(n, n1, seed=9)
    X = _host(S.invert(_dev_f(torch, A), leaf=leaf))
    assert np.all(X[:n1, n1:] == 0) and np.all(X[n1:, :n1] == 0)
    X11 = _host(S.invert(_dev_f(torch, A[:n1, :n1]), leaf=leaf))
    X22 = _host(S.invert(_dev_f(torch, A[n1:, n1:]), leaf=leaf))
    assert np.array_equal(X[:n1, :n1], X11) and np.array_equal(X[n1:, n1:], X22)


def test_golden_unimodular_exact(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    here = os.path.join(os.path.dirname(__file__), "golden")
    A = np.loadtxt(os.path.join(here, "unimodular64_A.txt"))
    ref = np.loadtxt(os.path.join(here, "unimodular64_Ainv.txt"))
    X = _host(S.invert(_dev_f(torch, A), leaf=16))
    assert np.array_equal(X, ref)


def test_status_survives_a_growing_residual_call(torch_cuda):
    """spin_residual may grow the stream's workspace; the status words of the
    inversion before it move along, so spin_info still reports it."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    S.release()
    n, leaf = 256, 128
    A = W.diag_dominant(n, seed=2)
    A[:, 100] = 0.0
    A[100, :] = 0.0
    dA = _dev_f(torch, A)
    dX = S.invert(dA, leaf=leaf)
    assert S.workspace_bytes(n, leaf) < 16384 + 8 * n * n  # the residual needs more
    S.residual(dA, dX)
    assert S.info() == 101


def test_singular_leaf_reports_column(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n, leaf = 256, 64
    A = W.diag_dominant(n, seed=2)
    A[:, 40] = 0.0
    A[40, :] = 0.0
    S.invert(_dev_f(torch, A), leaf=leaf)
    assert S.info() == 41
    B = W.diag_dominant(n, seed=2)
    B[200, 200] = np.nan
    S.invert(_dev_f(torch, B), leaf=leaf)
    assert S.info() > 128  # NaN sits in the trailing block; a later leaf flags it
    # a clean call afterwards resets the status
    S.invert(_dev_f(torch, W.diag_dominant(n, seed=2)), leaf=leaf)
    assert S.info() == 0


def test_graph_replay_and_eager_agree_bitwise(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = _dev_f(torch, W.spd_gram(768, seed=4))
    out = torch.empty_like(A)
    X1 = _host(S.invert(A, leaf=128, out=out))   # captures a graph
    X2 = _host(S.invert(A, leaf=128, out=out))   # replays it
    os.environ["SPIN_NO_GRAPH"] = "1"
    try:
        X3 = _host(S.invert(A, leaf=128, out=out))
    finally:
        del os.environ["SPIN_NO_GRAPH"]
    assert np.array_equal(X1, X2) and np.array_equal(X1, X3)


# ------------------------------------------------------------ mixed + Newton
@pytest.mark.parametrize("n,leaf,steps", [(512, 128, 2), (1024, 128, 2), (1024, 256, 3)])
def test_mixed_fp32_refined_to_fp64(torch_cuda, n, leaf, steps):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(n, seed=n, kappa=1e4)
    dA = _dev_f(torch, A)
    X, rep = S.invert_mixed(dA, leaf=leaf, ns_steps=steps, report=True)
    X = _host(X)
    assert rep["status"] == 0
    assert rep["rho_before"] <= 1e-3
    assert rep["rho_after"] <= 1e-12, rep
    rho = oracle.residual(A, X)
    assert rho <= 1e-12
    assert abs(rep["rho_after"] - rho) <= 0.05 * rho + 1e-17
    ref, _ = oracle.strassen_inv(A, leaf)
    kap = _kappa(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= max(1e-13, 100 * kap * U)
    # residual norms square from step to step until the FP64 floor
    r = rep["r_fro"]
    assert r[1] <= max(10 * r[0] ** 2, 1e-9)


def test_mixed_newton_step_matches_oracle_step(torch_cuda):
    """One refinement step on the GPU equals the oracle's X + X (I - A X) to
    rounding: run 0 and 1 steps from the same FP32 start."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 256
    A = W.spd_spectrum(n, seed=8, kappa=1e3)
    dA = _dev_f(torch, A)
    X0 = _host(S.invert_mixed(dA, leaf=64, ns_steps=0))
    X1 = _host(S.invert_mixed(dA, leaf=64, ns_steps=1))
    ref = oracle.ns_step(A, X0)
    assert np.linalg.norm(X1 - ref) / np.linalg.norm(ref) <= 100 * _kappa(A) * U


# --------------------------------------------------- full-size configuration
@pytest.mark.parametrize("n,leaf", [(8192, 256)])
def test_full_size_spd_sampled(torch_cuda, n, leaf):
    """The benchmark configuration: SPD B B^T/n + I, n = 8192, leaf 256.
    Checked by the residual and by sampled columns against LAPACK solves."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(n, seed=2)
    dA = _dev_f(torch, A)
    dX = S.invert(dA, leaf=leaf)
    assert S.info() == 0
    rho = S.residual(dA, dX)
    assert rho <= 1e-12, rho
    g = np.random.default_rng(0)
    cols = np.sort(g.choice(n, size=6, replace=False))
    Xs = _host(dX[:, cols])
    E = np.zeros((n, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    ref = np.linalg.solve(A, E)
    assert np.linalg.norm(Xs - ref) / np.linalg.norm(ref) <= 1e-12
    assert np.linalg.norm(A @ Xs - E) / np.linalg.norm(E) <= 1e-12


def _lambda_max_power(A, iters=60, seed=0):
    """Largest eigenvalue of a symmetric positive-definite A by power iteration
    (an upper estimate once converged: the Rayleigh quotient of the last iterate)."""
    v = np.random.default_rng(seed).standard_normal(A.shape[0])
    for _ in range(iters):
        v = A @ v
        v /= np.linalg.norm(v)
    return float(v @ (A @ v))


@pytest.mark.parametrize("n,leaf", [(8192, 256)])
def test_full_size_spd_against_oracle(torch_cuda, n, leaf):
    """The benchmark configuration against the oracle's recursion (O2) on the
    same matrix: forward error <= max(1e-13, 100 kappa u), and every element
    within 100 kappa u of its column's largest oracle entry.  A = B B^T / n + I
    has smallest eigenvalue >= 1, so kappa <= lambda_max (power iteration,
    with 5 % slack)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_gram(n, seed=2)
    dA = _dev_f(torch, A)
    X = _host(S.invert(dA, leaf=leaf))
    assert S.info() == 0
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    kap = 1.05 * _lambda_max_power(A)
    assert 1.0 < kap < 10.0, kap
    tol = max(1e-13, 100 * kap * U)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    assert err <= tol, (err, tol)
    colmax = np.abs(ref).max(axis=0)
    elem = (np.abs(X - ref).max(axis=0) / colmax).max()
    assert elem <= 100 * kap * U, elem


def test_graph_cache_stays_bounded_and_correct(torch_cuda):
    """More distinct buffer sets than the graph cache holds: the cache is
    emptied and rebuilt, and every call still returns the same inverse."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 96
    A = W.diag_dominant(n, seed=77)
    dA = _dev_f(torch, A)
    first = _host(S.invert(dA, leaf=32))
    outs = [torch.empty_like(dA) for _ in range(80)]
    for o in outs:
        S.invert(dA, leaf=32, out=o)
    torch.cuda.synchronize()
    assert S.info() == 0
    for o in outs:
        assert np.array_equal(_host(o), first)
