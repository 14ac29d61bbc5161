"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each compares the oracle
with a closed form, an exact rational inverse, a library routine (LAPACK via
numpy), an algebraic invariant of Strassen's scheme (Alg. 1, Sec. 3.1), or
the other oracle program.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.exact import exact_inverse, to_float

U = 2.0 ** -53


def _kappa_f(a):
    return float(np.linalg.cond(a, "fro"))


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(6))
def test_gj_2x2_closed_form(oracle_lib, seed):
    g = np.random.default_rng(seed)
    a, b, c, d = g.uniform(-2, 2, size=4)
    A = np.array([[a, b], [c, d]])
    det = a * d - b * c
    ref = np.array([[d, -b], [-c, a]]) / det
    X, info = oracle.gj_inv(A, oracle_lib)
    assert info == 0
    np.testing.assert_allclose(X, ref, rtol=64 * U * max(1.0, _kappa_f(A)), atol=0)


@pytest.mark.parametrize("seed", range(6))
def test_strassen_scalar_2x2_is_closed_form(oracle_lib, seed):
    """Alg. 1 with 1x1 leaves on a 2x2 matrix is the closed-form 2x2 inverse."""
    g = np.random.default_rng(100 + seed)
    a, b, c, d = g.uniform(0.5, 2, size=4) * g.choice([-1, 1], size=4)
    A = np.array([[a, b], [c, d]])
    det = a * d - b * c
    ref = np.array([[d, -b], [-c, a]]) / det
    X, info = oracle.strassen_inv(A, 1, oracle_lib)
    assert info == 0
    np.testing.assert_allclose(X, ref, rtol=64 * U * max(1.0, _kappa_f(A)), atol=0)


def test_unimodular_2x2_exact(oracle_lib):
    A = np.array([[2.0, 3.0], [1.0, 2.0]])  # det 1, inverse [[2,-3],[-1,2]]
    ref = np.array([[2.0, -3.0], [-1.0, 2.0]])
    for X, info in (oracle.gj_inv(A, oracle_lib), oracle.strassen_inv(A, 1, oracle_lib)):
        assert info == 0
        assert np.array_equal(X, ref)


# ------------------------------------------------------------- exact inverses
@pytest.mark.parametrize("n", [1, 5, 16, 64, 130])
@pytest.mark.parametrize("leaf", [1, 4, 16, 64])
def test_pow2_diagonal_bitwise(oracle_lib, n, leaf):
    A = W.pow2_diagonal(n, seed=n + leaf)
    ref = np.diag(1.0 / np.diag(A))
    X1, i1 = oracle.gj_inv(A, oracle_lib)
    X2, i2 = oracle.strassen_inv(A, leaf, oracle_lib)
    assert i1 == 0 and i2 == 0
    assert np.array_equal(X1, ref)
    assert np.array_equal(X2, ref)


@pytest.mark.parametrize("n", [2, 7, 33, 96])
def test_permutation_exact_gj(oracle_lib, n):
    """Pivoting is exercised: the inverse of a permutation is its transpose."""
    P = W.permutation(n, seed=n)
    X, info = oracle.gj_inv(P, oracle_lib)
    assert info == 0
    assert np.array_equal(X, P.T)


@pytest.mark.parametrize("n,leaf", [(16, 4), (32, 8), (64, 16), (64, 64), (96, 16), (128, 32)])
def test_unimodular_exact(oracle_lib, n, leaf):
    """All leading minors are 1 and the inverse is integral: both oracles
    must return the exact rational inverse."""
    A = W.unimodular_bidiag(n, seed=n + leaf)
    ref = to_float(exact_inverse(A))
    assert np.all(ref == np.round(ref))
    X1, i1 = oracle.gj_inv(A, oracle_lib)
    X2, i2 = oracle.strassen_inv(A, leaf, oracle_lib)
    assert i1 == 0 and i2 == 0
    assert np.array_equal(X1, ref)
    assert np.array_equal(X2, ref)


@pytest.mark.parametrize("seed", range(8))
def test_small_random_vs_exact_rational(oracle_lib, seed):
    """Brute force on tiny inputs: exact rational inverse, then error bound."""
    g = np.random.default_rng(seed)
    n = int(g.integers(2, 10))
    A = g.integers(-9, 10, size=(n, n)).astype(np.float64)
    A[np.diag_indices(n)] += 40.0  # keeps every leading block nonsingular
    ex = exact_inverse(A)
    ref = to_float(ex)
    kap = _kappa_f(A)
    for leaf in (1, 2, 3, n):
        X, info = oracle.strassen_inv(A, leaf, oracle_lib)
        assert info == 0
        err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
        assert err <= 16 * n * kap * U, (leaf, err)
    X, info = oracle.gj_inv(A, oracle_lib)
    assert info == 0
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= 16 * n * kap * U


# ------------------------------------------------------ structural invariants
@pytest.mark.parametrize("n,leaf", [(64, 32), (128, 64), (256, 64), (200, 50)])
def test_block_diagonal_structure(oracle_lib, n, leaf):
    """A12 = A21 = 0 makes II = III = 0 in Alg. 1, so C12 = C21 = 0 exactly and
    the diagonal blocks are the inverses of A11 and A22."""
    n1 = oracle.split(n, oracle_lib)
    A = W.block_diagonal(n, n1, seed=n)
    X, info = oracle.strassen_inv(A, leaf, oracle_lib)
    assert info == 0
    assert np.all(X[:n1, n1:] == 0.0) and np.all(X[n1:, :n1] == 0.0)
    X11, _ = oracle.strassen_inv(A[:n1, :n1], leaf, oracle_lib)
    X22, _ = oracle.strassen_inv(A[n1:, n1:], leaf, oracle_lib)
    assert np.array_equal(X[:n1, :n1], X11)
    assert np.array_equal(X[n1:, n1:], X22)


@pytest.mark.parametrize("n,leaf", [(64, 16), (128, 32), (192, 64)])
def test_block_lower_triangular_structure(oracle_lib, n, leaf):
    """A12 = 0 gives III = 0 hence C12 = 0 exactly (inverse of a block lower
    triangular matrix is block lower triangular)."""
    n1 = oracle.split(n, oracle_lib)
    A = W.block_lower_triangular(n, n1, seed=n)
    X, info = oracle.strassen_inv(A, leaf, oracle_lib)
    assert info == 0
    assert np.all(X[:n1, n1:] == 0.0)
    ref = np.linalg.inv(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("n,leaf", [(64, 8), (256, 16), (256, 64)])
def test_householder_self_inverse(oracle_lib, n, leaf):
    """H = I - 2 v v^T is its own inverse; every leading minor is <= -0.2, so
    the recursion never breaks down."""
    H = W.householder(n, seed=n)
    for X, info in (oracle.gj_inv(H, oracle_lib), oracle.strassen_inv(H, leaf, oracle_lib)):
        assert info == 0
        assert np.max(np.abs(X - H)) <= 8 * n * U


def test_leaf_equal_n_reduces_to_gj(oracle_lib):
    A = W.diag_dominant(96, seed=7)
    X1, _ = oracle.gj_inv(A, oracle_lib)
    X2, _ = oracle.strassen_inv(A, 96, oracle_lib)
    X3, _ = oracle.strassen_inv(A, 1000, oracle_lib)
    assert np.array_equal(X1, X2) and np.array_equal(X1, X3)


def test_breakdown_without_cross_block_pivoting(oracle_lib):
    """The scheme does not pivot across blocks: a singular A11 stops it even
    though A is invertible, while Gauss-Jordan with pivoting succeeds."""
    n = 16
    J = np.fliplr(np.eye(n))
    X1, i1 = oracle.gj_inv(J, oracle_lib)
    assert i1 == 0 and np.array_equal(X1, J)
    _, i2 = oracle.strassen_inv(J, 4, oracle_lib)
    assert i2 >= 1


def test_singular_and_nonfinite_report_column(oracle_lib):
    A = W.diag_dominant(32, seed=3)
    S = A.copy()
    S[:, 5] = 0.0
    _, info = oracle.gj_inv(S, oracle_lib)
    assert info == 6
    N = A.copy()
    N[20, 20] = np.nan
    _, info = oracle.gj_inv(N, oracle_lib)
    assert 1 <= info <= 21
    _, info = oracle.strassen_inv(N, 8, oracle_lib)
    assert info >= 17  # NaN sits in the trailing block, so a later leaf fails


# ---------------------------------------------------------- cross-checks
@pytest.mark.parametrize("gen,n,leaf", [("dd", 256, 64), ("dd", 512, 128), ("spd", 256, 32),
                                        ("spd", 384, 64), ("spdk", 256, 64), ("dd", 300, 64)])
def test_gj_vs_strassen_agree(oracle_lib, gen, n, leaf):
    if gen == "dd":
        A = W.diag_dominant(n, seed=n)
    elif gen == "spd":
        A = W.spd_gram(n, seed=n)
    else:
        A = W.spd_spectrum(n, seed=n, kappa=1e4)
    kap = _kappa_f(A)
    X1, i1 = oracle.gj_inv(A, oracle_lib)
    X2, i2 = oracle.strassen_inv(A, leaf, oracle_lib)
    assert i1 == 0 and i2 == 0
    diff = np.linalg.norm(X1 - X2) / np.linalg.norm(X1)
    assert diff <= max(1e-14, 8 * kap * U), (diff, kap)
    assert oracle.residual(A, X2) <= 1e-14


@pytest.mark.parametrize("n", [50, 200])
def test_gj_matches_lapack(oracle_lib, n):
    A = W.diag_dominant(n, seed=11) - 0.9 * n * np.eye(n)  # weaker dominance, pivoting active
    X, info = oracle.gj_inv(A, oracle_lib)
    assert info == 0
    ref = np.linalg.inv(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= 64 * _kappa_f(A) * U


def test_gemm_exact_integers(oracle_lib):
    g = np.random.default_rng(4)
    A = g.integers(-50, 50, size=(37, 23)).astype(np.float64)
    B = g.integers(-50, 50, size=(23, 41)).astype(np.float64)
    C = oracle.gemm(A, B, oracle_lib)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(C, ref)
    assert not np.array_equal(oracle.gemm(B.T, A.T, oracle_lib), ref)  # orientation matters


def test_gemm_ascending_k_order(oracle_lib):
    """Each entry is summed left to right: (1e16 + 1) - 1e16 loses the 1."""
    A = np.array([[1e16, 1.0, -1e16]])
    B = np.ones((3, 1))
    assert oracle.gemm(A, B, oracle_lib)[0, 0] == 0.0
    A2 = np.array([[1e16, -1e16, 1.0]])
    assert oracle.gemm(A2, B, oracle_lib)[0, 0] == 1.0


def test_ns_step_squares_residual(oracle_lib):
    """R_{k+1} = I - A X_{k+1} equals R_k^2 in exact arithmetic."""
    n = 96
    A = W.spd_gram(n, seed=9)
    X, _ = oracle.gj_inv(A, oracle_lib)
    g = np.random.default_rng(1)
    X0 = X * (1.0 + 1e-3 * g.standard_normal(X.shape))
    R0 = np.eye(n) - A @ X0
    X1 = oracle.ns_step(A, X0, oracle_lib)
    R1 = np.eye(n) - A @ X1
    assert np.linalg.norm(R1 - R0 @ R0) <= 1e-12 * max(1.0, np.linalg.norm(R0))
    assert np.linalg.norm(R1) < 0.1 * np.linalg.norm(R0)


def test_ns_step_fixed_point(oracle_lib):
    A = W.diag_dominant(64, seed=2)
    X, _ = oracle.gj_inv(A, oracle_lib)
    X1 = oracle.ns_step(A, X, oracle_lib)
    assert np.linalg.norm(X1 - X) / np.linalg.norm(X) <= 1e-15


# ---------------------------------------------------------- counts and split
@pytest.mark.parametrize("n,leaf", [(256, 64), (8192, 256), (16384, 128), (16384, 2048), (1024, 1)])
def test_flop_count_is_2n3(n, leaf):
    """Summing 2L^3 per leaf and 2mnk per product over the recursion gives
    exactly 2n^3 when n = leaf * 2^d."""
    assert oracle.flops(n, leaf) == 2 * n ** 3


@pytest.mark.parametrize("m", [2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 300, 4096, 4160])
def test_split_rule(oracle_lib, m):
    n1 = oracle.split(m, oracle_lib)
    assert 1 <= n1 < m
    if m >= 128:
        assert n1 % 64 == 0 and n1 >= m / 2 and n1 - m / 2 < 64
    if m & (m - 1) == 0:
        assert n1 == m // 2


def test_recursion_counts_match_paper():
    """2^i nodes at level i and 2^d leaves (Sec. 4, Fig. 1): count the leaves
    the oracle visits by inverting a diagonal matrix with an instrumented leaf
    size sweep -- the number of leaves equals n / leaf."""
    for n, leaf in [(256, 64), (512, 64), (1024, 128)]:
        d = int(math.log2(n // leaf))
        # leaf blocks are exactly the diagonal blocks of size leaf
        sizes = []

        def walk(m):
            if m <= leaf:
                sizes.append(m)
                return
            n1 = oracle.split(m)
            walk(n1)
            walk(m - n1)

        walk(n)
        assert len(sizes) == 2 ** d and all(s == leaf for s in sizes)


# ---------------------------------------------------------- stored fixtures
@pytest.mark.parametrize("n,leaf", [(16, 4), (64, 16)])
def test_golden_unimodular(oracle_lib, n, leaf):
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    A = np.loadtxt(os.path.join(here, f"unimodular{n}_A.txt"))
    ref = np.loadtxt(os.path.join(here, f"unimodular{n}_Ainv.txt"))
    assert np.array_equal(A, W.unimodular_bidiag(n, n))
    for X, info in (oracle.gj_inv(A, oracle_lib), oracle.strassen_inv(A, leaf, oracle_lib)):
        assert info == 0 and np.array_equal(X, ref)
