"""Pins of O3, the oracle's Alg. 1 specialised to symmetric A (CPU only).

O3 is checked against results that do not come from itself: exact rational
inverses, a closed form, O1 (Gauss-Jordan on [A | I]) within its error bound,
O2 (the general recursion), and the structure the specialisation promises.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.exact import exact_inverse, to_float

U = 2.0 ** -53


@pytest.mark.parametrize("n,leaf", [(32, 8), (64, 16), (33, 8), (48, 5), (130, 64)])
def test_exact_on_symmetric_unimodular(n, leaf):
    """L L^T with unit bidiagonal L: every intermediate is a small integer, so
    the recursion must reproduce the exact rational inverse bit for bit."""
    A = W.spd_unimodular(n, seed=n + leaf)
    ref = to_float(exact_inverse(A))
    X, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    assert np.array_equal(X, ref)


def test_closed_form_2x2():
    """[[a, b], [b, c]]^-1 = [[c, -b], [-b, a]] / (ac - b^2), with dyadic values."""
    A = np.array([[4.0, 2.0], [2.0, 3.0]])
    X, info = oracle.strassen_inv_spd(A, 1)
    assert info == 0
    assert np.array_equal(X, np.array([[3.0, -2.0], [-2.0, 4.0]]) / 8.0)


@pytest.mark.parametrize("n,leaf", [(64, 8), (100, 7)])
def test_exact_on_pow2_diagonal_squares(n, leaf):
    """A diagonal SPD matrix with entries 2^e: every reciprocal is exact."""
    d = np.abs(np.diag(W.pow2_diagonal(n, seed=3)))
    A = np.diag(d)
    X, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    assert np.array_equal(X, np.diag(1.0 / d))


@pytest.mark.parametrize("gen,n,leaf", [("gram", 256, 64), ("gram", 200, 32), ("spectrum", 128, 16),
                                        ("gram", 300, 64)])
def test_agrees_with_gauss_jordan(gen, n, leaf):
    """Forward error against O1 within kappa u times a modest factor of n."""
    A = W.spd_gram(n, 2) if gen == "gram" else W.spd_spectrum(n, 4, kappa=1e4)
    X, info = oracle.strassen_inv_spd(A, leaf)
    R, info1 = oracle.gj_inv(A)
    assert info == 0 and info1 == 0
    kappa = np.linalg.cond(A)
    assert oracle.forward_error(X, R) <= 4 * n * kappa * U
    assert oracle.residual(A, X) <= n * kappa * U


@pytest.mark.parametrize("n,leaf", [(256, 64), (200, 32)])
def test_agrees_with_general_recursion(n, leaf):
    """O3 and O2 compute the same inverse by different product sequences."""
    A = W.spd_gram(n, 5)
    X3, i3 = oracle.strassen_inv_spd(A, leaf)
    X2, i2 = oracle.strassen_inv(A, leaf)
    assert i3 == 0 and i2 == 0
    assert oracle.forward_error(X3, X2) <= 4 * n * np.linalg.cond(A) * U


@pytest.mark.parametrize("n,leaf", [(256, 64), (200, 32), (130, 64), (512, 64)])
def test_symmetry_outside_the_leaves(n, leaf):
    """C12 = C21^T exactly; C11 exactly symmetric once it is an internal node
    (its lower triangle mirrored); only leaf blocks are symmetric merely up
    to rounding."""
    A = W.spd_gram(n, 6)
    X, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    n1 = oracle.split(n)
    assert np.array_equal(X[:n1, n1:], X[n1:, :n1].T)
    if n1 > leaf:
        assert np.array_equal(X[:n1, :n1], X[:n1, :n1].T)
    assert np.linalg.norm(X - X.T) <= 8 * n * U * np.linalg.norm(X)


@pytest.mark.parametrize("n,leaf", [(512, 64), (2048, 256)])
def test_residual_at_kappa_1e4_stays_near_u(n, leaf):
    """With V and C11 kept symmetric, the residual is that of the general
    recursion (about 3e-16 at kappa = 1e4); a node that passed an asymmetric
    V or C11 on would leave it near kappa u (about 2e-13)."""
    A = W.spd_spectrum(n, 4, kappa=1e4)
    X, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    assert oracle.residual(A, X) <= 1e-14


def test_single_leaf_is_gauss_jordan():
    A = W.spd_gram(96, 7)
    X, info = oracle.strassen_inv_spd(A, 96)
    R, _ = oracle.gj_inv(A)
    assert info == 0 and np.array_equal(X, R)


def test_breakdown_reports_global_column():
    """A zero row and column in the second leaf: status = its 1-based column."""
    A = W.spd_gram(64, 8)
    A[:, 40] = 0.0
    A[40, :] = 0.0
    _, info = oracle.strassen_inv_spd(A, 32)
    assert info == 41
