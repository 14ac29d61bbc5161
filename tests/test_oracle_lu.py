"""Pins of O4, the oracle's inversion through a block LU factorisation (the
paper's comparison method): against exact rational inverses, a closed form,
O1 within its error bound, and breakdown reporting.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.exact import exact_inverse, to_float

U = 2.0 ** -53


@pytest.mark.parametrize("n,leaf", [(32, 8), (64, 16), (33, 5), (100, 100), (130, 64)])
def test_exact_on_unimodular_lu_products(n, leaf):
    """L U with unit bidiagonal factors: the factorisation without pivoting
    recovers them exactly, so every step stays on small integers."""
    A = W.unimodular_bidiag(n, seed=n + leaf)
    X, info = oracle.lu_inv(A, leaf)
    assert info == 0
    assert np.array_equal(X, to_float(exact_inverse(A)))


def test_closed_form_2x2():
    X, info = oracle.lu_inv(np.array([[4.0, 2.0], [2.0, 3.0]]), 1)
    assert info == 0
    assert np.array_equal(X, np.array([[3.0, -2.0], [-2.0, 4.0]]) / 8.0)


@pytest.mark.parametrize("gen,n,leaf", [("dd", 256, 64), ("spd", 200, 32), ("dd", 300, 64),
                                        ("spdk", 128, 16), ("dd", 96, 96)])
def test_agrees_with_gauss_jordan(gen, n, leaf):
    A = {"dd": lambda: W.diag_dominant(n, 1), "spd": lambda: W.spd_gram(n, 2),
         "spdk": lambda: W.spd_spectrum(n, 4, kappa=1e4)}[gen]()
    X, info = oracle.lu_inv(A, leaf)
    R, info1 = oracle.gj_inv(A)
    assert info == 0 and info1 == 0
    kappa = np.linalg.cond(A)
    assert oracle.forward_error(X, R) <= 4 * n * kappa * U
    assert oracle.residual(A, X) <= n * kappa * U


def test_breakdown_reports_global_column():
    """A zero row and column in the second leaf: status = its 1-based column."""
    A = W.diag_dominant(64, seed=8)
    A[:, 40] = 0.0
    A[40, :] = 0.0
    _, info = oracle.lu_inv(A, 32)
    assert info == 41
