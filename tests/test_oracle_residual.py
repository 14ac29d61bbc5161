"""Pins of the oracle's acceptance measures, against closed forms and exact
rational arithmetic (CPU only).

rho = |A X - I|_F / (|A|_F |X|_F) is the residual measure every inverse is
accepted by (the paper reports none; the measure is this project's gate), and
|X - X_ref|_F / |X_ref|_F is the forward error against an oracle inverse.
Each pin fixes a value independently of the numpy code under test: closed
forms for scaled identities and a hand-worked 3 x 3 case, and the exact value
of the squared ratio in Fractions for random integer matrices.  Planted
mistakes (a dropped identity, X A instead of A X, a spectral or entrywise
norm, a squared or missing denominator factor) must each fail a pin.
"""
import inspect
import math
import textwrap
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _exact_rho2(A, X) -> Fraction:
    n = len(A)
    num = Fraction(0)
    for i in range(n):
        for j in range(n):
            s = sum(Fraction(int(A[i][k])) * Fraction(int(X[k][j])) for k in range(n))
            s -= 1 if i == j else 0
            num += s * s
    na = sum(Fraction(int(v)) ** 2 for row in A for v in row)
    nx = sum(Fraction(int(v)) ** 2 for row in X for v in row)
    return num / (na * nx)


def _exact_fwd2(X, R) -> Fraction:
    num = sum((Fraction(int(x)) - Fraction(int(r))) ** 2 for xr, rr in zip(X, R) for x, r in zip(xr, rr))
    return num / sum(Fraction(int(r)) ** 2 for rr in R for r in rr)


def _rho_pins(residual) -> bool:
    ok = True
    # A = 2 I, X = I / 4: A X - I = -I / 2, so rho = (sqrt(n) / 2) / (2 sqrt(n) sqrt(n) / 4) = 1 / sqrt(n)
    for n in (1, 3, 16, 100):
        r = residual(2.0 * np.eye(n), 0.25 * np.eye(n))
        ok &= math.isclose(r, 1.0 / math.sqrt(n), rel_tol=1e-15)
    # exact inverse of a non-diagonal matrix: rho = 0 exactly
    A = np.array([[2.0, 1.0], [1.0, 1.0]])
    ok &= residual(A, np.array([[1.0, -1.0], [-1.0, 2.0]])) == 0.0
    # hand-worked, non-commuting 3 x 3:
    #   A = [[1,1,0],[0,1,0],[0,0,1]], X = [[1,0,0],[1,1,0],[0,0,1]]
    #   A X = [[2,1,0],[1,1,0],[0,0,1]], A X - I = [[1,1,0],[1,0,0],[0,0,0]]
    #   |A X - I|_F = sqrt(3), |A|_F = |X|_F = 2, rho = sqrt(3) / 4
    A = np.array([[1.0, 1.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    X = np.array([[1.0, 0.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    ok &= math.isclose(residual(A, X), math.sqrt(3.0) / 4.0, rel_tol=1e-15)
    # exact rational value on random integer matrices (these also tell A X from X A)
    g = np.random.default_rng(7)
    for n in (2, 3, 5):
        for _ in range(4):
            A = g.integers(-4, 5, size=(n, n))
            X = g.integers(-4, 5, size=(n, n))
            if not A.any() or not X.any():
                continue
            want = math.sqrt(float(_exact_rho2(A.tolist(), X.tolist())))
            ok &= math.isclose(residual(A.astype(float), X.astype(float)), want, rel_tol=1e-14)
    return bool(ok)


def _fwd_pins(forward_error) -> bool:
    ok = True
    # X = 2 X_ref: error exactly 1; X = X_ref: exactly 0
    for n in (1, 4, 9):
        R = np.arange(1.0, n * n + 1).reshape(n, n)
        ok &= forward_error(2.0 * R, R) == 1.0
        ok &= forward_error(R, R) == 0.0
    # known perturbation: X_ref = I (n), X = I + eps e_0 e_1^T -> eps / sqrt(n)
    for n, eps in ((4, 1e-3), (16, 0.5)):
        X = np.eye(n)
        X[0, 1] = eps
        ok &= math.isclose(forward_error(X, np.eye(n)), eps / math.sqrt(n), rel_tol=1e-15)
    # exact rational value on random integer matrices (the reference is the second argument)
    g = np.random.default_rng(11)
    for n in (2, 3, 6):
        for _ in range(4):
            X = g.integers(-5, 6, size=(n, n))
            R = g.integers(-5, 6, size=(n, n))
            if not R.any():
                continue
            want = math.sqrt(float(_exact_fwd2(X.tolist(), R.tolist())))
            ok &= math.isclose(forward_error(X.astype(float), R.astype(float)), want, rel_tol=1e-14)
    return bool(ok)


def test_residual_pins():
    assert _rho_pins(oracle.residual)


def test_forward_error_pins():
    assert _fwd_pins(oracle.forward_error)


def _mutant(func, old: str, new: str):
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) == 1, old
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    return ns[func.__name__]


RHO_MUTANTS = {
    "dropped_identity": ("    r[np.diag_indices(a.shape[0])] -= 1.0\n", ""),
    "x_times_a": ("r = a @ x", "r = x @ a"),
    "spectral_norm": ("np.linalg.norm(r) /", "np.linalg.norm(r, 2) /"),
    "entrywise_1norm": ("np.linalg.norm(r) /", "np.abs(r).sum() /"),
    "squared_denominator": ("(np.linalg.norm(a) * np.linalg.norm(x))",
                            "(np.linalg.norm(a) * np.linalg.norm(x)) ** 2"),
    "missing_x_norm": ("(np.linalg.norm(a) * np.linalg.norm(x))", "(np.linalg.norm(a))"),
    "plus_identity": ("-= 1.0", "+= 1.0"),
}

FWD_MUTANTS = {
    "relative_to_x": ("/ np.linalg.norm(x_ref)", "/ np.linalg.norm(x)"),
    "max_norm": ("np.linalg.norm(x - x_ref)", "np.abs(x - x_ref).max()"),
    "squared": ("np.linalg.norm(x - x_ref) /", "np.linalg.norm(x - x_ref) ** 2 /"),
    "sum_not_difference": ("x - x_ref", "x + x_ref"),
}


@pytest.mark.parametrize("name", sorted(RHO_MUTANTS))
def test_residual_mutant_is_caught(name):
    assert not _rho_pins(_mutant(oracle.residual, *RHO_MUTANTS[name])), name


@pytest.mark.parametrize("name", sorted(FWD_MUTANTS))
def test_forward_error_mutant_is_caught(name):
    assert not _fwd_pins(_mutant(oracle.forward_error, *FWD_MUTANTS[name])), name
