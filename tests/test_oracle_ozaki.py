"""Pins of the emulated FP64 product (oracle.ozaki), CPU only.

Each pin fixes a value without the module's own arithmetic: the splitting
step against hand-worked integers (round to nearest, ties to even, negative
values, the scale from the row's largest magnitude), products of integer
matrices against numpy's exact int64 product, the error bound of the
splitting against the exact rational product (fractions.Fraction), the
residual of an exact integer inverse (exactly zero), and the modulus budget.
Planted mistakes (truncation instead of rounding, the wrong scaling axis, a
dropped scale, a flipped residual or update sign) must each fail a pin.
"""
import inspect
import math
import textwrap
from fractions import Fraction

import numpy as np
import pytest

from oracle import ozaki as O
import workloads as W
from oracle.exact import exact_inverse, to_float


def test_split_rows_hand_worked():
    beta = 4
    # row max 3.5 = 0.875 * 2^2 -> shift 4 - 2 = 2: values times 4, rounded to nearest even
    a = np.array([[3.5, 0.3125, -0.3125, 0.375, 0.125, -0.625]])
    ai, s = O.split_rows(a, beta)
    assert s.tolist() == [2]
    #   3.5*4 = 14, 0.3125*4 = 1.25 -> 1, -1.25 -> -1, 0.375*4 = 1.5 -> 2 (even),
    #   0.125*4 = 0.5 -> 0 (even), -0.625*4 = -2.5 -> -2 (even)
    assert [int(v) for v in ai[0]] == [14, 1, -1, 2, 0, -2]
    # a zero row keeps shift 0; a row max that is a power of two: 1 = 0.5 * 2^1
    ai, s = O.split_rows(np.array([[0.0, 0.0], [1.0, -0.75]]), 3)
    assert s.tolist() == [0, 2] and [int(v) for v in ai[1]] == [4, -3]
    # column scaling of the right operand
    bi, t = O.split_cols(np.array([[1.0, 8.0], [0.5, -3.0]]), 3)
    assert t.tolist() == [2, -1] and [[int(v) for v in r] for r in bi] == [[4, 4], [2, -2]]


def _split_pins(split_rows) -> bool:
    """The scaled row maximum lands in [2^(beta-1), 2^beta]: the integers use
    the whole budget of beta bits and never exceed it."""
    ok = True
    g = np.random.default_rng(8)
    A = g.standard_normal((20, 9)) * np.exp2(g.integers(-40, 40, size=(20, 1)))
    for beta in (8, 30, 47):
        ai, _ = split_rows(A, beta)
        for row in ai:
            mx = max(abs(int(v)) for v in row)
            ok &= (1 << (beta - 1)) <= mx <= (1 << beta)
    return bool(ok)


def test_split_uses_the_bit_budget():
    assert _split_pins(O.split_rows)


def _int_pins(emulated_product) -> bool:
    """Integer operands whose scaled values are exact: the product is exact."""
    ok = True
    g = np.random.default_rng(3)
    for m, k, n in ((1, 1, 1), (5, 9, 4), (16, 40, 12)):
        A = g.integers(-1000, 1001, size=(m, k))
        B = g.integers(-1000, 1001, size=(k, n))
        ok &= np.array_equal(emulated_product(A.astype(float), B.astype(float), 40, 40),
                             (A @ B).astype(float))
    return bool(ok)


def _bound_pins(emulated_product, beta=20) -> bool:
    """|D - A B| <= 2^-beta (m_i sum_k |b_kj| + n_j sum_k |a_ik|) + k 2^-2beta m_i n_j
    + 2^-53 |D|, with m_i, n_j the largest magnitudes of row i of A and column j
    of B (rounding to nearest moves each scaled entry by at most half a unit),
    checked against the exact rational product; rows of very different scale."""
    ok = True
    g = np.random.default_rng(5)
    for m, k, n in ((4, 7, 3), (6, 12, 5)):
        A = g.standard_normal((m, k)) * np.exp2(g.integers(-30, 30, size=(m, 1)))
        B = g.standard_normal((k, n)) * np.exp2(g.integers(-30, 30, size=(1, n)))
        D = emulated_product(A, B, beta, beta)
        mi = np.abs(A).max(axis=1)
        nj = np.abs(B).max(axis=0)
        for i in range(m):
            for j in range(n):
                exact = sum(Fraction(A[i, q]) * Fraction(B[q, j]) for q in range(k))
                err = abs(Fraction(D[i, j]) - exact)
                bound = (math.ldexp(1.0, -beta) * (mi[i] * np.abs(B[:, j]).sum() + nj[j] * np.abs(A[i]).sum())
                         + k * math.ldexp(1.0, -2 * beta) * mi[i] * nj[j] + math.ldexp(abs(D[i, j]), -53))
                ok &= err <= Fraction(bound) * Fraction(1 + 1e-12)
    return bool(ok)


def test_integer_products_exact():
    assert _int_pins(O.emulated_product)


def test_error_bound_against_exact_rational():
    assert _bound_pins(O.emulated_product)


def test_residual_and_update_of_exact_inverse():
    A = W.unimodular_bidiag(24, seed=9)
    X = to_float(exact_inverse(A))
    R = O.residual(A, X, 47, 47)
    assert np.array_equal(R, np.zeros_like(R))  # A X = I exactly
    assert np.array_equal(O.update(X, R, 47, 47), X)
    # a perturbed inverse: R = I - A X exactly for integer data
    Xp = X.copy()
    Xp[3, 5] += 1.0
    assert np.array_equal(O.residual(A, Xp, 47, 47), np.eye(24) - A @ Xp)


def test_nonfinite_rows_and_columns():
    A = np.ones((3, 4))
    A[1, 2] = np.nan
    B = np.ones((4, 2))
    B[0, 1] = np.inf
    D = O.emulated_product(A, B, 30, 30)
    assert np.isnan(D[1]).all() and np.isnan(D[:, 1]).all()
    assert D[0, 0] == 4.0 and D[2, 0] == 4.0


def test_modulus_budget():
    # 2 k 2^(2 beta) must stay below the product of the moduli
    for k, lm in ((16384, 110.2), (1, 64.0), (300, 117.8)):
        b = O.beta_for(k, lm)
        assert 1 + math.log2(k) + 2 * b < lm <= 1 + math.log2(k) + 2 * (b + 1) + 1e-9


def _mutant(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) == 1, old
    ns = dict(vars(O))
    exec(src.replace(old, new), ns)
    return ns[func.__name__]


def _product_with(split_rows=None, split_cols=None, emulated=None):
    ns = dict(vars(O))
    if split_rows:
        ns["split_rows"] = split_rows
    if split_cols:
        ns["split_cols"] = split_cols
    src = textwrap.dedent(inspect.getsource(O.emulated_product))
    exec(src, ns)
    return ns["emulated_product"]


MUTANTS = {
    "truncate": ("split_rows", "int(np.rint(math.ldexp(v, int(s[i]))))", "int(math.ldexp(v, int(s[i])))"),
    "scale_off_by_one": ("_shifts", "out[i] = beta - math.frexp(float(m))[1]",
                         "out[i] = beta + 1 - math.frexp(float(m))[1]"),
    "no_scale_back": ("emulated_product", "math.ldexp(float(p[i, j]), -int(s[i]) - int(t[j]))",
                      "float(p[i, j])"),
    "wrong_axis": ("split_rows", "np.max(np.abs(a), axis=1)", "np.max(np.abs(a), axis=0).max() * np.ones(a.shape[0])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_product_mutant_is_caught(name):
    fname, old, new = MUTANTS[name]
    ns = dict(vars(O))
    src = textwrap.dedent(inspect.getsource(getattr(O, fname)))
    assert src.count(old) == 1, old
    exec(src.replace(old, new), ns)
    # rebuild the chain on top of the mutated function
    for f in ("split_rows", "split_cols", "emulated_product"):
        if f != fname:
            exec(textwrap.dedent(inspect.getsource(getattr(O, f))), ns)
    prod = ns["emulated_product"]
    caught = not _int_pins(prod) or not _bound_pins(prod) or not _split_pins(ns["split_rows"])
    if name == "truncate":
        # truncation stays within twice the rounding bound on random data;
        # the hand-worked splitting pin tells the two apart
        ai, _ = ns["split_rows"](np.array([[3.5, 0.375]]), 4)
        caught = caught or [int(v) for v in ai[0]] != [14, 2]
    assert caught, name


def test_residual_and_update_sign_mutants_are_caught():
    A = W.unimodular_bidiag(12, seed=2)
    X = to_float(exact_inverse(A))
    Xp = X.copy()
    Xp[0, 1] += 1.0
    want_r = np.eye(12) - A @ Xp
    bad_r = _mutant(O.residual, "return np.eye(d.shape[0], d.shape[1]) - d",
                    "return d - np.eye(d.shape[0], d.shape[1])")
    assert np.array_equal(O.residual(A, Xp, 47, 47), want_r)
    assert not np.array_equal(bad_r(A, Xp, 47, 47), want_r)
    bad_u = _mutant(O.update, "return np.asarray(x, dtype=np.float64) + emulated_product(x, r, beta_a, beta_b)",
                    "return np.asarray(x, dtype=np.float64) - emulated_product(x, r, beta_a, beta_b)")
    R = np.eye(12) - A @ Xp
    assert np.array_equal(O.update(Xp, R, 47, 47), Xp + Xp @ R)
    assert not np.array_equal(bad_u(Xp, R, 47, 47), Xp + Xp @ R)
