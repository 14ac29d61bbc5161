"""Exact rational Gauss-Jordan inverse for tiny matrices -- TEST INFRASTRUCTURE.

Used only by the tests to pin the floating-point oracle: for integer (or
dyadic) inputs it returns the mathematically exact inverse as
``fractions.Fraction`` entries.  Pure Python loops; intended for n <= 64.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_inverse(a) -> list[list[Fraction]] | None:
    """Exact inverse of a float matrix whose entries are exactly representable
    rationals (every float is).  Returns None if the matrix is singular."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    m = [[Fraction(float(a[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for k in range(n):
        p = next((i for i in range(k, n) if m[i][k] != 0), None)
        if p is None:
            return None
        m[k], m[p] = m[p], m[k]
        piv = m[k][k]
        m[k] = [v / piv for v in m[k]]
        for i in range(n):
            if i != k and m[i][k] != 0:
                f = m[i][k]
                m[i] = [vi - f * vk for vi, vk in zip(m[i], m[k])]
    return [row[n:] for row in m]


def to_float(x: list[list[Fraction]]) -> np.ndarray:
    """Correctly rounded float64 image of an exact matrix."""
    return np.array([[float(v) for v in row] for row in x], dtype=np.float64)
