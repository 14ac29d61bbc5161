"""FP64-accurate block products on integer matrix cores: the exact value the
emulation computes -- TEST INFRASTRUCTURE (only tests/, the smoke check and the
benchmark's CPU leg may import it).

The Newton refinement (the paper's stabiliser of Strassen inversion, Sec. 2.1)
needs the residual R = I - A X and the update X + X R accurate to FP64.  They
are emulated on INT8 matrix cores by the integer modular scheme of Ozaki,
Uchino and Imamura ("Ozaki Scheme II", 2025), which rests on the error-free
splitting of Ozaki, Ogita, Oishi and Rump (2012):

1. every row i of the left operand is scaled by a power of two 2^s_i and
   rounded to the nearest integer (ties to even), every column j of the right
   operand likewise by 2^t_j, with the shifts chosen so that no integer
   exceeds 2^beta in magnitude:  s_i = beta - E_i, where the row's largest
   magnitude is f 2^E_i with f in [1/2, 1) (a zero row has shift 0);
2. the product P = A' B' of the two integer matrices is formed exactly (the
   GPU forms it modulo several moduli below 256 with INT8 products and
   rebuilds it by Chinese remaindering);
3. P is rounded once to FP64 (nearest, ties to even) and scaled back by
   2^-(s_i + t_j);
4. the epilogue: R = I - D (one rounding) for the residual, X + D (one
   rounding) for the update.

This module computes that value directly, with the exact integer product
formed from 17-bit limbs by int64 matrix products (exact: every partial sum
stays below 2^63) and combined in Python integers.  It shares nothing with
the GPU library.  A row of the left operand or a column of the right operand
that holds a non-finite value yields NaN in its row or column of the result.
"""
from __future__ import annotations

import math

import numpy as np

LIMB = 17  # bits per limb of the exact product


def _shifts(mags: np.ndarray, beta: int) -> np.ndarray:
    """Shift per row of `mags` (the largest magnitude of each row)."""
    out = np.zeros(mags.shape[0], dtype=np.int64)
    for i, m in enumerate(mags):
        if m > 0 and math.isfinite(m):
            out[i] = beta - math.frexp(float(m))[1]
    return out


def split_rows(a, beta: int):
    """(A' as Python-int object array, shifts s): A'_ij = rint(a_ij 2^s_i)."""
    a = np.asarray(a, dtype=np.float64)
    mags = np.max(np.abs(a), axis=1) if a.shape[1] else np.zeros(a.shape[0])
    s = _shifts(mags, beta)
    ai = np.empty(a.shape, dtype=object)
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            v = a[i, j]
            ai[i, j] = int(np.rint(math.ldexp(v, int(s[i])))) if math.isfinite(v) else 0
    return ai, s


def split_cols(b, beta: int):
    """(B' object array, shifts t): B'_ij = rint(b_ij 2^t_j), column scaling."""
    bi, t = split_rows(np.asarray(b, dtype=np.float64).T, beta)
    return bi.T, t


def _limbs(m: np.ndarray, n_limbs: int) -> list[np.ndarray]:
    """Signed limbs: m = sum_p L_p 2^(LIMB p), |L_p| < 2^LIMB, as int64 arrays."""
    sign = np.vectorize(lambda x: -1 if x < 0 else 1, otypes=[np.int64])(m)
    mag = np.vectorize(abs, otypes=[object])(m)
    out = []
    for p in range(n_limbs):
        lp = np.vectorize(lambda x: (x >> (LIMB * p)) & ((1 << LIMB) - 1), otypes=[np.int64])(mag)
        out.append(sign * lp)
    return out


def exact_product(ai: np.ndarray, bi: np.ndarray, beta: int) -> np.ndarray:
    """The exact integer product of two integer matrices with entries of at
    most beta + 1 bits, as a Python-int object array."""
    k = ai.shape[1]
    assert k < (1 << (63 - 2 * LIMB - 1)), "inner dimension too long for exact int64 limbs"
    nl = (beta + 1 + LIMB - 1) // LIMB + 1
    la, lb = _limbs(ai, nl), _limbs(bi, nl)
    out = np.zeros((ai.shape[0], bi.shape[1]), dtype=object)
    for p in range(nl):
        for q in range(nl):
            part = (la[p] @ lb[q]).astype(object)  # exact: |terms| < 2^34, k < 2^28
            out = out + part * (1 << (LIMB * (p + q)))
    return out


def emulated_product(a, b, beta_a: int, beta_b: int) -> np.ndarray:
    """D = A B as the emulation forms it (steps 1-3 above), float64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ai, s = split_rows(a, beta_a)
    bi, t = split_cols(b, beta_b)
    p = exact_product(ai, bi, max(beta_a, beta_b))
    m, n = p.shape
    d = np.empty((m, n), dtype=np.float64)
    bad_r = ~np.all(np.isfinite(a), axis=1) if a.shape[1] else np.zeros(m, bool)
    bad_c = ~np.all(np.isfinite(b), axis=0) if b.shape[0] else np.zeros(n, bool)
    for i in range(m):
        for j in range(n):
            if bad_r[i] or bad_c[j]:
                d[i, j] = np.nan
            else:
                d[i, j] = math.ldexp(float(p[i, j]), -int(s[i]) - int(t[j]))
    return d


def residual(a, x, beta_a: int, beta_b: int) -> np.ndarray:
    """R = I - A X with the emulated product (one rounding in the difference)."""
    d = emulated_product(a, x, beta_a, beta_b)
    return np.eye(d.shape[0], d.shape[1]) - d


def update(x, r, beta_a: int, beta_b: int) -> np.ndarray:
    """X + X R with the emulated product (one rounding in the sum)."""
    return np.asarray(x, dtype=np.float64) + emulated_product(x, r, beta_a, beta_b)


def beta_for(k: int, log2_modulus: float) -> int:
    """Largest beta with 2 k 2^(2 beta) below the product of the moduli, so
    that the exact product of two beta-bit integer matrices with inner
    dimension k is fixed by its residues."""
    return int(math.floor((log2_modulus - 1.0 - math.log2(max(k, 1))) / 2.0 - 1e-9))
