"""Reduced-precision block products -- TEST INFRASTRUCTURE (part of the oracle).

The paper computes every block product in double precision (Sec. 3.3,
`multiply` with JBlas DGEMM).  The mixed modes of the GPU library run the
recursion's products with FP32 operands rounded to BF16 on their way into the
matrix cores, with FP32 accumulation; this module is the plain definition of
those products, for the parity tests of that path:

  * ``bf16_round(x)``   -- FP32 -> nearest BF16 value, ties to even (IEEE
                           round-to-nearest on the top 16 bits of the FP32
                           pattern), returned as FP32.  NaN stays NaN,
                           overflow rounds to infinity.
  * ``bf16_split(x)``   -- hi = bf16_round(x), lo = bf16_round(x - hi); the
                           FP32 difference x - hi is exact.
  * ``gemm_lowprec(a, b, mode)`` -- the product the matrix cores accumulate,
                           evaluated in float64: "fp32" a b; "bf16"
                           r(a) r(b); "bf16x3" hi_a hi_b + lo_a hi_b + hi_a lo_b.

Pins (tests/test_oracle_lowprec.py): the rounding agrees bit for bit with
torch's CPU float32 -> bfloat16 conversion, and with hand-worked ties; the
split reconstructs x to 2^-16 relative and is exact on 8-bit values; the
products equal exact integer products on small integer matrices and drop
exactly the lo*lo term.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Nearest BF16 value of each FP32 entry (ties to even), as FP32 (at least 1-D)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    # add half an ulp of the 16-bit result, minus one unless the kept lsb is 1
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).copy()
    out[nan] = np.float32(np.nan)
    return out


def bf16_split(x):
    """(hi, lo) with hi = bf16_round(x) and lo = bf16_round(x - hi)."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


def gemm_lowprec(a, b, mode: str) -> np.ndarray:
    """Exact-operand product of FP32 matrices a (m x k) and b (k x n) in float64."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    if mode == "fp32":
        return a.astype(np.float64) @ b.astype(np.float64)
    if mode == "bf16":
        return bf16_round(a).astype(np.float64) @ bf16_round(b).astype(np.float64)
    if mode == "bf16x3":
        ah, al = (t.astype(np.float64) for t in bf16_split(a))
        bh, bl = (t.astype(np.float64) for t in bf16_split(b))
        return ah @ bh + al @ bh + ah @ bl
    raise ValueError(f"unknown mode {mode!r}")


def abs_product(a, b, mode: str) -> np.ndarray:
    """|op(a)| |op(b)| with the operands of ``gemm_lowprec`` (bound for the
    FP32 accumulation error)."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    if mode == "fp32":
        return np.abs(a.astype(np.float64)) @ np.abs(b.astype(np.float64))
    if mode == "bf16":
        return np.abs(bf16_round(a).astype(np.float64)) @ np.abs(bf16_round(b).astype(np.float64))
    ah, al = (np.abs(t.astype(np.float64)) for t in bf16_split(a))
    bh, bl = (np.abs(t.astype(np.float64)) for t in bf16_split(b))
    return ah @ bh + al @ bh + ah @ bl
