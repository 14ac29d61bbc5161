"""Pins of the oracle's reduced-precision products (oracle/lowprec.py).

The rounding is checked against a library routine (torch's CPU
float32 -> bfloat16 conversion, round to nearest even) and hand-worked ties;
the split and the products against exact arithmetic."""
import numpy as np
import pytest
import torch

from oracle import lowprec as LP


def _bits(x):
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def test_round_matches_torch_bfloat16():
    g = np.random.default_rng(11)
    x = np.concatenate([
        g.standard_normal(20000).astype(np.float32),
        (g.standard_normal(5000) * 1e30).astype(np.float32),
        (g.standard_normal(5000) * 1e-30).astype(np.float32),
        # exact ties: 8 kept bits + a lone half-ulp bit, both parities
        (np.float32(1.0) + np.arange(256, dtype=np.float32) * np.float32(2.0 ** -7)
         + np.float32(2.0 ** -8)),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, -3.3895314e38,
                  np.finfo(np.float32).max, 1e-45], dtype=np.float32),
    ])
    ours = LP.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(_bits(ours), _bits(ref))


@pytest.mark.parametrize("x,expect", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                      # tie, kept lsb even -> down
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie, kept lsb odd -> up
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above the tie -> up
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),
    (255.0, 255.0),                              # 8 significant bits: exact
    (257.0, 256.0),                              # tie at 2^8 + 1 -> even 256
    (259.0, 260.0),                              # tie, odd lsb -> up
])
def test_round_hand_cases(x, expect):
    assert float(LP.bf16_round(np.float32(x))[0]) == expect


def test_round_nan_and_overflow():
    r = LP.bf16_round(np.array([np.nan, np.finfo(np.float32).max], dtype=np.float32))
    assert np.isnan(r[0]) and np.isinf(r[1]) and r[1] > 0


def test_split_reconstructs_to_16_bits():
    g = np.random.default_rng(12)
    x = g.standard_normal(50000).astype(np.float32)
    hi, lo = LP.bf16_split(x)
    # hi and lo are BF16 values
    assert np.array_equal(LP.bf16_round(hi), hi) and np.array_equal(LP.bf16_round(lo), lo)
    err = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - x.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    # and the split is no better than 24 - 2*8 bits can be: some error remains
    assert err.max() > 0


def test_split_exact_on_8_bit_values():
    x = np.arange(-255, 256, dtype=np.float32) * np.float32(2.0 ** -5)
    hi, lo = LP.bf16_split(x)
    assert np.array_equal(hi, x) and np.all(lo == 0)


@pytest.mark.parametrize("mode", ["fp32", "bf16", "bf16x3"])
def test_products_exact_on_small_integers(mode):
    g = np.random.default_rng(13)
    a = g.integers(-128, 129, size=(7, 9))
    b = g.integers(-128, 129, size=(9, 5))
    exact = np.array([[sum(int(a[i, k]) * int(b[k, j]) for k in range(9)) for j in range(5)]
                      for i in range(7)], dtype=np.float64)
    assert np.array_equal(LP.gemm_lowprec(a.astype(np.float32), b.astype(np.float32), mode), exact)


def test_bf16x3_drops_only_lo_lo():
    g = np.random.default_rng(14)
    a = g.standard_normal((6, 8)).astype(np.float32)
    b = g.standard_normal((8, 4)).astype(np.float32)
    ah, al = (t.astype(np.float64) for t in LP.bf16_split(a))
    bh, bl = (t.astype(np.float64) for t in LP.bf16_split(b))
    full = (ah + al) @ (bh + bl)
    got = LP.gemm_lowprec(a, b, "bf16x3")
    assert np.allclose(got + al @ bl, full, rtol=0, atol=1e-12)
    # and it is far closer to the FP32 product than plain BF16
    ref = a.astype(np.float64) @ b.astype(np.float64)
    e3 = np.abs(got - ref).max()
    e1 = np.abs(LP.gemm_lowprec(a, b, "bf16") - ref).max()
    assert e3 < e1 / 50
