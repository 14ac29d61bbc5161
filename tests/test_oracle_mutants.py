"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle source, plants one plausible mistake (a dropped
term, a flipped sign, a transposed operand, a missing row swap, an index
slip), compiles the mutant into a temporary library and checks that at least
one pin fails against it.  The unmodified source must pass the same checks.
Everything runs on the CPU.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.exact import exact_inverse, to_float

SRC = os.path.join(os.path.dirname(oracle.__file__), "spin_oracle.c")

MUTANTS = {
    "c22_sign": ("mat_neg(f.invn, n2, c22, ldc, n2, n2);\nout:\n    factors_free(&f);\n    return info;\n}\n\nint oracle_strassen_inv(",
                 "mat_copy(f.invn, n2, c22, ldc, n2, n2);\nout:\n    factors_free(&f);\n    return info;\n}\n\nint oracle_strassen_inv("),
    "schur_sign": ("mat_sub(f.work, n2, a22, lda, f.negs, n2, n2, n2);\n    info = strassen_rec(",
                   "mat_sub(a22, lda, f.work, n2, f.negs, n2, n2, n2);\n    info = strassen_rec("),
    "rowfac_transposed": ("oracle_gemm(a21, lda, f.inv11, n1, f.rowfac, n2, n2, n1, n1);\n    oracle_gemm(f.inv11,",
                          "oracle_gemm(f.inv11, n1, a21, lda, f.rowfac, n2, n2, n1, n1);\n    oracle_gemm(f.inv11,"),
    "c11_dropped_term": ("mat_sub(f.inv11, n1, f.work, n1, c11, ldc, n1, n1);\n    mat_neg(",
                         "mat_copy(f.inv11, n1, c11, ldc, n1, n1);\n    mat_neg("),
    "c21_operand_order": ("oracle_gemm(f.invn, n2, f.rowfac, n2, c21, ldc, n2, n1, n2);\n    oracle_gemm(f.colfac, n1, c21",
                          "oracle_gemm(f.rowfac, n2, f.invn, n2, c21, ldc, n2, n1, n2);\n    oracle_gemm(f.colfac, n1, c21"),
    "no_row_swap": ("if (p != k)\n            for", "if (0)\n            for"),
    "gemm_k_slip": ("for (int64_t p = 0; p < k; ++p) {", "for (int64_t p = 1; p < k; ++p) {"),
    "scale_left_half_only": ("for (int64_t j = 0; j < w; ++j)\n            AT(M, k, j, n) = AT(M, k, j, n) / piv;",
                             "for (int64_t j = 0; j < n; ++j)\n            AT(M, k, j, n) = AT(M, k, j, n) / piv;"),
    "eliminate_below_only": ("if (i != k)\n                    AT(M, i, j, n)", "if (i > k)\n                    AT(M, i, j, n)"),
    "second_leaf_offset": ("info = strassen_rec(f.negs, n2, n2, f.invn, n2, leaf, col0 + n1);",
                           "info = strassen_rec(f.negs, n2, n2, f.invn, n2, leaf, col0);"),
}


# Mistakes planted in O3, the symmetric specialisation.
SPD_MUTANTS = {
    "spd_c12_not_transposed": ("mat_transpose(c21, ldc, c12, ldc, n2, n1);",
                               "mat_copy(c21, ldc, c12, ldc, n1, n2);"),
    "spd_c11_operand_order": ("oracle_gemm(c12, ldc, f.rowfac, n2, f.work, n1, n1, n1, n2);",
                              "oracle_gemm(f.rowfac, n2, c12, ldc, f.work, n1, n1, n1, n2);"),
    "spd_schur_uses_a21": ("oracle_gemm(f.rowfac, n2, a12, lda, f.work, n2, n2, n2, n1);",
                           "oracle_gemm(f.rowfac, n2, a21, lda, f.work, n2, n2, n2, n1);"),
    "spd_schur_sign": ("mat_sub(f.work, n2, a22, lda, f.negs, n2, n2, n2);\n    mat_mirror_lower(",
                       "mat_sub(a22, lda, f.work, n2, f.negs, n2, n2, n2);\n    mat_mirror_lower("),
    "spd_c22_sign": ("mat_neg(f.invn, n2, c22, ldc, n2, n2);\nout:\n    factors_free(&f);\n    return info;\n}\n\nint oracle_strassen_inv_spd(",
                     "mat_copy(f.invn, n2, c22, ldc, n2, n2);\nout:\n    factors_free(&f);\n    return info;\n}\n\nint oracle_strassen_inv_spd("),
    "spd_c11_dropped_term": ("mat_sub(f.inv11, n1, f.work, n1, c11, ldc, n1, n1);\n    mat_mirror_lower(",
                             "mat_copy(f.inv11, n1, c11, ldc, n1, n1);\n    mat_mirror_lower("),
    "spd_second_leaf_offset": ("info = strassen_spd_rec(f.negs, n2, n2, f.invn, n2, leaf, col0 + n1);",
                               "info = strassen_spd_rec(f.negs, n2, n2, f.invn, n2, leaf, col0);"),
    "spd_no_schur_mirror": ("    mat_mirror_lower(f.negs, n2, n2);", "    (void)0;"),
    "spd_no_c11_mirror": ("    mat_mirror_lower(c11, ldc, n1);", "    (void)0;"),
}


# Mistakes planted in O4, the block-LU inversion.
LU_MUTANTS = {
    "lu_multiplier_not_divided": ("AT(F, i, k, m) = AT(F, i, k, m) / piv;                 /* multiplier l_ik */",
                                  "AT(F, i, k, m) = AT(F, i, k, m);"),
    "lu_li21_sign": ("mat_neg(&AT(Li, n1, 0, ldl), ldl, &AT(Li, n1, 0, ldl), ldl, n2, n1); /* Li21 = -Li22 T1 */",
                     "(void)0;"),
    "lu_u12_operand_order": ("oracle_gemm(Li, ldl, A12, lda, U12, n1, n1, n2, n1);                /* U12 = Li11 A12  */",
                             "oracle_gemm(A12, lda, Li, ldl, U12, n1, n1, n2, n1);"),
    "lu_no_zero_fill": ("            AT(Li, i, j, ldl) = 0.0;                                    /* Li12 = 0        */",
                        "            (void)0;"),
    "lu_final_order": ("oracle_gemm(Ui, n, Li, n, X, ldx, n, n, n);                  /* X = Ui Li       */",
                       "oracle_gemm(Li, n, Ui, n, X, ldx, n, n, n);"),
    "lu_second_leaf_offset": ("ldu, leaf, col0 + n1);", "ldu, leaf, col0);"),
}


def _lu_pins_pass(lib) -> bool:
    """A compact set of the pins from test_oracle_lu; True iff all hold."""
    ok = True
    A = W.unimodular_bidiag(32, seed=40)
    X, info = oracle.lu_inv(A, 8, lib)
    ok &= info == 0 and np.array_equal(X, to_float(exact_inverse(A)))
    G = W.diag_dominant(200, 2)
    X, info = oracle.lu_inv(G, 32, lib)
    ref = np.linalg.inv(G)
    ok &= info == 0 and np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-12
    Z = W.diag_dominant(64, seed=8)
    Z[:, 40] = 0.0
    Z[40, :] = 0.0
    _, info = oracle.lu_inv(Z, 32, lib)
    ok &= info == 41
    return bool(ok)


def _spd_pins_pass(lib) -> bool:
    """A compact set of the pins from test_oracle_spd; True iff all hold."""
    ok = True
    A = W.spd_unimodular(32, seed=40)
    X, info = oracle.strassen_inv_spd(A, 8, lib)
    ok &= info == 0 and np.array_equal(X, to_float(exact_inverse(A)))
    G = W.spd_gram(200, 2)
    X, info = oracle.strassen_inv_spd(G, 32, lib)
    ref = np.linalg.inv(G)
    ok &= info == 0 and np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-12
    Z = W.spd_gram(64, 8)
    Z[:, 40] = 0.0
    Z[40, :] = 0.0
    _, info = oracle.strassen_inv_spd(Z, 32, lib)
    ok &= info == 41
    # symmetry outside the leaves, and the residual at kappa = 1e4
    X, info = oracle.strassen_inv_spd(G, 16, lib)
    n1 = oracle.split(200)
    ok &= info == 0 and np.array_equal(X[:n1, :n1], X[:n1, :n1].T)
    K = W.spd_spectrum(512, 4, kappa=1e4)
    X, info = oracle.strassen_inv_spd(K, 64, lib)
    ok &= info == 0 and oracle.residual(K, X) <= 1e-14
    return bool(ok)


def _pins_pass(lib) -> bool:
    """A compact set of the pins from test_oracle_pins; True iff all hold."""
    ok = True
    # exact unimodular inverse through both programs
    A = W.unimodular_bidiag(32, seed=5)
    ref = to_float(exact_inverse(A))
    X1, i1 = oracle.gj_inv(A, lib)
    X2, i2 = oracle.strassen_inv(A, 8, lib)
    ok &= i1 == 0 and i2 == 0 and np.array_equal(X1, ref) and np.array_equal(X2, ref)
    # permutation (pivoting)
    P = W.permutation(9, seed=2)
    Xp, ip = oracle.gj_inv(P, lib)
    ok &= ip == 0 and np.array_equal(Xp, P.T)
    # agreement with LAPACK on a non-symmetric matrix, both programs
    B = W.diag_dominant(128, seed=1) - 100.0 * np.eye(128)
    ref = np.linalg.inv(B)
    for X, info in (oracle.gj_inv(B, lib), oracle.strassen_inv(B, 32, lib)):
        ok &= info == 0 and np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-12
    # gemm on integers
    g = np.random.default_rng(0)
    M = g.integers(-9, 9, size=(7, 5)).astype(np.float64)
    N = g.integers(-9, 9, size=(5, 6)).astype(np.float64)
    ok &= np.array_equal(oracle.gemm(M, N, lib), M @ N)
    # breakdown column reporting: a zero column in the second leaf
    S = W.diag_dominant(64, seed=8)
    S[:, 40] = 0.0
    S[40, :] = 0.0
    _, info = oracle.strassen_inv(S, 32, lib)
    ok &= info == 41
    return bool(ok)


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    out = str(tmp_path / f"libmut_{name}.so")
    oracle.build(str(path), out)
    return oracle.load(out)


def test_unmutated_passes(tmp_path):
    path = tmp_path / "same.c"
    path.write_text(open(SRC).read())
    out = str(tmp_path / "libsame.so")
    oracle.build(str(path), out)
    lib = oracle.load(out)
    assert _pins_pass(lib)
    assert _spd_pins_pass(lib)
    assert _lu_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_variant(tmp_path, name, old, new)
    assert not _pins_pass(lib), f"mutant {name} survived the oracle pins"


@pytest.mark.parametrize("name", sorted(SPD_MUTANTS))
def test_spd_mutant_is_caught(tmp_path, name):
    old, new = SPD_MUTANTS[name]
    lib = _build_variant(tmp_path, name, old, new)
    assert not _spd_pins_pass(lib), f"mutant {name} survived the O3 pins"


@pytest.mark.parametrize("name", sorted(LU_MUTANTS))
def test_lu_mutant_is_caught(tmp_path, name):
    old, new = LU_MUTANTS[name]
    lib = _build_variant(tmp_path, name, old, new)
    assert not _lu_pins_pass(lib), f"mutant {name} survived the O4 pins"
