"""CPU oracle for Strassen's block-recursive inversion -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and this package imports nothing from the GPU library.

Contents
  * ``gj_inv``        -- O1, Gauss-Jordan with partial pivoting on [A | I]
                         (leaf inversion; the paper leaves the method open,
                         Alg. 1, Sec. 3.1).
  * ``strassen_inv``  -- O2, the block-inverse identity Alg. 1 (Sec. 3.1)
                         evaluates, recursing on the leading block and on the
                         negated Schur complement A21 A11^-1 A12 - A22.
  * ``strassen_inv_spd`` -- O2 specialised to symmetric A (the positive-
                         definite matrices of Sec. 2.1): the column factor
                         A11^-1 A12 is the transpose of the row factor
                         A21 A11^-1, so C12 = C21^T; the Schur complement and
                         C11 keep their lower triangles, mirrored.
  * ``lu_inv``        -- O4, inversion through a block LU factorisation
                         without pivoting: L^-1 and U^-1 by block recursion,
                         then X = U^-1 L^-1 (the paper's comparison method).
  * ``gemm``          -- the plain matrix product of ``multiply`` (Sec. 3.3).
  * ``ns_step``       -- one Newton refinement step X + X (I - A X)
                         (Newton iteration as Strassen-inversion stabiliser,
                         Sec. 2.1).
  * ``residual``      -- rho = |A X - I|_F / (|A|_F |X|_F) in float64.
  * ``split``         -- order of the leading block when a block is split.
  * ``flops``         -- the method's flop count by direct summation over the
                         recursion (leaf Gauss-Jordan 2 L^3, each product 2 m n k).

The numerical core lives in ``spin_oracle.c`` (plain C, OpenMP over
independent columns, ``-O2 -ffp-contract=off``); ``exact.py`` holds an exact
rational Gauss-Jordan for tiny integer matrices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spin_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]

_lock = threading.Lock()
_lib = None


def build(src: str = _SRC, out: str = _LIB, extra: list[str] | None = None) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", *CFLAGS, *(extra or []), src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_gemm.argtypes = [dp, i64, dp, i64, dp, i64, i64, i64, i64]
    lib.oracle_gemm.restype = None
    lib.oracle_gj_inv.argtypes = [dp, i64, i64, dp, i64]
    lib.oracle_gj_inv.restype = ctypes.c_int
    lib.oracle_strassen_inv.argtypes = [dp, i64, i64, dp, i64, i64]
    lib.oracle_strassen_inv.restype = ctypes.c_int
    lib.oracle_strassen_inv_spd.argtypes = [dp, i64, i64, dp, i64, i64]
    lib.oracle_strassen_inv_spd.restype = ctypes.c_int
    lib.oracle_lu_inv.argtypes = [dp, i64, i64, dp, i64, i64]
    lib.oracle_lu_inv.restype = ctypes.c_int
    lib.oracle_lu_leaf.argtypes = [dp, i64, i64, dp, i64, dp, i64]
    lib.oracle_lu_leaf.restype = ctypes.c_int
    lib.oracle_ns_step.argtypes = [dp, i64, i64, dp, i64, dp, i64]
    lib.oracle_ns_step.restype = ctypes.c_int
    lib.oracle_split.argtypes = [i64]
    lib.oracle_split.restype = i64
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _f64(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    return np.asfortranarray(a)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gemm(a, b, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """C = A B by the plain triple loop."""
    lib = lib or load()
    a, b = _f64(a), _f64(b)
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    c = np.zeros((m, n), dtype=np.float64, order="F")
    lib.oracle_gemm(_ptr(a), max(m, 1), _ptr(b), max(k, 1), _ptr(c), max(m, 1), m, n, k)
    return c


def gj_inv(a, lib: ctypes.CDLL | None = None):
    """O1: returns (X, info); info = 0 or the 1-based failing pivot column."""
    lib = lib or load()
    a = _f64(a)
    n = a.shape[0]
    assert a.shape == (n, n)
    x = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.oracle_gj_inv(_ptr(a), n, max(n, 1), _ptr(x), max(n, 1))
    return x, int(info)


def strassen_inv(a, leaf: int, lib: ctypes.CDLL | None = None):
    """O2 (block-inverse identity of Alg. 1): returns (X, info)."""
    lib = lib or load()
    a = _f64(a)
    n = a.shape[0]
    assert a.shape == (n, n)
    x = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.oracle_strassen_inv(_ptr(a), n, max(n, 1), _ptr(x), max(n, 1), int(leaf))
    return x, int(info)


def strassen_inv_spd(a, leaf: int, lib: ctypes.CDLL | None = None):
    """O3 (O2 for symmetric A, four products per split): returns (X, info)."""
    lib = lib or load()
    a = _f64(a)
    n = a.shape[0]
    assert a.shape == (n, n)
    x = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.oracle_strassen_inv_spd(_ptr(a), n, max(n, 1), _ptr(x), max(n, 1), int(leaf))
    return x, int(info)


def lu_inv(a, leaf: int, lib: ctypes.CDLL | None = None):
    """O4 (block LU without pivoting, X = U^-1 L^-1): returns (X, info)."""
    lib = lib or load()
    a = _f64(a)
    n = a.shape[0]
    assert a.shape == (n, n)
    x = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.oracle_lu_inv(_ptr(a), n, max(n, 1), _ptr(x), max(n, 1), int(leaf))
    return x, int(info)


def lu_leaf(a, lib: ctypes.CDLL | None = None):
    """O4's leaf: (L^-1, U^-1, info) of A = L U without pivoting."""
    lib = lib or load()
    a = _f64(a)
    n = a.shape[0]
    li = np.zeros((n, n), dtype=np.float64, order="F")
    ui = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.oracle_lu_leaf(_ptr(a), n, max(n, 1), _ptr(li), max(n, 1), _ptr(ui), max(n, 1))
    return li, ui, int(info)


def ns_step(a, x, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """One refinement step X + X (I - A X)."""
    lib = lib or load()
    a, x = _f64(a), _f64(x)
    n = a.shape[0]
    xn = np.zeros((n, n), dtype=np.float64, order="F")
    rc = lib.oracle_ns_step(_ptr(a), n, n, _ptr(x), n, _ptr(xn), n)
    assert rc == 0
    return xn


def split(m: int, lib: ctypes.CDLL | None = None) -> int:
    lib = lib or load()
    return int(lib.oracle_split(int(m)))


def residual(a, x) -> float:
    """rho = |A X - I|_F / (|A|_F |X|_F), float64 (numpy matmul)."""
    a = np.asarray(a, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    r = a @ x
    r[np.diag_indices(a.shape[0])] -= 1.0
    return float(np.linalg.norm(r) / (np.linalg.norm(a) * np.linalg.norm(x)))


def forward_error(x, x_ref) -> float:
    """|X - X_ref|_F / |X_ref|_F."""
    x = np.asarray(x, dtype=np.float64)
    x_ref = np.asarray(x_ref, dtype=np.float64)
    return float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))


def flops(n: int, leaf: int) -> int:
    """Flops of the recursion by direct summation: 2 L^3 per leaf of order L,
    2 m n k per product (six per internal node, Alg. 1)."""
    if n <= leaf:
        return 2 * n ** 3
    n1 = split(n)
    n2 = n - n1
    prod = 2 * (n2 * n1 * n1 + n1 * n1 * n2 + n2 * n1 * n2 + n1 * n2 * n2 + n2 * n2 * n1 + n1 * n2 * n1)
    return flops(n1, leaf) + flops(n2, leaf) + prod
