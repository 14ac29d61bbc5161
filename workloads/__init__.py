"""Seeded synthetic inputs for the Strassen-inversion workloads.

This module is shared by the CPU oracle (``oracle/``), the tests and the
benchmark.  It holds no part of the inversion method's arithmetic: it only
draws random matrices of the classes the method is specified for and builds
special test matrices whose inverses are known in closed form.

The paper inverts dense matrices drawn from Java's ``Random`` class with an
unstated distribution and no seed (Sec. 5.1, test setup).  The generators
below stand in for them with explicit, seeded distributions:

* ``diag_dominant``  -- entries U(-1, 1), ``n`` added to every diagonal entry
  (strictly diagonally dominant, so every leading block and every Schur
  complement is nonsingular);
* ``spd_gram``       -- ``B B^T / n + I`` with ``B`` i.i.d. N(0, 1);
* ``spd_spectrum``   -- ``Q diag(lam) Q^T`` with ``Q`` from the QR factorisation
  of a Gaussian matrix and ``lam`` geometrically spaced over ``[1, kappa]``.

Symmetric outputs are symmetrised as ``(M + M^T) / 2`` so that the stored
matrix is exactly symmetric.  All matrices are returned as float64 numpy
arrays in Fortran (column-major) order, the layout of the paper's blocks
(Sec. 3.2).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "diag_dominant",
    "spd_gram",
    "spd_spectrum",
    "householder",
    "unimodular_bidiag",
    "permutation",
    "pow2_diagonal",
    "block_diagonal",
    "block_lower_triangular",
    "gaussian",
    "serving_trace",
    "CONFIG_SEEDS",
]

# One seed per benchmark configuration (diag-dominant n=256 parity case,
# SPD n=8192, diag-dominant n=16384 leaf sweep, SPD spectrum n=16384,
# serving trace); request i of the serving trace uses seed 5000 + i.
CONFIG_SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5}


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 generator for ``seed``."""
    return np.random.default_rng(int(seed))


def _fortran(m: np.ndarray) -> np.ndarray:
    return np.asfortranarray(m, dtype=np.float64)


def diag_dominant(n: int, seed: int) -> np.ndarray:
    """Entries U(-1, 1) with ``n`` added to each diagonal entry."""
    g = rng(seed)
    a = g.uniform(-1.0, 1.0, size=(n, n))
    a[np.diag_indices(n)] += float(n)
    return _fortran(a)


def gaussian(n: int, seed: int, m: int | None = None) -> np.ndarray:
    """i.i.d. N(0, 1) matrix of shape (n, m or n)."""
    g = rng(seed)
    return _fortran(g.standard_normal(size=(n, n if m is None else m)))


def spd_gram(n: int, seed: int) -> np.ndarray:
    """``B B^T / n + I`` with ``B`` i.i.d. N(0, 1); spectrum inside ~[1, 5]."""
    g = rng(seed)
    b = g.standard_normal(size=(n, n))
    a = (b @ b.T) / float(n)
    a = 0.5 * (a + a.T)
    a[np.diag_indices(n)] += 1.0
    return _fortran(a)


def _haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    z = g.standard_normal(size=(n, n))
    q, r = np.linalg.qr(z)
    # fix the column signs by sign(diag R) so that Q is Haar distributed
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def spd_spectrum(n: int, seed: int, kappa: float = 1e4) -> np.ndarray:
    """``Q diag(lam) Q^T`` with ``lam_i = kappa^(i/(n-1))`` over ``[1, kappa]``."""
    g = rng(seed)
    q = _haar_orthogonal(n, g)
    if n == 1:
        lam = np.array([1.0])
    else:
        lam = np.power(float(kappa), np.arange(n, dtype=np.float64) / (n - 1))
    a = (q * lam[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return _fortran(a)


def householder(n: int, seed: int, v1sq: float = 0.6) -> np.ndarray:
    """``H = I - 2 v v^T`` with ``|v| = 1`` and ``v_1^2 = v1sq``.

    ``H`` is orthogonal and symmetric, so ``H^{-1} = H``.  With
    ``v_1^2 >= 0.6`` every leading minor ``1 - 2 |v_{:m}|^2`` is at most
    ``-0.2``, so a block recursion without cross-block pivoting never meets a
    singular leading block.
    """
    g = rng(seed)
    rest = g.standard_normal(n - 1)
    rest *= math.sqrt(1.0 - v1sq) / np.linalg.norm(rest)
    v = np.concatenate([[math.sqrt(v1sq)], rest])
    h = np.eye(n) - 2.0 * np.outer(v, v)
    return _fortran(h)


def unimodular_bidiag(n: int, seed: int) -> np.ndarray:
    """``L U`` with unit lower/upper bidiagonal factors whose off-diagonals are +-1.

    All leading principal minors equal 1 and the inverse is an integer
    matrix, so an exact rational inverse exists and every intermediate of a
    block recursion is an integer of modest size.
    """
    g = rng(seed)
    lo = np.eye(n)
    up = np.eye(n)
    if n > 1:
        lo[np.arange(1, n), np.arange(n - 1)] = g.choice([-1.0, 1.0], size=n - 1)
        up[np.arange(n - 1), np.arange(1, n)] = g.choice([-1.0, 1.0], size=n - 1)
    return _fortran(lo @ up)


def spd_unimodular(n: int, seed: int) -> np.ndarray:
    """``L L^T`` with ``L`` unit lower bidiagonal, off-diagonals +-1.

    Symmetric positive definite and tridiagonal, with determinant 1 and an
    integer inverse; every leading block is of the same form, so its
    Schur complements are too.
    """
    g = rng(seed)
    lo = np.eye(n)
    if n > 1:
        lo[np.arange(1, n), np.arange(n - 1)] = g.choice([-1.0, 1.0], size=n - 1)
    return _fortran(lo @ lo.T)


def permutation(n: int, seed: int) -> np.ndarray:
    """A random permutation matrix."""
    g = rng(seed)
    p = g.permutation(n)
    a = np.zeros((n, n))
    a[np.arange(n), p] = 1.0
    return _fortran(a)


def pow2_diagonal(n: int, seed: int) -> np.ndarray:
    """Diagonal matrix with entries +-2^e, e in [-8, 8]: reciprocals are exact."""
    g = rng(seed)
    e = g.integers(-8, 9, size=n)
    s = g.choice([-1.0, 1.0], size=n)
    return _fortran(np.diag(s * np.ldexp(1.0, e)))


def block_diagonal(n: int, n1: int, seed: int) -> np.ndarray:
    """diag(A11, A22) with diagonally dominant blocks of order n1 and n - n1."""
    a = np.zeros((n, n))
    a[:n1, :n1] = diag_dominant(n1, seed)
    a[n1:, n1:] = diag_dominant(n - n1, seed + 1)
    return _fortran(a)


def block_lower_triangular(n: int, n1: int, seed: int) -> np.ndarray:
    """[[A11, 0], [A21, A22]] with diagonally dominant diagonal blocks."""
    a = block_diagonal(n, n1, seed)
    g = rng(seed + 2)
    a[n1:, :n1] = g.uniform(-1.0, 1.0, size=(n - n1, n1))
    return _fortran(a)


def serving_trace(rate: float, duration: float, seed: int = 5,
                  n_min: int = 64, n_max: int = 4096, align: int = 64,
                  frac_spd: float = 0.5, frac_mixed: float = 0.7):
    """Open-loop request trace: Poisson arrivals, log-uniform sizes.

    Returns a list of dicts with keys ``t`` (arrival time, s), ``n`` (order,
    padded up to a multiple of ``align``), ``kind`` ("dd" or "spd"),
    ``kappa`` (for SPD requests, log-uniform in [10, 1e4]), ``mixed`` (bool)
    and ``seed`` (5000 + request index).
    """
    g = rng(seed)
    out = []
    t = 0.0
    i = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        raw = math.exp(g.uniform(math.log(n_min), math.log(n_max)))
        n = int(align * math.ceil(raw / align))
        n = max(align, min(n, n_max))
        spd = bool(g.uniform() < frac_spd)
        kappa = float(math.exp(g.uniform(math.log(10.0), math.log(1e4)))) if spd else 0.0
        mixed = bool(g.uniform() < frac_mixed)
        out.append({"t": t, "n": n, "kind": "spd" if spd else "dd",
                    "kappa": kappa, "mixed": mixed, "seed": 5000 + i})
        i += 1
    return out


# ------------------------------------------------------------ GPU generators
def torch_diag_dominant(n: int, seed: int, device="cuda"):
    """Seeded U(-1, 1) + n I generated on a torch device (column-major view)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    a = torch.rand((n, n), generator=g, dtype=torch.float64, device=device) * 2.0 - 1.0
    a.diagonal().add_(float(n))
    return a.t().contiguous().t()


def torch_spd_spectrum(n: int, seed: int, kappa: float, device="cuda"):
    """Seeded Q diag(lam) Q^T on a torch device: Q from the QR factorisation of
    a Gaussian matrix, lam geometric over [1, kappa]; symmetrised."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    q, r = torch.linalg.qr(z)
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    q = q * s[None, :]
    if n == 1:
        lam = torch.ones(1, dtype=torch.float64, device=device)
    else:
        lam = torch.pow(torch.tensor(float(kappa), dtype=torch.float64, device=device),
                        torch.arange(n, dtype=torch.float64, device=device) / (n - 1))
    a = (q * lam[None, :]) @ q.t().contiguous()
    a = 0.5 * (a + a.t())
    return a.t().contiguous().t()
