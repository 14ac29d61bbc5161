"""GPU parity of the BF16 product flavours and of the BF16 mixed modes.

Products: the GPU result (operands rounded or split to BF16 in the kernel,
FP32 accumulation) against the oracle's exact-operand product of the same
FP32 inputs (oracle/lowprec.py), element by element, within the FP32
accumulation bound (k + 2) u32 (|op(A)| |op(B)| + |C|).  A BF16 rounding that
differed from round-to-nearest-even anywhere would miss by about 2^-9 of a
term, far outside that bound.

Inversions: the mixed modes refined by FP64 Newton steps reach the FP64
residual target where the rounding error of their products allows it
(bf16x3, about 2^-16 per operand, on SPD kappa = 1e4; plain BF16, 2^-9, on
diagonally dominant input), and plain BF16 on SPD kappa = 1e4, where
kappa * 2^-9 exceeds 1, is reported as diverged.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import lowprec as LP

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev32(torch, a):
    a = np.asarray(a, dtype=np.float32)
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def _dev64(torch, a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).T)).cuda().t()


def _host(t):
    return t.detach().cpu().numpy()


# m % 4, k % 4 and the leading dimensions decide between the vector and the
# guarded kernel; the tile count decides between 128, 64 and 32 tiles, and,
# for plain BF16 vector products of at least 256 of them, the eight-wave
# 256 x 256 tile (the last two shapes, the last with ragged edges and a
# partial k slab).
SHAPES = [(64, 64, 64), (200, 136, 300), (130, 70, 45), (33, 17, 5), (1, 1, 1),
          (512, 512, 512), (2048, 1536, 96), (2050, 1540, 99), (2048, 2048, 64),
          (4096, 4096, 64), (4100, 4104, 100)]


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_gemm_lowprec_parity(torch_cuda, mode, m, n, k):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    g = np.random.default_rng(m * 7 + n * 3 + k)
    A = g.standard_normal((m, k)).astype(np.float32)
    B = g.standard_normal((k, n)).astype(np.float32)
    C = g.standard_normal((m, n)).astype(np.float32)
    dA, dB, dC = _dev32(torch, A), _dev32(torch, B), _dev32(torch, C)
    dD = torch.zeros_like(dC)
    S.gemm_cm(m, n, k, -1.0, dA, m, dB, k, 1.0, dC, m, dD, m, False, mode)
    torch.cuda.synchronize()
    ref = C.astype(np.float64) - LP.gemm_lowprec(A, B, mode)
    bound = 2 * (k + 2) * U32 * (LP.abs_product(A, B, mode) + np.abs(C))
    err = np.abs(_host(dD).astype(np.float64) - ref)
    assert np.all(err <= bound), (float(err.max()), float(bound.min()))


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
def test_gemm_lowprec_identity_epilogue_and_ld(torch_cuda, mode):
    """R = I - A B with padded leading dimensions (the residual form)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    m, k, lda, ldb, ldd = 96, 80, 100, 84, 104
    g = np.random.default_rng(5)
    A = g.uniform(-1, 1, (lda, k)).astype(np.float32)
    B = g.uniform(-1, 1, (ldb, m)).astype(np.float32)
    dA, dB = _dev32(torch, A), _dev32(torch, B)
    dD = _dev32(torch, np.full((ldd, m), 7.0, np.float32))
    S.gemm_cm(m, m, k, -1.0, dA, lda, dB, ldb, 0.0, None, ldd, dD, ldd, True, mode)
    torch.cuda.synchronize()
    a, b = A[:m, :], B[:k, :]
    ref = np.eye(m) - LP.gemm_lowprec(a, b, mode)
    bound = 2 * (k + 2) * U32 * (LP.abs_product(a, b, mode) + 1.0)
    D = _host(dD)
    assert np.all(np.abs(D[:m, :].astype(np.float64) - ref) <= bound)
    assert np.all(D[m:, :] == 7.0)  # rows beyond m untouched


def test_bf16_is_coarser_than_bf16x3_is_coarser_than_fp32(torch_cuda):
    """The three flavours differ from the FP64 product in the expected order."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 256
    g = np.random.default_rng(9)
    A = g.standard_normal((n, n)).astype(np.float32)
    B = g.standard_normal((n, n)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    errs = {}
    for mode in ("fp32", "bf16x3", "bf16"):
        dD = _dev32(torch, np.zeros((n, n), np.float32))
        S.gemm_cm(n, n, n, 1.0, _dev32(torch, A), n, _dev32(torch, B), n, 0.0, None, n, dD, n,
                  False, mode)
        torch.cuda.synchronize()
        errs[mode] = float(np.abs(_host(dD) - ref).max())
    assert errs["fp32"] < errs["bf16x3"] < errs["bf16"] / 30, errs


# ------------------------------------------------------------- inversions
@pytest.mark.parametrize("n,leaf", [(512, 128), (1024, 256)])
def test_mixed_bf16x3_spd_refined_to_fp64(torch_cuda, n, leaf):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(n, seed=n + 1, kappa=1e4)
    dA = _dev64(torch, A)
    X, rep = S.invert_mixed(dA, leaf=leaf, mode="bf16x3", ns_steps=3, report=True)
    X = _host(X)
    assert rep["status"] == 0, rep
    assert rep["rho_before"] <= 1e-3, rep
    assert rep["rho_after"] <= 1e-12, rep
    assert oracle.residual(A, X) <= 1e-12
    ref, _ = oracle.strassen_inv(A, leaf)
    kap = np.linalg.cond(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= max(1e-13, 100 * kap * U)


@pytest.mark.parametrize("mode,steps", [("fp32", 2), ("bf16x3", 3)])
@pytest.mark.parametrize("n,leaf", [(512, 128), (1000, 64)])
def test_mixed_symmetric_schedule_refined_to_fp64(torch_cuda, mode, steps, n, leaf):
    """The symmetric schedule with FP32-storage products (mode | SYMMETRIC):
    unrefined residual of the same order as the plain schedule's, refined to
    the FP64 target.  Newton steps square the error of X0 until the FP64
    floor of about kappa u, so after the same number of steps the distance to
    O3 is compared with the plain schedule's (or that floor), not with the
    floor alone: two steps from an FP32 start at kappa = 1e4 can still sit
    above it."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(n, seed=n + 7, kappa=1e4)
    dA = _dev64(torch, A)
    Xs, rs = S.invert_mixed(dA, leaf=leaf, mode=mode + "_sym", ns_steps=steps, report=True)
    Xp, rp = S.invert_mixed(dA, leaf=leaf, mode=mode, ns_steps=steps, report=True)
    Xs = _host(Xs)
    assert rs["status"] == 0 and rp["status"] == 0, (rs, rp)
    assert rs["rho_before"] <= 10 * rp["rho_before"], (rs, rp)
    assert rs["rho_after"] <= 1e-12, rs
    assert oracle.residual(A, Xs) <= 1e-12
    ref, _ = oracle.strassen_inv_spd(A, leaf)
    kap = np.linalg.cond(A)
    err_s = np.linalg.norm(Xs - ref) / np.linalg.norm(ref)
    err_p = np.linalg.norm(_host(Xp) - ref) / np.linalg.norm(ref)
    assert err_s <= max(10 * err_p, 100 * kap * U), (err_s, err_p)


def test_mixed_bf16_diag_dominant_refined(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 512
    A = W.diag_dominant(n, seed=21)
    dA = _dev64(torch, A)
    X, rep = S.invert_mixed(dA, leaf=128, mode="bf16", ns_steps=3, report=True)
    assert rep["status"] == 0, rep
    assert rep["rho_before"] <= 1e-3, rep
    assert rep["rho_after"] <= 1e-12, rep
    assert oracle.residual(A, _host(X)) <= 1e-12


def test_mixed_bf16_spd_kappa_1e4_flagged_diverged(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n = 512
    A = W.spd_spectrum(n, seed=22, kappa=1e4)
    dA = _dev64(torch, A)
    _, rep = S.invert_mixed(dA, leaf=128, mode="bf16", ns_steps=3, report=True)
    assert rep["status"] == S.NS_DIVERGED, rep
    assert not (rep["rho_after"] <= 1e-12)
    assert S.info() == S.NS_DIVERGED


@pytest.mark.parametrize("mode,steps", [("fp32", 2), ("bf16", 3), ("bf16x3", 3)])
def test_mixed_modes_odd_order_padded_ld(torch_cuda, mode, steps):
    """n = 301 (odd: the guarded BF16 kernel runs inside the recursion), leaf 64,
    input and output with leading dimensions 306 and 309."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    n, lda, ldx = 301, 306, 309
    A = W.diag_dominant(n, seed=31)
    bufA = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
    bufA[:, :n] = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dA = bufA.t()[:n, :]                    # column-major view, ld 306
    bufX = torch.full((n, ldx), 7.0, dtype=torch.float64, device="cuda")
    dX = bufX.t()[:n, :]
    _, rep = S.invert_mixed(dA, leaf=64, mode=mode, ns_steps=steps, out=dX, report=True)
    assert rep["status"] == 0, rep
    assert rep["rho_after"] <= 1e-12, rep
    X = _host(dX)
    ref, _ = oracle.strassen_inv(A, 64)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= max(1e-13, 100 * np.linalg.cond(A) * U)
    # padding rows of the output are untouched
    assert bool(torch.all(bufX[:, n:] == 7.0))


def test_empty_batch(torch_cuda):
    import paper_1801_04723_amd as S
    outs, info = S.invert_batch([], leaf=64)
    assert outs == [] and info == []


@pytest.mark.parametrize("mode,steps,ok", [("bf16x3", 1, False), ("bf16x3", 3, True), ("fp32", 2, True)])
def test_final_residual_acceptance(torch_cuda, mode, steps, ok):
    """After the refinement steps the library checks rho <= 1e-12 on the
    device and reports SPIN_NS_DIVERGED otherwise, with or without a report."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(512, seed=21, kappa=1e4)
    dA = _dev64(torch, A)
    X = S.invert_mixed(dA, leaf=128, mode=mode, ns_steps=steps)
    status = S.info()
    rho = oracle.residual(A, _host(X))
    _, rep = S.invert_mixed(dA, leaf=128, mode=mode, ns_steps=steps, report=True)
    assert rep["status"] == status
    assert abs(rep["rho_after"] - rho) <= 0.05 * rho + 1e-18
    if ok:
        assert status == 0 and rho <= 1e-12, (status, rho)
    else:
        assert status == S.NS_DIVERGED and rho > 1e-12, (status, rho)
