"""spin_invert_noalloc through the C ABI: the allocation-free variant of
spin_invert on the library's fixed scratch array.

It must give spin_invert's result bit for bit (the same kernels and schedule
on a different workspace), also on a second call with a smaller order that
reuses the array the first call left behind, report its numerical status
through the caller's device int, and reject orders beyond the array's size.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda").t()


def _noalloc(torch, dA, leaf, dX, info):
    import paper_1801_04723_amd as S
    n = dA.shape[0]
    s = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    return S.lib().spin_invert_noalloc(dA.data_ptr(), n, dA.stride(1), dX.data_ptr(), dX.stride(1),
                                       leaf, info.data_ptr(), s)


def test_noalloc_equals_invert_on_two_calls(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    for n, leaf, seed in ((1536, 256, 1), (300, 64, 2)):   # the second call is smaller
        A = W.diag_dominant(n, seed=seed)
        dA = _dev(torch, A)
        ref = S.invert(dA, leaf=leaf)
        assert S.info() == 0
        dX = torch.full_like(ref, float("nan"))
        assert _noalloc(torch, dA, leaf, dX, info) == 0
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert torch.equal(dX, ref), (n, leaf)


def test_noalloc_status_and_limits(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    A = W.diag_dominant(256, seed=3)
    A[:, 40] = 0.0
    A[40, :] = 0.0
    dA = _dev(torch, A)
    dX = torch.empty_like(dA)
    assert _noalloc(torch, dA, 64, dX, info) == 0
    torch.cuda.synchronize()
    assert int(info.item()) == 41
    # too large for the fixed scratch: rejected before anything is enqueued
    big = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda").t()
    bigx = torch.empty_like(big)
    assert S.workspace_bytes(4096, 256) > S.NOALLOC_SCRATCH_MB << 20
    assert _noalloc(torch, big, 256, bigx, info) == -8  # SPIN_E_SCRATCH
    # a clean call afterwards reports 0 again, through the Python binding
    B = W.diag_dominant(256, seed=4)
    dB = _dev(torch, B)
    out = torch.empty_like(dB)
    S.invert_noalloc(dB, 64, out, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert torch.equal(out, S.invert(dB, leaf=64))
