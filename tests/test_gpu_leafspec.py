"""The leaves' speculative elimination against their pivot search.

Leaves first try the elimination with row k as the pivot of step k and check
every choice exactly against partial pivoting; on the first failed check the
workgroup redoes the block with the search, and later leaves of the same
inversion go straight to the search.  Either way the result must be the
search's bit for bit, which these tests compare by running each case with
speculation on and off (environment variable SPIN_NO_SPEC), and against the
oracle's Gauss-Jordan (O1) within the parity tolerance.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda").t()


def _both(fn):
    """fn() with speculation off, then on: (result_off, status_off, result_on, status_on)."""
    import paper_1801_04723_amd as S
    old = os.environ.get("SPIN_NO_SPEC")
    try:
        os.environ["SPIN_NO_SPEC"] = "1"
        x0 = fn().cpu().numpy()
        s0 = S.info()
        os.environ["SPIN_NO_SPEC"] = "0"
        x1 = fn().cpu().numpy()
        s1 = S.info()
    finally:
        if old is None:
            os.environ.pop("SPIN_NO_SPEC", None)
        else:
            os.environ["SPIN_NO_SPEC"] = old
    return x0, s0, x1, s1


def _swap_rows(a, i, j):
    a = a.copy()
    a[[i, j]] = a[[j, i]]
    return a


def _same_bits(x, y):
    return np.array_equal(x.view(np.int64), y.view(np.int64))


# diagonal pivots all the way (speculation holds) and a late off-diagonal
# pivot (speculation fails at step k and the block is redone by the search).
# Leaves of order 129-256 run their full 64-column panels on two workgroups,
# each owning 32 of the panel's steps: the failing step falls in the first
# workgroup's half (3, 150) or the second's (40, 100, 170, 254), in the first
# panel (read from the input) or a later one (read from the leaf's copy).
LEAF_CASES = [(L, None) for L in (1, 17, 64, 100, 128, 129, 200, 256, 300, 512)] + \
             [(64, 40), (128, 126), (256, 150), (256, 3), (256, 40), (256, 100), (200, 170),
              (256, 254), (512, 300)]


@pytest.mark.parametrize("L,swap", LEAF_CASES)
def test_single_leaf_spec_equals_search(torch_cuda, L, swap):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(L, seed=L + 7)
    if swap is not None:
        A = _swap_rows(A, swap, swap + 1)  # step `swap` pivots on row swap + 1
    dA = _dev(torch, A)
    x0, s0, x1, s1 = _both(lambda: S.invert(dA, leaf=L))
    assert s0 == s1 == 0
    assert _same_bits(x0, x1)
    ref, info = oracle.gj_inv(A)
    assert info == 0
    err = np.linalg.norm(x1 - ref) / np.linalg.norm(ref)
    assert err <= max(1e-13, 100 * np.linalg.cond(A) * U), err


@pytest.mark.parametrize("n,leaf,swap", [(1024, 256, None), (1024, 256, 300), (1024, 128, 5),
                                         (1000, 64, 700), (2048, 512, 1100), (1100, 512, None),
                                         (1100, 512, 936), (600, 300, None)])
def test_inversion_spec_equals_search(torch_cuda, n, leaf, swap):
    """A whole recursion; with a swap, an early leaf speculates successfully and
    the leaf holding the swapped rows fails its check.  n = 1100 with leaf 512
    has leaves of orders 320, 256, 320 and 204, and n = 600 with leaf 300
    leaves of orders 192, 128 and 280, so the two-workgroup panels' exchange
    areas pass across leaves of other tiers and orders."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(n, seed=n + leaf)
    if swap is not None:
        A = _swap_rows(A, swap, swap + 1)
    dA = _dev(torch, A)
    x0, s0, x1, s1 = _both(lambda: S.invert(dA, leaf=leaf))
    assert s0 == s1 == 0
    assert _same_bits(x0, x1)
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    assert np.linalg.norm(x1 - ref) / np.linalg.norm(ref) <= 1e-13


def test_spd_and_mixed_spec_equals_search(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.spd_spectrum(512, seed=12, kappa=1e4)
    dA = _dev(torch, A)
    x0, s0, x1, s1 = _both(lambda: S.invert_spd(dA, leaf=128))
    assert s0 == s1 == 0 and _same_bits(x0, x1)
    x0, s0, x1, s1 = _both(lambda: S.invert_mixed(dA, leaf=256, mode="fp32", ns_steps=2))
    assert _same_bits(x0, x1)


def test_batch_spec_equals_search(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    mats = [_dev(torch, W.diag_dominant(n, seed=n)) for n in (64, 200, 384)]
    mats.append(_dev(torch, _swap_rows(W.diag_dominant(256, seed=3), 10, 11)))

    def run():
        outs, info = S.invert_batch(mats, leaf=128, modes=["fp64", "fp32", "fp64", "fp64"])
        assert all(s == 0 for s in info), info
        return torch.cat([o.reshape(-1) for o in outs])

    x0, _, x1, _ = _both(run)
    assert _same_bits(x0, x1)


@pytest.mark.parametrize("L,z", [(64, 20), (256, 20), (256, 45), (200, 150)])
def test_breakdown_reported_the_same(torch_cuda, L, z):
    """A zero row and column: both ways report the same 1-based column (for
    order 256 and 200 in either workgroup's half of a two-workgroup panel)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(L, seed=5)
    A[:, z] = 0.0
    A[z, :] = 0.0
    dA = _dev(torch, A)
    _, s0, _, s1 = _both(lambda: S.invert(dA, leaf=L))
    assert s0 == s1 == z + 1
    A = W.diag_dominant(L, seed=6)
    A[7, 3] = np.nan
    dA = _dev(torch, A)
    _, s0, _, s1 = _both(lambda: S.invert(dA, leaf=L))
    assert s0 == s1 and s0 > 0


@pytest.mark.parametrize("n,leaf", [(256, 256), (200, 256), (1024, 256)])
@pytest.mark.parametrize("spin", [1, 4])
def test_two_workgroup_panels_give_up_to_the_search(torch_cuda, n, leaf, spin):
    """Panels of leaves of order 129-256 run on two workgroups that wait for
    each other a bounded number of polls.  With that bound forced down
    (SPIN_DUO_SPIN) the waits run out, the panel falls back to the search, and
    the inverse is still the search's bit for bit (eager launches, so that no
    cached graph keeps the default bound)."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    A = W.diag_dominant(n, seed=n + spin)
    dA = _dev(torch, A)
    keys = ("SPIN_DUO_SPIN", "SPIN_NO_GRAPH")
    old = {k: os.environ.get(k) for k in keys}
    try:
        os.environ["SPIN_NO_GRAPH"] = "1"
        os.environ["SPIN_DUO_SPIN"] = str(spin)
        x0, s0, x1, s1 = _both(lambda: S.invert(dA, leaf=leaf))
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    assert s0 == s1 == 0
    assert _same_bits(x0, x1)
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    assert np.linalg.norm(x1 - ref) / np.linalg.norm(ref) <= 1e-13
