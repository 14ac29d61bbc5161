"""Cross-request batching and the continuous-batching server on the GPU.

Every request's result must be bit for bit the one the single-call entry
points give it alone: each kernel computes a product or a leaf the same way
whichever requests share its launch, and each request's steps keep their
order.  Inputs are seeded; the oracle pins the solo results elsewhere, and
here the residual guards against a shared wrong answer.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_04723_amd  # noqa: F401
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).cuda().t()


def _solo(S, a, mode, leaf, ns_steps):
    if mode == "fp64":
        return S.invert(a, leaf=leaf)
    if mode == "fp64_sym":
        return S.invert_spd(a, leaf=leaf)
    return S.invert_mixed(a, leaf=leaf, mode=mode, ns_steps=ns_steps)


REQS = [(256, "dd", "fp64"), (320, "spd", "fp32"), (64, "dd", "fp64"), (512, "spdk", "fp32"),
        (130, "dd", "fp64"), (1024, "spd", "fp64"), (192, "spdk", "fp32"), (40, "dd", "fp32"),
        (384, "dd", "bf16x3"), (200, "dd", "bf16"), (512, "spd", "fp64_sym"),
        (200, "spdk", "fp64_sym"), (64, "spd", "fp64_sym"), (320, "spdk", "fp32_sym"),
        (256, "spd", "bf16x3_sym")]


def _mat(n, kind, seed):
    if kind == "dd":
        return W.diag_dominant(n, seed)
    if kind == "spd":
        return W.spd_gram(n, seed)
    return W.spd_spectrum(n, seed, kappa=1e3)


@pytest.mark.parametrize("leaf", [64, 128, 256])
def test_invert_batch_equals_solo_bitwise(torch_cuda, leaf):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    mats = [_dev(torch, _mat(n, k, 100 + i)) for i, (n, k, _) in enumerate(REQS)]
    modes = [m for _, _, m in REQS]
    outs, info = S.invert_batch(mats, leaf=leaf, modes=modes, ns_steps=2)
    assert info == [0] * len(REQS)
    for a, x, m, (n, k, _) in zip(mats, outs, modes, REQS):
        solo = _solo(S, a, m, leaf, 2)
        torch.cuda.synchronize()
        assert torch.equal(x, solo), (n, k, m)
        assert oracle.residual(a.cpu().numpy(), x.cpu().numpy()) <= 1e-12


def test_server_staggered_arrivals_equal_solo(torch_cuda):
    """Requests join while others are in flight and leave independently."""
    import paper_1801_04723_amd as S
    torch = torch_cuda
    leaf = 64
    srv = S.Server(1 << 32, max_active=4, leaf=leaf, ns_steps=2)
    mats = [_dev(torch, _mat(n, k, 300 + i)) for i, (n, k, _) in enumerate(REQS)]
    outs = [torch.empty_like(a) for a in mats]
    done = {}
    i = 0
    ticks = 0
    while len(done) < len(REQS):
        if i < len(REQS) and ticks % 3 == 0:  # one new request every third tick
            srv.submit(mats[i], outs[i], REQS[i][2], tag=i)
            i += 1
        st = srv.stats()
        if st["active"] or st["queued"]:
            srv.tick()
        for tag, info in srv.poll():
            done[tag] = info
        ticks += 1
        assert ticks < 100000
    srv.close()
    assert all(v == 0 for v in done.values())
    for a, x, (n, k, m) in zip(mats, outs, REQS):
        assert torch.equal(x, _solo(S, a, m, leaf, 2)), (n, k, m)


def test_singular_request_does_not_disturb_others(torch_cuda):
    import paper_1801_04723_amd as S
    torch = torch_cuda
    good = [_dev(torch, _mat(256, "dd", 7)), _dev(torch, _mat(320, "spd", 8))]
    bad_np = W.diag_dominant(256, 9)
    bad_np[:, 100] = 0.0
    bad_np[100, :] = 0.0
    mats = [good[0], _dev(torch, bad_np), good[1]]
    outs, info = S.invert_batch(mats, leaf=64, modes=["fp64", "fp64", "fp32"], ns_steps=2)
    assert info[0] == 0 and info[2] == 0 and info[1] == 101
    assert torch.equal(outs[0], S.invert(good[0], leaf=64))
    assert torch.equal(outs[2], S.invert_mixed(good[1], leaf=64, ns_steps=2))


@pytest.mark.parametrize("split,sym", [(None, False), ([128, 256], False), ([128, 256], True)])
def test_serving_loop_short_trace(torch_cuda, split, sym):
    """One lane, and three lanes on three streams split by order (SPD FP64
    requests on the plain or the symmetric schedule)."""
    import paper_1801_04723_amd.serve as serve
    import workloads as W
    trace = W.serving_trace(rate=100.0, duration=0.5, seed=11, n_max=512)
    stats = serve.run_trace(trace, leaf=64, ns_steps=2, pool_bytes=4 << 30, max_active=16,
                            split_n=split, symmetric=sym, check_every=3)
    assert stats["symmetric"] == sym
    assert stats["requests"] == len(trace) > 10
    assert stats["status_counts"] == {0: len(trace)}
    # every sampled result meets the residual target
    chk = stats["residual_check"]
    assert chk["mixed"]["count"] + chk["fp64"]["count"] >= len(trace) // 25
    for k in ("mixed", "fp64"):
        assert chk[k]["above_1e-12"] == 0 and chk[k]["nonzero_status"] == 0, chk
    assert stats["p50_ms"] <= stats["p99_ms"] <= stats["max_ms"]
    assert stats["lanes"] == (1 if split is None else 3)
