"""Host-side tests of the GPU library (no GPU needed).

* the shared library loads and exports every function include/spin.h declares;
* argument validation returns the documented codes before touching the GPU;
* the recursion schedule has the structure Alg. 2 prescribes (counts per
  internal node, leaves, levels), the flop count 2 n^3, the n^2 - L^2
  workspace bound, and the same split rule as the oracle;
* replaying the library's schedule on the CPU with the oracle's product and
  leaf inverse reproduces the oracle's literal Strassen recursion bit for bit
  (S-form schedule == V-form algorithm under IEEE sign symmetry).
"""
import ctypes
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_1801_04723_amd as S
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_header_symbol():
    L = S.lib()
    names = S.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -10, -11, -100, 17):
        assert S.strerror(code)
    assert "overlap" in S.strerror(-5)


def test_argument_validation_codes():
    L = S.lib()
    p = ctypes.c_void_p
    A = p(0x10000000)
    X = p(0x20000000)
    s = p(0)
    assert L.spin_invert(None, 4, 4, X, 4, 2, s) == -1
    assert L.spin_invert(A, 0, 4, X, 4, 2, s) == -2
    assert L.spin_invert(A, 8, 4, X, 8, 2, s) == -3
    assert L.spin_invert(A, 8, 8, X, 7, 2, s) == -3
    assert L.spin_invert(A, 8, 8, X, 8, 0, s) == -4
    assert L.spin_invert(A, 8, 8, X, 8, 4096, s) == -4
    # overlapping ranges: X starts inside A's last column
    assert L.spin_invert(A, 8, 8, p(0x10000000 + 8 * 60), 8, 2, s) == -5
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 2, 7, 2, None, s) == -6
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 2, 1, 9, None, s) == -6
    assert L.spin_gemm(5, 4, 4, 4, 1.0, A, 4, A, 4, 0.0, None, 4, X, 4, 0, s) == -6
    assert L.spin_gemm(0, 4, 4, 4, 1.0, A, 3, A, 4, 0.0, None, 4, X, 4, 0, s) == -3
    assert L.spin_gemm(0, 4, 4, 4, 1.0, A, 4, A, 4, 1.0, None, 4, X, 4, 0, s) == -1
    assert L.spin_workspace_bytes(0, 4, 0) == 0
    assert L.spin_workspace_bytes(64, 4, 9) == 0
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 2, 0, 2, None, s) == -6  # FP64 is not mixed
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 2, 4, 2, None, s) == -6
    assert L.spin_gemm(4, 4, 4, 4, 1.0, A, 4, A, 4, 0.0, None, 4, X, 4, 0, s) == -6
    # the symmetric variant validates exactly like spin_invert, before any GPU work
    assert L.spin_invert_spd(None, 4, 4, X, 4, 2, s) == -1
    assert L.spin_invert_spd(A, 0, 4, X, 4, 2, s) == -2
    assert L.spin_invert_spd(A, 8, 4, X, 8, 2, s) == -3
    assert L.spin_invert_spd(A, 8, 8, X, 7, 2, s) == -3
    assert L.spin_invert_spd(A, 8, 8, X, 8, 0, s) == -4
    assert L.spin_invert_spd(A, 8, 8, X, 8, 4096, s) == -4
    assert L.spin_invert_spd(A, 8, 8, p(0x10000000 + 8 * 60), 8, 2, s) == -5
    assert L.spin_plan_describe_spd(0, 1, 1, 1, None, 0, None) == -2
    assert L.spin_plan_describe_spd(8, 4, 8, 2, None, 0, None) == -3
    assert L.spin_plan_describe_spd(8, 8, 8, 0, None, 0, None) == -4
    assert L.spin_plan_describe_spd(8, 8, 8, 2, None, 3, None) == -1


def test_mixed_modes_share_one_layout():
    """The BF16 modes keep FP32 working copies: same workspace as FP32 mode."""
    for n, leaf in ((64, 16), (1000, 128), (4096, 256)):
        b1 = S.workspace_bytes(n, leaf, S.MIXED_FP32)
        assert b1 > S.workspace_bytes(n, leaf, S.FP64) > 0
        assert S.workspace_bytes(n, leaf, S.MIXED_BF16) == b1
        assert S.workspace_bytes(n, leaf, S.MIXED_BF16X3) == b1
        assert S.server_request_bytes(n, leaf, S.MIXED_BF16X3) == S.server_request_bytes(
            n, leaf, S.MIXED_FP32)
    assert S.MODES["bf16"] == S.MIXED_BF16 and S.MODES["bf16x3"] == S.MIXED_BF16X3


def _levels(n, leaf):
    return 0 if n <= leaf else 1 + max(_levels(oracle.split(n), leaf), _levels(n - oracle.split(n), leaf))


@pytest.mark.parametrize("n,leaf", [(256, 64), (8192, 256), (16384, 128), (16384, 2048), (2048, 2048)])
def test_schedule_counts_and_flops(n, leaf):
    ops, fl = S.plan_describe(n, leaf)
    d = int(math.log2(n // leaf))
    counts = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    leaves = [o for o in ops if o["kind"] == "leaf"]
    prods = [o for o in ops if o["kind"] == "products"]
    internal = 2 ** d - 1
    assert len(leaves) == 2 ** d                          # 2^(p-q) leaves
    assert len(prods) == 4 * internal                     # launches per node
    logical = sum(len(o["products"]) for o in prods)
    assert logical == counts["multiply_per_internal_node"] * internal
    # the two `subtract`s of each node become beta = 1 epilogues
    subtracts = sum(1 for o in prods for p in o["products"] if p["beta"] == 1.0)
    assert subtracts == counts["subtract_per_internal_node"] * internal
    assert fl == 2.0 * n ** 3
    # 2^i nodes at level i (Fig. 1)
    for lvl in range(d):
        nodes = {o["products"][0]["d"] for o in prods if o["level"] == lvl}
        assert len([o for o in prods if o["level"] == lvl]) == 4 * 2 ** lvl
    assert all(o["L"] == leaf for o in leaves)
    assert max(o["level"] for o in leaves) == d


@pytest.mark.parametrize("n,leaf", [(256, 64), (1024, 128), (8192, 256), (300, 64), (4160, 128), (100, 7)])
def test_workspace_bound(n, leaf):
    ws = S.plan_ws_elems(n, leaf)
    assert ws <= n * n
    if n % leaf == 0 and (n // leaf) & (n // leaf - 1) == 0:
        assert ws == n * n - leaf * leaf
    assert S.workspace_bytes(n, leaf, "fp64") >= 8 * ws
    assert S.workspace_bytes(n, leaf, "fp32") >= 4 * ws + 24 * n * n


@pytest.mark.parametrize("n,leaf", [(256, 64), (1024, 128), (8192, 256), (300, 64), (100, 7)])
@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_workspace_bytes_symmetric(n, leaf, mode):
    """The symmetric schedule's workspace (mode | SPIN_SYMMETRIC) is sized from
    its own plan: nonzero, and no larger than the plain schedule's."""
    plain = S.workspace_bytes(n, leaf, mode)
    sym = S.workspace_bytes(n, leaf, S.MODES[mode] | S.SYMMETRIC)
    assert 0 < sym <= plain
    assert S.workspace_bytes(n, leaf, 7 | S.SYMMETRIC) == 0


@pytest.mark.parametrize("m", list(range(1, 300, 7)) + [4096, 4160, 8191, 16384])
def test_split_rule_matches_oracle(m):
    if m == 1:
        ops, _ = S.plan_describe(1, 1)
        assert len(ops) == 1 and ops[0]["kind"] == "leaf"
        return
    ops, _ = S.plan_describe(m, min(m - 1, 2048))
    top = next(o for o in ops if o["kind"] == "products" and o["level"] == 0)
    n1 = top["products"][0]["k"]  # II = A21 I has inner dimension n1
    assert n1 == oracle.split(m)


def _run_schedule_on_cpu(A, leaf, spd=False, lu=False, fold=False):
    """Replay the library's schedule with the oracle's GEMM and leaf routines.

    fold=True replays it as the executor runs it: a product flagged
    folds_next stores only its lower triangle when it is a lower-half product,
    and also stores its result transposed (onto its own upper triangle for a
    mirror, into the transpose's destination otherwise); the next step is
    skipped."""
    n = A.shape[0]
    ops, _ = S.plan_describe(n, leaf, spd=spd, lu=lu)
    ws = S.plan_ws_elems_lu(n, leaf) if lu else S.plan_ws_elems(n, leaf)
    bufs = [np.asfortranarray(A).ravel(order="F").copy(),
            np.full(n * n, np.nan), np.full(max(ws, 1), np.nan)]

    def view(ref, r, c):
        b, off, ld = ref
        flat = bufs[b]
        return np.lib.stride_tricks.as_strided(flat[off:], shape=(r, c), strides=(8, 8 * ld))

    skip = False
    for i, o in enumerate(ops):
        if skip:
            skip = False
            continue
        if o["kind"] == "leaf":
            L = o["L"]
            src = np.array(view(o["src"], L, L))
            x, info = oracle.gj_inv(src)
            assert info == 0
            dst = view(o["dst"], L, L)
            dst[...] = x
        elif o["kind"] == "lu_leaf":
            L = o["L"]
            li, ui, info = oracle.lu_leaf(np.array(view(o["src"], L, L)))
            assert info == 0
            view(o["li"], L, L)[...] = li
            view(o["ui"], L, L)[...] = ui
        elif o["kind"] == "fill":
            view(o["dst"], o["m"], o["n"])[...] = 0.0
        elif o["kind"] == "transpose":
            src = np.array(view(o["src"], o["m"], o["n"]))
            view(o["dst"], o["n"], o["m"])[...] = src.T
        elif o["kind"] == "mirror":
            # a lower-half product followed by its mirror leaves the lower
            # triangle of the full product, whatever the upper one held
            d = view(o["dst"], o["n"], o["n"])
            iu = np.triu_indices(o["n"], 1)
            d[iu] = d.T[iu]
        else:
            results = []
            for p in o["products"]:
                a = np.array(view(p["a"], p["m"], p["k"]))
                b = np.array(view(p["b"], p["k"], p["n"]))
                prod = oracle.gemm(a, b)
                d = p["alpha"] * prod
                if p["beta"] != 0.0:
                    d = d + p["beta"] * np.array(view(p["c"], p["m"], p["n"]))
                results.append((p, d))
            if fold and o["folds_next"]:
                (p, d), = results
                nxt = ops[i + 1]
                dv = view(p["d"], p["m"], p["n"])
                if p["lower"]:
                    assert nxt["kind"] == "mirror" and nxt["dst"] == p["d"]
                    il = np.tril_indices(p["m"])
                    dv[il] = d[il]
                    iu = np.triu_indices(p["m"], 1)
                    dv[iu] = d.T[iu]
                else:
                    assert nxt["kind"] == "transpose" and nxt["src"] == p["d"]
                    dv[...] = d
                    view(nxt["dst"], p["n"], p["m"])[...] = d.T
                skip = True
                continue
            for p, d in results:
                view(p["d"], p["m"], p["n"])[...] = d
    return bufs[1].reshape((n, n), order="F")


@pytest.mark.parametrize("gen,n,leaf", [("dd", 256, 64), ("spd", 128, 16), ("dd", 200, 32), ("hh", 96, 16)])
def test_schedule_replay_equals_oracle_bitwise(gen, n, leaf):
    A = {"dd": lambda: W.diag_dominant(n, 1), "spd": lambda: W.spd_gram(n, 2),
         "hh": lambda: W.householder(n, 3)}[gen]()
    X = _run_schedule_on_cpu(A, leaf)
    ref, info = oracle.strassen_inv(A, leaf)
    assert info == 0
    assert np.array_equal(X, ref)


@pytest.mark.parametrize("n,leaf", [(256, 64), (128, 16), (200, 32), (300, 64), (130, 64), (64, 64)])
def test_spd_schedule_replay_equals_oracle_bitwise(n, leaf):
    """The four-product schedule of spin_invert_spd, replayed with the oracle's
    product and leaf routines, is O3 bit for bit (S-form against V-form)."""
    A = W.spd_gram(n, 2)
    X = _run_schedule_on_cpu(A, leaf, spd=True)
    ref, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    assert np.array_equal(X, ref)


@pytest.mark.parametrize("n,leaf", [(256, 64), (200, 32), (300, 64), (130, 64), (5, 2)])
def test_spd_folded_schedule_replay_equals_oracle_bitwise(n, leaf):
    """Every mirror and transpose of the symmetric schedule is folded into the
    epilogue of the product before it, and the schedule run that way is still
    O3 bit for bit."""
    A = W.spd_gram(n, 2)
    ops, _ = S.plan_describe(n, leaf, spd=True)
    for i, o in enumerate(ops):
        if o["kind"] in ("mirror", "transpose"):
            assert ops[i - 1]["kind"] == "products" and ops[i - 1]["folds_next"]
    for lda, ldx in ((n, n), (n + 3, n + 5)):
        assert all(ops[i - 1]["folds_next"]
                   for ops in [S.plan_describe(n, leaf, lda, ldx, spd=True)[0]]
                   for i, o in enumerate(ops) if o["kind"] in ("mirror", "transpose"))
    assert not any(o.get("folds_next") for o in S.plan_describe(n, leaf)[0])
    X = _run_schedule_on_cpu(A, leaf, spd=True, fold=True)
    ref, info = oracle.strassen_inv_spd(A, leaf)
    assert info == 0
    assert np.array_equal(X, ref)


def _spd_flops(m, leaf):
    """Direct sum over the recursion: 2 L^3 per leaf; per node II (2 n2 n1 n1),
    the lower half of S (n2 (n2 + 1) n1), C21 (2 n2 n1 n2) and the lower half
    of C11 (n1 (n1 + 1) n2)."""
    if m <= leaf:
        return 2 * m ** 3
    n1 = oracle.split(m)
    n2 = m - n1
    return (_spd_flops(n1, leaf) + _spd_flops(n2, leaf)
            + 2 * n2 * n1 * n1 + n2 * (n2 + 1) * n1 + 2 * n2 * n1 * n2 + n1 * (n1 + 1) * n2)


@pytest.mark.parametrize("n,leaf", [(256, 64), (8192, 256), (16384, 128), (300, 64), (4160, 128), (1, 1)])
def test_spd_plan_structure(n, leaf):
    ops, fl = S.plan_describe(n, leaf, spd=True)
    plain, fl_plain = S.plan_describe(n, leaf)
    assert fl == _spd_flops(n, leaf)
    leaves = [o for o in ops if o["kind"] == "leaf"]
    assert [(o["L"], o["col0"]) for o in leaves] == [(o["L"], o["col0"]) for o in plain if o["kind"] == "leaf"]
    internal = sum(1 for o in plain if o["kind"] == "products") // 4
    assert sum(1 for o in ops if o["kind"] == "transpose") == internal
    assert sum(1 for o in ops if o["kind"] == "mirror") == 2 * internal
    prods = [o for o in ops if o["kind"] == "products"]
    assert len(prods) == 4 * internal and all(len(o["products"]) == 1 for o in prods)
    # S and C11 (the second and fourth product of a node) are lower halves,
    # each followed by the mirror of the same block
    for i, o in enumerate(ops):
        if o["kind"] == "products" and o["products"][0]["lower"]:
            p = o["products"][0]
            assert p["m"] == p["n"] and ops[i + 1]["kind"] == "mirror"
            assert ops[i + 1]["dst"] == p["d"] and ops[i + 1]["n"] == p["m"]
    assert sum(1 for o in prods if o["products"][0]["lower"]) == 2 * internal
    if n % leaf == 0 and (n // leaf) & (n // leaf - 1) == 0:
        assert fl_plain == 2 * n ** 3
    for o in ops:
        if o["kind"] == "transpose":
            # C12 (n1 x n2) := C21 (n2 x n1)^T, both in the output
            assert o["src"][0] == 1 and o["dst"][0] == 1 and o["m"] <= o["n"]


@pytest.mark.parametrize("n,leaf", [(256, 64), (8192, 256), (300, 64), (100, 7)])
def test_spd_workspace_within_plain(n, leaf):
    """II and S per node: the SPD schedule never addresses more workspace than
    spin_plan_ws_elems (the plain schedule's) provides."""
    ops, _ = S.plan_describe(n, leaf, spd=True)
    ws = S.plan_ws_elems(n, leaf)
    top = 0
    for o in ops:
        refs = []
        if o["kind"] == "products":
            for p in o["products"]:
                refs += [(p["a"], p["m"], p["k"]), (p["b"], p["k"], p["n"]), (p["d"], p["m"], p["n"])]
                if p["beta"] != 0.0:
                    refs.append((p["c"], p["m"], p["n"]))
        elif o["kind"] == "leaf":
            refs += [(o["src"], o["L"], o["L"]), (o["dst"], o["L"], o["L"])]
        for (buf, off, ld), r, c in refs:
            if buf == 2:
                top = max(top, off + (c - 1) * ld + r)
    assert top <= ws


@pytest.mark.parametrize("gen,n,leaf", [("dd", 256, 64), ("spd", 128, 16), ("dd", 300, 64), ("dd", 64, 64),
                                        ("dd", 130, 32)])
def test_lu_schedule_replay_equals_oracle_bitwise(gen, n, leaf):
    """The block-LU schedule of spin_invert_lu, replayed with the oracle's
    product and LU-leaf routines (every buffer starting as NaN), is O4 bit for
    bit: every block it reads has been written, the zeros included."""
    A = W.diag_dominant(n, 1) if gen == "dd" else W.spd_gram(n, 2)
    X = _run_schedule_on_cpu(A, leaf, lu=True)
    ref, info = oracle.lu_inv(A, leaf)
    assert info == 0
    assert np.array_equal(X, ref)


@pytest.mark.parametrize("n,leaf", [(256, 64), (8192, 128), (300, 64), (1, 1)])
def test_lu_plan_structure(n, leaf):
    ops, fl = S.plan_describe(n, leaf, lu=True)
    plain, _ = S.plan_describe(n, leaf)
    assert [o["kind"] for o in ops[:2]] == ["fill", "fill"]
    leaves = [(o["L"], o["col0"]) for o in ops if o["kind"] == "lu_leaf"]
    assert leaves == [(o["L"], o["col0"]) for o in plain if o["kind"] == "leaf"]
    internal = sum(1 for o in plain if o["kind"] == "products") // 4
    prods = [o for o in ops if o["kind"] == "products"]
    assert len(prods) == 4 * internal + 1  # three pairs and S per node, then X = Ui Li
    last = prods[-1]["products"][0]
    assert (last["m"], last["n"], last["k"]) == (n, n, n) and last["d"][0] == 1
    expect = sum(4 / 3 * L ** 3 for L, _ in leaves) + sum(
        2.0 * p["m"] * p["n"] * p["k"] for o in prods for p in o["products"])
    assert abs(fl - expect) <= 1e-9 * fl


def test_lu_argument_validation():
    L = S.lib()
    p = ctypes.c_void_p
    A, X, s = p(0x10000000), p(0x20000000), p(0)
    assert L.spin_invert_lu(None, 4, 4, X, 4, 2, s) == -1
    assert L.spin_invert_lu(A, 8, 8, X, 8, 129, s) == -4  # LU leaves stop at 128
    assert L.spin_invert_lu(A, 8, 8, p(0x10000000 + 8 * 60), 8, 2, s) == -5
    assert L.spin_plan_describe_lu(8, 8, 8, 129, None, 0, None) == -4


# ------------------------------------------------------- server admission (CPU)
def _fake(i):
    return 0x100000000 + i * 0x10000000


def test_server_fifo_admission_by_footprint():
    """FIFO admission: requests start while their workspace fits the pool and a
    slot is free; a request that does not fit blocks those behind it."""
    L = S.lib()
    leaf = 64
    b256 = S.server_request_bytes(256, leaf, "fp64")
    b1024 = S.server_request_bytes(1024, leaf, "fp64")
    assert 0 < b256 < b1024
    # two small requests fit; the big one only fits once they have left
    pool = b1024 + b256
    srv = S.Server(pool, max_active=8, leaf=leaf)
    h = srv._h
    for i, n in enumerate([256, 256, 1024, 256]):
        rc = L.spin_server_submit(h, _fake(2 * i), n, n, _fake(2 * i + 1), n, 0, i)
        assert rc == 0
    assert srv.admit() == 2
    st = srv.stats()
    assert st == {"queued": 2, "active": 2, "pool_used": 2 * b256}
    assert srv.admit() == 0  # the 1024 request blocks the 256 behind it
    srv.close()


def test_server_slot_cap_and_validation():
    L = S.lib()
    srv = S.Server(1 << 30, max_active=3, leaf=64)
    h = srv._h
    for i in range(5):
        assert L.spin_server_submit(h, _fake(2 * i), 128, 128, _fake(2 * i + 1), 128, 1, i) == 0
    assert srv.admit() == 3
    assert srv.stats()["queued"] == 2
    assert L.spin_server_submit(h, None, 128, 128, _fake(99), 128, 0, 9) == -1
    assert L.spin_server_submit(h, _fake(90), 0, 128, _fake(91), 128, 0, 9) == -2
    assert L.spin_server_submit(h, _fake(90), 128, 100, _fake(91), 128, 0, 9) == -3
    assert L.spin_server_submit(h, _fake(90), 128, 128, _fake(91), 128, 5, 9) == -6
    # overlap of input and output
    assert L.spin_server_submit(h, _fake(90), 128, 128, _fake(90) + 8, 128, 0, 9) == -5
    srv.close()
    tiny = S.Server(1 << 20, max_active=2, leaf=64)
    assert L.spin_server_submit(tiny._h, _fake(1), 1024, 1024, _fake(2), 1024, 0, 0) == -10
    tiny.close()
    assert L.spin_server_create(0, 4, 64, 2) is None
    assert L.spin_invert_batch(-1, None, None, None, None, None, None, 64, 2, None, None) == -7


def test_server_symmetric_mode_validation():
    """FP64 | SYMMETRIC is a server/batch mode with the symmetric schedule's
    footprint; the flag with an unknown mode is rejected everywhere."""
    L = S.lib()
    leaf = 64
    for n in (1, 64, 200, 1024):
        sym = S.server_request_bytes(n, leaf, "fp64_sym")
        assert 0 < sym <= S.server_request_bytes(n, leaf, "fp64")
    bad = 4 | S.SYMMETRIC
    assert S.server_request_bytes(256, leaf, bad) == 0
    assert S.server_request_bytes(256, leaf, S.SYMMETRIC | 32) == 0
    srv = S.Server(1 << 30, max_active=2, leaf=leaf)
    h = srv._h
    assert L.spin_server_submit(h, _fake(0), 256, 256, _fake(1), 256, S.FP64 | S.SYMMETRIC, 0) == 0
    assert L.spin_server_submit(h, _fake(2), 256, 256, _fake(3), 256, bad, 1) == -6
    assert srv.admit() == 1
    assert srv.stats()["pool_used"] == S.server_request_bytes(256, leaf, "fp64_sym")
    srv.close()
    i64 = ctypes.c_int64 * 1
    ptrs = ctypes.c_void_p * 1
    rc = L.spin_invert_batch(1, ptrs(_fake(4)), i64(256), i64(256), ptrs(_fake(5)), i64(256),
                             (ctypes.c_int * 1)(bad), leaf, 2, None, None)
    assert rc == -6


def test_int8_emulation_inner_dimension_limit():
    """The INT8 residue products accumulate k terms of at most 128^2 in int32:
    k above 131071 could wrap, so it is rejected before any GPU work, for the
    product and for the INT8-refined inversion."""
    L = S.lib()
    p = ctypes.c_void_p
    A, B, D = p(0x10000000), p(0x20000000), p(0x30000000)
    big = 131072
    assert L.spin_gemm_int8(4, 4, big, A, 4, B, big, 0, None, 1, D, 4, 14, 0, 0, p(0)) == -2
    assert L.spin_gemm_int8(4, 4, 4, A, 4, B, 4, 3, None, 1, D, 4, 14, 0, 0, p(0)) == -6
    # far-apart fake buffers, so that the order-131072 ranges do not overlap
    assert L.spin_invert_mixed(p(1 << 44), big, big, p(1 << 46), big, 256,
                               S.MIXED_FP32 | S.REFINE_INT8, 2, None, p(0)) == -2
    assert L.spin_invert_mixed(p(1 << 44), big, big, p(1 << 46), big, 256, S.MIXED_FP32, 9, None,
                               p(0)) == -6
    assert 128 * 128 * 131071 < 2 ** 31 <= 128 * 128 * big


def test_symmetric_mixed_modes_validation():
    """Mixed modes with SYMMETRIC: the symmetric schedule's footprint (no more
    than the plain one's) in the server, accepted by spin_invert_mixed's
    validation; FP64 | SYMMETRIC is not a mixed mode."""
    L = S.lib()
    leaf = 64
    for m in (S.MIXED_FP32, S.MIXED_BF16, S.MIXED_BF16X3):
        for n in (1, 200, 1024):
            sym = S.server_request_bytes(n, leaf, m | S.SYMMETRIC)
            assert 0 < sym <= S.server_request_bytes(n, leaf, m)
    for name in ("fp32_sym", "bf16_sym", "bf16x3_sym"):
        assert S.MODES[name] & S.SYMMETRIC
    srv = S.Server(1 << 30, max_active=2, leaf=leaf)
    assert L.spin_server_submit(srv._h, _fake(0), 256, 256, _fake(1), 256,
                                S.MIXED_BF16X3 | S.SYMMETRIC, 0) == 0
    assert L.spin_server_submit(srv._h, _fake(2), 256, 256, _fake(3), 256, 4 | S.SYMMETRIC, 1) == -6
    srv.close()
    p = ctypes.c_void_p
    A, X = p(0x10000000), p(0x20000000)
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 4, S.FP64 | S.SYMMETRIC, 2, None, p(0)) == -6
    assert L.spin_invert_mixed(A, 8, 8, X, 8, 4, S.MIXED_FP32 | S.SYMMETRIC, 9, None, p(0)) == -6
