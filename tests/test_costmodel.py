"""Host checks of the recursion cost model (no GPU): its schedule counts against
the library's own schedule, and its sums against closed forms."""
import pytest

import paper_1801_04723_amd as S
from paper_1801_04723_amd import costmodel as C


@pytest.mark.parametrize("n,leaf", [(16384, 128), (8192, 256), (300, 64), (1000, 7), (64, 64)])
def test_schedule_counts_match_plan(n, leaf):
    leaves, nodes = C.schedule(n, leaf)
    ops, _ = S.plan_describe(n, leaf)
    assert sum(leaves.values()) == sum(1 for o in ops if o["kind"] == "leaf")
    # four product launches per internal node
    assert 4 * sum(nodes.values()) == sum(1 for o in ops if o["kind"] == "products")
    assert sum(L * c for L, c in leaves.items()) == n  # the leaves tile the diagonal


@pytest.mark.parametrize("n,leaf", [(16384, 128), (16384, 2048), (8192, 256), (1024, 1024)])
def test_predict_closed_form(n, leaf):
    """t_leaf = a L^3 and t_node = b h^3 give a n L^2 + (b n^3 / 8) sum_l 4^-l."""
    a, b = 2e-9, 3e-10
    hs = [2 ** k for k in range(4, 15)]
    r = C.Rates(leaf_ms={L: a * L ** 3 for L in hs}, node_ms={h: b * h ** 3 for h in hs})
    p = C.predict(n, leaf, r)
    d = (n // leaf).bit_length() - 1
    expect = a * n * leaf ** 2 + b * n ** 3 / 8 * sum(4.0 ** -l for l in range(d))
    assert abs(p["ms"] - expect) <= 1e-9 * expect
    assert p["leaves"] == n // leaf and p["nodes"] == n // leaf - 1


def test_interpolation_is_exact_on_entries_and_monotone():
    r = C.Rates(leaf_ms={64: 1.0, 256: 16.0})
    assert r.leaf(64) == 1.0 and r.leaf(256) == 16.0
    assert r.leaf(128) == pytest.approx(4.0)  # log-log: a power law between entries
    assert r.leaf(64) < r.leaf(100) < r.leaf(200) < r.leaf(256)


def test_best_leaf_is_the_minimum_of_a_u_curve():
    """Leaves cost a L^2 per unit of n, nodes a fixed launch floor each: the
    prediction is U-shaped and best_leaf finds its bottom."""
    hs = [2 ** k for k in range(4, 15)]
    r = C.Rates(leaf_ms={L: 1e-6 * L ** 2 for L in hs}, node_ms={h: 0.05 + 1e-12 * h ** 3 for h in hs})
    n = 16384
    t = {L: C.predict(n, L, r)["ms"] for L in (32, 64, 128, 256, 512, 1024, 2048)}
    best = C.best_leaf(n, r)
    assert t[best] == min(t.values())
    assert t[32] > t[best] < t[2048]
