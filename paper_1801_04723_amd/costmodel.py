"""Cost model of the recursion on one GPU: the time of an order-n inversion
with leaf order L as a sum over its schedule, with per-launch costs measured
in isolation.

The paper prices its Spark schedule with a cost model (Sec. 4, Lemma 1, Eq. 1:
computation, communication and a parallelisation factor per method). It
compares that model with measured times over block counts (Fig. 4) and uses it
to explain why the time is U-shaped in the block size.  On one GPU the
communication terms disappear and the schedule is a strict chain, so
the model is additive:

    t(n, L) = sum over leaves of t_leaf(L_i) + sum over internal nodes of t_node(h)

* t_leaf(L): one leaf of order L inverted alone (all its launches);
* t_node(h): the four product launches of a node whose blocks have order h,
  {II, III}, S, {C12, C21}, C11.

The leaves run one after another on one compute unit, and their number n / L
halves as L doubles.  A leaf's cost grows faster than L (L pivot steps; above
order 128 also more panels, each with an update product), so the leaf term
grows with L.  The node term loses its deepest level each time L doubles, and
those are the launch-bound levels.  The U-curve is the sum of the two.

`calibrate()` measures both tables on the GPU (graph-replayed inversions for
leaves and small nodes, standalone products for large nodes); `predict()` and
`best_leaf()` are plain host arithmetic on them.
"""
from __future__ import annotations

from collections import Counter
from dataclasses import dataclass, field


def schedule(n: int, leaf: int) -> tuple[Counter, Counter]:
    """(leaves by order, internal nodes by (n1, n2)) of the plain schedule."""
    from . import plan_describe
    ops, _ = plan_describe(n, leaf)
    leaves = Counter(o["L"] for o in ops if o["kind"] == "leaf")
    nodes = Counter()
    for o in ops:
        # the first launch of every node is {II, III}: II = A21 I is n2 x n1 x n1
        if o["kind"] == "products" and len(o["products"]) == 2 and o["products"][0]["beta"] == 0.0 \
                and o["products"][0]["alpha"] == 1.0:
            p = o["products"][0]
            nodes[(p["k"], p["m"])] += 1
    return leaves, nodes


@dataclass
class Rates:
    """Milliseconds per leaf of order L and per internal node of block order h."""
    leaf_ms: dict = field(default_factory=dict)
    node_ms: dict = field(default_factory=dict)

    def leaf(self, L: int) -> float:
        return _interp(self.leaf_ms, L)

    def node(self, n1: int, n2: int) -> float:
        # ragged nodes (n1 > n2 by at most 64) are priced as the larger order
        return _interp(self.node_ms, max(n1, n2))


def _interp(table: dict, x: int) -> float:
    """Exact entry, else log-log interpolation between the nearest entries."""
    import math
    if x in table:
        return table[x]
    keys = sorted(table)
    lo = max((k for k in keys if k < x), default=keys[0])
    hi = min((k for k in keys if k > x), default=keys[-1])
    if lo == hi:
        return table[lo] * (x / lo) ** 3
    t = (math.log(x) - math.log(lo)) / (math.log(hi) - math.log(lo))
    return math.exp(math.log(table[lo]) + t * (math.log(table[hi]) - math.log(table[lo])))


def predict(n: int, leaf: int, rates: Rates) -> dict:
    """Predicted milliseconds, split into the leaf and node terms."""
    leaves, nodes = schedule(n, leaf)
    t_leaf = sum(c * rates.leaf(L) for L, c in leaves.items())
    t_node = sum(c * rates.node(n1, n2) for (n1, n2), c in nodes.items())
    return {"ms": t_leaf + t_node, "leaf_ms": t_leaf, "node_ms": t_node,
            "leaves": sum(leaves.values()), "nodes": sum(nodes.values())}


def best_leaf(n: int, rates: Rates, candidates=(32, 64, 128, 256, 512, 1024, 2048)) -> int:
    """The candidate leaf order with the smallest predicted time."""
    return min((c for c in candidates if c <= max(n, 1)), key=lambda c: predict(n, c, rates)["ms"])


# ------------------------------------------------------------- calibration
def _time_ms(fn, reps: int, warm: int = 2) -> float:
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _dd(n: int, seed: int):
    import workloads as W
    return W.torch_diag_dominant(n, seed)


def calibrate(leaves=(32, 64, 128, 256, 512, 1024, 2048), hs=(32, 64, 128, 256, 512, 1024, 2048, 4096, 8192),
              large_h: int = 1024) -> Rates:
    """Measure t_leaf(L) and t_node(h) on the current GPU.

    * t_leaf(L): spin_invert of an order-L matrix with leaf L (graph replay);
    * t_node(h), h < large_h: t(2h, leaf h) - 2 t_leaf(h), both graph-replayed,
      so the launch gaps inside a schedule are included;
    * t_node(h), h >= large_h: the node's four launches as standalone products
      (a pair timed as one (2h x h x h) product, which has the same tile
      configuration at these sizes), launched back to back.
    """
    import torch
    from . import invert, gemm_cm, release
    r = Rates()
    for L in sorted(set(leaves) | {h for h in hs if h < large_h}):
        A = _dd(L, L)
        X = torch.empty_like(A)
        r.leaf_ms[L] = _time_ms(lambda: invert(A, leaf=L, out=X), reps=20 if L <= 512 else 5)
        del A, X
    for h in hs:
        if h < large_h:
            A = _dd(2 * h, h)
            X = torch.empty_like(A)
            t = _time_ms(lambda: invert(A, leaf=h, out=X), reps=20)
            r.node_ms[h] = max(t - 2 * r.leaf_ms[h], 0.0)
            del A, X
        else:
            a = torch.randn(2 * h, h, dtype=torch.float64, device="cuda")
            b = torch.randn(h, h, dtype=torch.float64, device="cuda")
            c = torch.randn(h, h, dtype=torch.float64, device="cuda")
            d = torch.empty(2 * h, h, dtype=torch.float64, device="cuda")
            reps = 10 if h <= 4096 else 3
            pair = _time_ms(lambda: gemm_cm(2 * h, h, h, 1.0, a, 2 * h, b, h, 0.0, None, 2 * h, d, 2 * h),
                            reps=reps)
            single = _time_ms(lambda: gemm_cm(h, h, h, -1.0, a, 2 * h, b, h, 1.0, c, h, d, 2 * h),
                              reps=reps)
            r.node_ms[h] = 2 * pair + 2 * single
            del a, b, c, d
        release()
        torch.cuda.empty_cache()
    return r
