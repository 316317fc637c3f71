"""GPU parity of the single-target early exit (sssp_solve_target) against the
CPU oracle's round simulator stopped at the same point.

The rounds stop once the target is fixed, so the whole cost array (the upper
bounds D at the stop: exact for fixed vertices, tentative for the other
discovered ones, INF beyond) and the work counters must match the oracle bit
for bit; the target's own cost must equal Dijkstra's.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import oracle_mode, sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def check_target(sp, G, n, src, dst, w, source, target, label):
    print("case", label, "n=%d m=%d source=%d target=%d" % (n, len(src), source, target),
          flush=True)
    cost, st = sp.solve_target(G, source, target, with_stats=True)
    sync()
    mode = oracle_mode(G.effective_scope, G.effective_relax)
    ref = oracle.round_sim(n, src, dst, w, source, mode=mode, target=target,
                           delta=G.effective_delta)
    full, _ = oracle.dijkstra(n, src, dst, w, source)
    c = to_np(cost)
    bad = np.nonzero(c != ref["cost"])[0]
    assert bad.size == 0, "%s cost mismatch at %d vertices, first %s: gpu %s oracle %s" % (
        label, bad.size, bad[:5], c[bad[:5]], ref["cost"][bad[:5]])
    assert c[target] == full[target], label
    assert st["rounds"] == ref["rounds"], (label, st, ref["rounds"])
    assert st["settled"] == ref["settled"], (label, st, ref["settled"])
    assert st["relaxed_edges"] == ref["relaxed_edges"], (label, st, ref["relaxed_edges"])
    assert st["scanned_in_edges"] == ref["scanned_in_edges"], (label, st, ref["scanned_in_edges"])
    assert st["open_visits"] == ref["open_visits"], (label, st, ref["open_visits"])
    return st


def test_target_on_a_path(sp):
    k = 40
    src = np.arange(k, dtype=np.int32)
    dst = src + 1
    w = np.full(k, 7, np.int32)
    G = sp.Graph(k + 1, src, dst, w)
    for j in (0, 1, 2, 17, k):
        st = check_target(sp, G, k + 1, src, dst, w, 0, j, "path%d" % j)
        assert st["rounds"] == j and st["settled"] == j + 1


@pytest.mark.parametrize("order", ["auto", "degree"])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_target_random_small(sp, dtype, order):
    rng = np.random.default_rng(31 if dtype == "i32" else 32)
    for it in range(6):
        n = int(rng.integers(2, 3000))
        m = int(rng.integers(0, 8 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        if dtype == "i32":
            w = rng.integers(1, 1000, m).astype(np.int32)
        else:
            w = (rng.random(m) + 2.0 ** -20).astype(np.float32)
        s = int(rng.integers(0, n))
        G = sp.Graph(n, src, dst, w, order=order)
        full, _ = oracle.dijkstra(n, src, dst, w, s)
        reach = np.nonzero(full != (np.int32(2**31 - 1) if dtype == "i32" else np.inf))[0]
        unreach = np.setdiff1d(np.arange(n), reach)
        targets = [s, int(rng.choice(reach)), int(reach[np.argmax(full[reach])])]
        if unreach.size:
            targets.append(int(unreach[0]))
        for t in targets:
            check_target(sp, G, n, src, dst, w, s, t, "%s-%s-%d-t%d" % (dtype, order, it, t))


@pytest.mark.parametrize("scope,relax", [("open", "setting"), ("all", "setting"),
                                         ("open", "correcting")])
def test_target_rmat_and_grid(sp, scope, relax):
    g = gen.rmat_workload(scale=14)
    G = sp.Graph(g.n, g.src, g.dst, g.w, scope=scope, relax=relax)
    full, _ = oracle.dijkstra(g.n, g.src, g.dst, g.w, g.source)
    reach = np.nonzero(full != np.int32(2**31 - 1))[0]
    order = reach[np.argsort(full[reach], kind="stable")]
    unreach = np.setdiff1d(np.arange(g.n), reach)
    for t in (int(order[1]), int(order[len(order) // 2]), int(order[-1]), int(unreach[0])):
        check_target(sp, G, g.n, g.src, g.dst, g.w, g.source, t, "rmat14-t%d" % t)
    g = gen.grid_workload(side=64)
    G = sp.Graph(g.n, g.src, g.dst, g.w, scope=scope, relax=relax)
    for t in (0, g.n - 1, g.source + 1):
        check_target(sp, G, g.n, g.src, g.dst, g.w, g.source, t, "grid64-t%d" % t)


def test_target_rmat22_full(sp):
    g = gen.rmat_workload()
    G = sp.Graph(g.n, g.src, g.dst, g.w)
    full, _ = oracle.dijkstra(g.n, g.src, g.dst, g.w, g.source)
    reach = np.nonzero(full != np.int32(2**31 - 1))[0]
    t = int(reach[np.argsort(full[reach], kind="stable")][len(reach) // 2])
    st = check_target(sp, G, g.n, g.src, g.dst, g.w, g.source, t, "rmat22-median")
    print("rmat22 median target", st, flush=True)


def test_target_errors(sp):
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    G = sp.Graph(3, src, dst, np.array([1, 1], np.int32))
    for bad in (-1, 3):
        with pytest.raises(sp.SSSPError) as e:
            sp.solve_target(G, 0, bad)
        assert e.value.status == sp.SSSP_ERR_ARG
