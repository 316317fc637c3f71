"""GPU parity of the one-workgroup solver for small graphs (n <= 4096, state
in LDS) and of the persistent kernel on the same graphs.

Both paths must give the oracle's cost and pred and the round simulator's
counters (rounds, settled, relaxed, scanned) in every C scope and relax
step, for int32 and float32 weights, in input and degree order, and the same
open-visit counts as each other.  The persistent kernel is forced with
small_n = -1 (sssp_set_launch); the dispatch boundary sits between 4096 and
4097 vertices.
"""
import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_same_solution, oracle_solution, sync, to_np

pytestmark = pytest.mark.gpu

PATHS = {"lds": None, "grid": dict(small_n=-1)}


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def both_paths(sp, n, src, dst, w, source, label, order="auto", scope="auto", relax="auto",
               target=None):
    """Solves on both paths; checks each against the oracle and the two
    against each other.  Returns the stats of the LDS path."""
    print("case", label, "n=%d m=%d order=%s scope=%s relax=%s target=%s" % (
        n, len(src), order, scope, relax, target), flush=True)
    G = sp.Graph(n, src, dst, w, order=order, scope=scope, relax=relax)
    ref = oracle_solution(n, src, dst, w, source, G.effective_scope, G.effective_relax,
                          G.effective_delta)
    out = {}
    for name, launch in PATHS.items():
        sp.set_launch(launch)
        try:
            if target is None:
                cost, pred, st = sp.solve(G, source, with_pred=True, with_stats=True)
                sync()
                assert_same_solution(cost, pred, st, ref, "%s-%s" % (label, name))
            else:
                cost, st = sp.solve_target(G, source, target, with_stats=True)
                pred = None
                sync()
                assert to_np(cost)[target] == ref["cost"][target], (label, name)
        finally:
            sp.set_launch(None)
        out[name] = (to_np(cost), None if pred is None else to_np(pred), st)
    (c1, p1, s1), (c2, p2, s2) = out["lds"], out["grid"]
    assert np.array_equal(c1, c2), label
    if p1 is not None:
        assert np.array_equal(p1, p2), label
    assert s1 == s2, (label, s1, s2)
    return s1


def rand_graph(rng, n, deg, dtype):
    m = int(rng.integers(0, deg * n + 1))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if dtype == "i32":
        w = rng.integers(1, 60, m).astype(np.int32)
    else:
        w = (rng.integers(1, 2**24, m) * 2.0 ** -24).astype(np.float32)
    return src, dst, w


@pytest.mark.parametrize("scope,relax", [("open", "setting"), ("all", "setting"),
                                         ("open", "correcting"), ("all", "correcting")])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_random_both_paths(sp, dtype, scope, relax):
    rng = np.random.default_rng(401 + 7 * len(scope) + len(relax) + (dtype == "f32"))
    for trial in range(8):
        n = int(rng.integers(1, 4097))
        src, dst, w = rand_graph(rng, n, 8, dtype)
        both_paths(sp, n, src, dst, w, int(rng.integers(0, n)),
                   "rand-%s-%s-%s-%d" % (dtype, scope, relax, trial),
                   ["input", "degree"][trial % 2], scope, relax)


def test_dispatch_boundary_and_workload(sp):
    g = gen.random_workload()  # n = 4096: the largest graph of the LDS path
    st = both_paths(sp, g.n, g.src, g.dst, g.w, g.source, "random4096")
    assert st["settled"] == 4095
    rng = np.random.default_rng(409)
    for n in (4095, 4096, 4097):
        src, dst, w = rand_graph(rng, n, 6, "i32")
        both_paths(sp, n, src, dst, w, 0, "boundary-%d" % n)


def test_degenerate_shapes(sp):
    z = np.zeros(0, np.int32)
    both_paths(sp, 1, z, z, z, 0, "n1")
    both_paths(sp, 4, np.array([1, 2], np.int32), np.array([2, 3], np.int32),
               np.array([5, 5], np.int32), 0, "isolated-source")
    # a path over the whole LDS capacity: one vertex fixed per round
    k = 4095
    src = np.arange(k, dtype=np.int32)
    st = both_paths(sp, k + 1, src, src + 1, np.full(k, 3, np.int32), 0, "path4096")
    assert st["rounds"] == k + 1
    # a hub with 4000 out-edges (several relax windows in one round)
    leaves = 4000
    src = np.zeros(leaves, np.int32)
    dst = np.arange(1, leaves + 1, dtype=np.int32)
    st = both_paths(sp, leaves + 1, src, dst, gen.weights_int(11, leaves, 1, 1000), 0, "star")
    assert st["rounds"] == 2
    # a vertex with 2000 in-edges (one long in-list)
    fan = 2000
    src = np.concatenate([np.zeros(fan, np.int32), np.arange(1, fan + 1, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, fan + 1, dtype=np.int32), np.full(fan, fan + 1, np.int32)])
    for scope in ("open", "all"):
        both_paths(sp, fan + 2, src, dst, gen.weights_int(12, 2 * fan, 1, 1000), 0,
                   "in-star-" + scope, scope=scope)
    # float32 equal-cost edges (w below half an ulp of the cost)
    src = np.array([0, 1, 2, 1, 3], np.int32)
    dst = np.array([1, 2, 1, 3, 2], np.int32)
    w = np.array([1.0, 2.0**-30, 2.0**-30, 0.5, 2.0**-30], np.float32)
    both_paths(sp, 4, src, dst, w, 0, "equal-cost")


@pytest.mark.parametrize("scope,relax", [("open", "setting"), ("all", "setting"),
                                         ("open", "correcting")])
def test_target_both_paths(sp, scope, relax):
    rng = np.random.default_rng(417)
    for trial in range(4):
        n = int(rng.integers(2, 4097))
        src, dst, w = rand_graph(rng, n, 8, ["i32", "f32"][trial % 2])
        for t in (0, int(rng.integers(0, n)), n - 1):
            both_paths(sp, n, src, dst, w, 0, "target-%d-%d" % (trial, t), scope=scope,
                       relax=relax, target=t)


def test_sequence_plan_of_small_graphs(sp):
    rng = np.random.default_rng(431)
    glist, graphs = [], []
    for k in range(5):
        n = int(rng.integers(1, 4097))
        src, dst, w = rand_graph(rng, n, 8, "f32")
        glist.append((n, src, dst, w))
        graphs.append(sp.Graph(n, src, dst, w))
    inst_graph = [0, 1, 2, 3, 4, 1]
    inst_source = [int(rng.integers(0, glist[g][0])) for g in inst_graph]
    plan = sp.Plan(graphs, inst_graph, inst_source, kind="sequence", with_stats=True)
    try:
        for rep in range(2):
            cost, pred = plan.run()
            sync()
            stats = plan.stats()
            bases, _ = sp.batch_layout(graphs, inst_graph)
            for i, (gi, s) in enumerate(zip(inst_graph, inst_source)):
                n, src, dst, w = glist[gi]
                ref = oracle_solution(n, src, dst, w, s, graphs[gi].effective_scope,
                                      graphs[gi].effective_relax, graphs[gi].effective_delta)
                sl = slice(bases[i], bases[i] + n)
                assert_same_solution(cost[sl], pred[sl], stats[i], ref, "plan-%d-%d" % (rep, i))
    finally:
        plan.close()
