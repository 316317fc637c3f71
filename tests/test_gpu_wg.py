"""GPU parity of the one-workgroup-per-instance path (every instance's
rounds in a workgroup of its own, state in global memory, block barriers
only) against the oracle and against the persistent kernel on the same
solves: single, target and batched, label-setting and label-correcting in
Delta buckets.  The default takes it for C scope OPEN graphs of low degree
spread; wg = 1 forces it (any scope-OPEN graph), wg = -1 turns it off.
"""
import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_same_solution, oracle_solution, sync, to_np

pytestmark = pytest.mark.gpu

PATHS = {"wg": dict(wg=1), "grid": dict(wg=-1)}


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def both(sp, g, label, scope="auto", relax="auto", delta=None, target=None, source=None):
    source = g.source if source is None else source
    G = sp.Graph(g.n, g.src, g.dst, g.w, scope=scope, relax=relax, delta=delta)
    assert G.n > 4096  # above the LDS solver
    print("wg case", label, "n=%d m=%d scope=%s relax=%s delta=%s target=%s" % (
        g.n, g.m, G.effective_scope, G.effective_relax, G.effective_delta, target), flush=True)
    ref = oracle_solution(g.n, g.src, g.dst, g.w, source, G.effective_scope, G.effective_relax,
                          G.effective_delta)
    out = {}
    for name, launch in PATHS.items():
        sp.set_launch(launch)
        try:
            if target is None:
                cost, pred, st = sp.solve(G, source, with_pred=True, with_stats=True)
                sync()
                assert_same_solution(cost, pred, st, ref, "%s-%s" % (label, name))
                out[name] = (to_np(cost), to_np(pred), st)
            else:
                cost, st = sp.solve_target(G, source, target, with_stats=True)
                sync()
                assert to_np(cost)[target] == ref["cost"][target], (label, name)
                out[name] = (to_np(cost), None, st)
        finally:
            sp.set_launch(None)
    (c1, p1, s1), (c2, p2, s2) = out["wg"], out["grid"]
    assert np.array_equal(c1, c2), label
    if p1 is not None:
        assert np.array_equal(p1, p2), label
    assert s1 == s2, (label, s1, s2)
    return s1


def grid_f32(side, seed):
    g = gen.grid_workload(side=side)
    w = (np.random.default_rng(seed).integers(0, 2**23 + 1, g.m) * 2.0 ** -23 + 0.5)
    return gen.Graph("gridf32_%d" % side, g.n, g.src, g.dst, w.astype(np.float32), g.source)


def test_grids_both_paths(sp):
    g = gen.grid_workload(side=128)          # int [1,1000]: AUTO takes Delta buckets
    st = both(sp, g, "grid128")
    both(sp, g, "grid128-setting", relax="setting")
    both(sp, g, "grid128-lc-inf", relax="correcting")
    both(sp, g, "grid128-delta-50", relax="correcting", delta=50)
    both(sp, g, "grid128-corner", source=0)
    f = grid_f32(96, 5)                      # f32 [0.5,1.5]: AUTO is label-setting
    both(sp, f, "grid96f32")
    both(sp, f, "grid96f32-delta", relax="correcting", delta=0.3)
    assert st["settled"] == g.n


def test_forced_on_skewed_open_graph(sp):
    # wg = 1 on a scope-OPEN R-MAT graph: big rounds in one workgroup
    g = gen.rmat_workload(scale=13)
    both(sp, g, "rmat13-open", scope="open")
    both(sp, g, "rmat13-open-lc", scope="open", relax="correcting", delta=64)


def test_targets_both_paths(sp):
    g = gen.grid_workload(side=100)
    for t in (g.source, 0, g.n - 1, g.source + 7):
        both(sp, g, "grid100-t%d" % t, target=t)


def test_batch_of_grids(sp):
    """A C5-shaped batch (grids, several sources, two graphs, one of them
    label-correcting), default path against the persistent kernel and the
    oracle, instance by instance."""
    f = grid_f32(80, 9)
    g72 = gen.grid_workload(side=72)  # float32 weights in [1, 1000]: AUTO takes Delta buckets
    gi = gen.Graph("gridwide72", g72.n, g72.src, g72.dst, g72.w.astype(np.float32), g72.source)
    graphs = [sp.Graph(f.n, f.src, f.dst, f.w), sp.Graph(gi.n, gi.src, gi.dst, gi.w)]
    assert graphs[1].effective_relax == "correcting" and graphs[0].effective_relax == "setting"
    glist = [f, gi]
    rng = np.random.default_rng(71)
    inst_graph = [0, 1, 0, 1, 0, 0, 1]
    inst_source = [int(rng.integers(0, glist[k].n)) for k in inst_graph]
    res = {}
    for name, launch in PATHS.items():
        sp.set_launch(launch)
        try:
            cost, pred, stats = sp.solve_batch(graphs, inst_graph, inst_source, with_pred=True,
                                               with_stats=True)
            sync()
        finally:
            sp.set_launch(None)
        res[name] = (to_np(cost), to_np(pred), stats)
        bases, _ = sp.batch_layout(graphs, inst_graph)
        for i, (k, s) in enumerate(zip(inst_graph, inst_source)):
            g = glist[k]
            ref = oracle_solution(g.n, g.src, g.dst, g.w, s, graphs[k].effective_scope,
                                  graphs[k].effective_relax, graphs[k].effective_delta)
            sl = slice(bases[i], bases[i] + g.n)
            assert_same_solution(cost[sl], pred[sl], stats[i], ref, "%s-%d" % (name, i))
    assert np.array_equal(res["wg"][0], res["grid"][0])
    assert np.array_equal(res["wg"][1], res["grid"][1])
    assert res["wg"][2] == res["grid"][2]
    # more instances than workgroups: blocks loop over instances
    sp.set_launch(dict(wg=1, blocks=2))
    try:
        cost, pred, stats = sp.solve_batch(graphs, inst_graph, inst_source, with_pred=True,
                                           with_stats=True)
        sync()
    finally:
        sp.set_launch(None)
    assert np.array_equal(to_np(cost), res["wg"][0]) and stats == res["wg"][2]


def test_plan_sequence_on_wg(sp):
    f = grid_f32(64, 13)
    G = sp.Graph(f.n, f.src, f.dst, f.w)
    srcs = [0, f.n - 1, 777]
    plan = sp.Plan([G], [0, 0, 0], srcs, kind="sequence", with_stats=True)
    try:
        cost, pred = plan.run()
        sync()
        stats = plan.stats()
        for i, s in enumerate(srcs):
            ref = oracle_solution(f.n, f.src, f.dst, f.w, s, G.effective_scope,
                                  G.effective_relax, G.effective_delta)
            sl = slice(i * f.n, (i + 1) * f.n)
            assert_same_solution(cost[sl], pred[sl], stats[i], ref, "seq-%d" % i)
    finally:
        plan.close()


@pytest.mark.parametrize("order", ["auto", "degree"])
def test_backward_both_paths(sp, order):
    """The backward pass with each tree in a workgroup of its own: the same
    bits as the grid-wide level pass (children summed in edge-id order on
    both), and the oracle's fp64 gradient within 1e-5 (relative norm)."""
    import oracle
    d, gco = gen.diff_workload(side=72, num_sources=6)
    G = sp.Graph(d.n, d.src, d.dst, d.w, order=order)
    srcs = [int(s) for s in d.sources]
    ig = [0] * len(srcs)
    gcost = torch.from_numpy(gco.reshape(-1)).cuda()
    out = {}
    for name, launch in PATHS.items():
        sp.set_launch(launch)
        try:
            cost, pred, _ = sp.solve_batch([G], ig, srcs)
            gw = sp.backward([G], ig, srcs, pred, gcost)
            sync()
        finally:
            sp.set_launch(None)
        out[name] = (to_np(pred), to_np(gw))
    assert np.array_equal(out["wg"][0], out["grid"][0])
    assert np.array_equal(out["wg"][1], out["grid"][1])
    O = oracle.csr(d.n, d.src, d.dst)
    ref = oracle.grad(O, srcs, out["wg"][0].astype(np.int64).reshape(len(srcs), d.n),
                      gco.astype(np.float64))
    err = np.linalg.norm(out["wg"][1].astype(np.float64) - ref) / np.linalg.norm(ref)
    assert err <= 1e-5, err


def test_batch_plan_on_wg(sp):
    """A batch plan of grid instances (the one-workgroup-per-instance path)
    replayed three times, each replay against the oracle."""
    f = grid_f32(64, 17)
    G = sp.Graph(f.n, f.src, f.dst, f.w)
    srcs = [0, f.n // 2 + 5, f.n - 1, 1234]
    refs = [oracle_solution(f.n, f.src, f.dst, f.w, s, G.effective_scope, G.effective_relax,
                            G.effective_delta) for s in srcs]
    plan = sp.Plan([G], [0] * len(srcs), srcs, kind="batch", with_stats=True)
    try:
        for rep in range(3):
            plan.cost.fill_(-1.0)
            cost, pred = plan.run()
            sync()
            stats = plan.stats()
            for i, ref in enumerate(refs):
                sl = slice(i * f.n, (i + 1) * f.n)
                assert_same_solution(cost[sl], pred[sl], stats[i], ref, "plan-%d-%d" % (rep, i))
    finally:
        plan.close()
