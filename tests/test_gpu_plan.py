"""GPU parity of replayed solves (HIP-graph plans) and the launch autotuner.

A plan records every kernel of a batch (one persistent launch) or of a
sequence of single solves into a HIP graph; each replay must give the
oracle's cost and pred and the round simulator's counters, instance by
instance, on every replay, with other GPU work in between.  Launch geometry
(grid size, one-block threshold, work per block) changes speed only: every
geometry the autotuner may pick gives the same bits and counters.
"""
import numpy as np
import pytest
import torch

import gen
from gpu_util import oracle_solution, sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


@pytest.fixture(scope="module")
def case(sp):
    """Six random f32 instances over three graphs (one of them scope ALL,
    one label-correcting), with the oracle's solution per instance."""
    glist = gen.batch_workload(count=3, nmin=1000, nmax=30000)
    graphs = [sp.Graph(glist[0].n, glist[0].src, glist[0].dst, glist[0].w, scope="open"),
              sp.Graph(glist[1].n, glist[1].src, glist[1].dst, glist[1].w, scope="all"),
              sp.Graph(glist[2].n, glist[2].src, glist[2].dst, glist[2].w, relax="correcting")]
    rng = np.random.default_rng(77)
    inst_graph = [0, 1, 2, 1, 0, 2]
    inst_source = [int(rng.integers(0, glist[g].n)) for g in inst_graph]
    refs = {}
    for gi, s in zip(inst_graph, inst_source):
        if (gi, s) not in refs:
            g = glist[gi]
            refs[(gi, s)] = oracle_solution(g.n, g.src, g.dst, g.w, s,
                                            graphs[gi].effective_scope,
                                            graphs[gi].effective_relax, graphs[gi].effective_delta)
    return dict(glist=glist, graphs=graphs, inst_graph=inst_graph, inst_source=inst_source,
                refs=refs)


def check_against_oracle(sp, case, cost, pred, stats, label):
    graphs, inst_graph, inst_source = case["graphs"], case["inst_graph"], case["inst_source"]
    bases, total = sp.batch_layout(graphs, inst_graph)
    assert cost.numel() == total
    c = to_np(cost)
    p = to_np(pred).astype(np.int64) if pred is not None else None
    for i, (gi, s) in enumerate(zip(inst_graph, inst_source)):
        ref = case["refs"][(gi, s)]
        sl = slice(bases[i], bases[i] + graphs[gi].n)
        assert np.array_equal(c[sl], ref["cost"]), (label, i)
        if p is not None:
            assert np.array_equal(p[sl], ref["pred"]), (label, i)
        if stats is not None:
            st = stats[i]
            assert st["rounds"] == ref["rounds"], (label, i, st, ref["rounds"])
            assert st["settled"] == ref["settles"], (label, i)
            assert st["relaxed_edges"] == ref["relaxed"], (label, i)
            assert st["scanned_in_edges"] == ref["scanned"], (label, i)
            assert st["open_visits"] == ref["open_visits"], (label, i)


@pytest.mark.parametrize("kind", ["batch", "sequence"])
def test_plan_replays_match_oracle(sp, case, kind):
    print("plan", kind, flush=True)
    plan = sp.Plan(case["graphs"], case["inst_graph"], case["inst_source"], kind=kind,
                   with_pred=True, with_stats=True)
    try:
        for rep in range(3):
            # poison the outputs, replay, check; eager work between replays
            plan.cost.fill_(-7 if plan.cost.dtype == torch.int32 else -7.0)
            plan.pred.fill_(-5)
            cost, pred = plan.run()
            sync()
            check_against_oracle(sp, case, cost, pred, plan.stats(), "%s-rep%d" % (kind, rep))
            c1, p1, _ = sp.solve_batch(case["graphs"], case["inst_graph"],
                                       case["inst_source"], with_pred=True)
            x = torch.arange(1 << 20, device="cuda", dtype=torch.float32).sum()
            sync()
            assert np.array_equal(to_np(c1), to_np(plan.cost))
            assert float(x) > 0
    finally:
        plan.close()


def test_plan_without_pred_or_stats(sp, case):
    plan = sp.Plan(case["graphs"], case["inst_graph"], case["inst_source"], kind="batch",
                   with_pred=False, with_stats=False)
    try:
        cost, pred = plan.run()
        sync()
        assert pred is None
        check_against_oracle(sp, case, cost, None, None, "no-pred")
        with pytest.raises(sp.SSSPError) as e:
            plan.stats()  # a batch plan made without counters has none
        assert e.value.status == sp.SSSP_ERR_ARG
    finally:
        plan.close()


@pytest.mark.parametrize("launch", [
    dict(blocks=1), dict(blocks=8), dict(blocks=64, solo_edges=-1),
    dict(solo_edges=1 << 30), dict(block_units=512), dict(blocks=128, block_units=65536)])
@pytest.mark.parametrize("kind", ["batch", "sequence"])
def test_geometry_changes_nothing(sp, case, kind, launch):
    print("geometry", kind, launch, flush=True)
    plan = sp.Plan(case["graphs"], case["inst_graph"], case["inst_source"], kind=kind,
                   with_pred=True, with_stats=True, launch=launch)
    try:
        cost, pred = plan.run()
        sync()
        check_against_oracle(sp, case, cost, pred, plan.stats(), "%s-%s" % (kind, launch))
    finally:
        plan.close()


def test_geometry_limits(sp, case):
    with pytest.raises(sp.SSSPError) as e:
        sp.Plan(case["graphs"], case["inst_graph"], case["inst_source"],
                launch=dict(blocks=1 << 20))
    assert e.value.status == sp.SSSP_ERR_ARG
    with pytest.raises(sp.SSSPError) as e:
        sp.set_launch(dict(blocks=1 << 20))
    assert e.value.status == sp.SSSP_ERR_ARG


def test_autotune_and_direct_geometry(sp, case):
    best, ms = sp.autotune(case["graphs"], case["inst_graph"], case["inst_source"],
                           kind="batch", reps=2)
    print("autotune", best, "%.3f ms" % ms, flush=True)
    assert ms > 0 and best["blocks"] >= 1 and best["block_units"] > 0
    plan = sp.Plan(case["graphs"], case["inst_graph"], case["inst_source"], with_stats=True,
                   launch=best)
    try:
        cost, pred = plan.run()
        sync()
        check_against_oracle(sp, case, cost, pred, plan.stats(), "tuned-plan")
    finally:
        plan.close()
    # the tuned geometry as the default of direct calls, then back
    sp.set_launch(dict(blocks=4, solo_edges=-1, block_units=256))
    try:
        cost, pred, stats = sp.solve_batch(case["graphs"], case["inst_graph"],
                                           case["inst_source"], with_pred=True, with_stats=True)
        sync()
        check_against_oracle(sp, case, cost, pred, stats, "set_launch")
        g, s = case["graphs"][1], case["inst_source"][1]
        c1, p1, st1 = sp.solve(g, s, with_pred=True, with_stats=True)
        sync()
        ref = case["refs"][(1, s)]
        assert np.array_equal(to_np(c1), ref["cost"])
        assert st1["rounds"] == ref["rounds"]
    finally:
        sp.set_launch(None)


def test_plan_sees_new_weights(sp):
    # a plan holds the graph's pointers: new weights reach the next replay
    g = gen.grid_workload(side=48)
    w = (np.random.default_rng(5).integers(1, 2**23, g.m) * 2.0 ** -23 + 0.5).astype(np.float32)
    G = sp.Graph(g.n, g.src, g.dst, w)
    plan = sp.Plan([G], [0, 0], [0, g.n - 1], kind="batch", with_stats=True)
    try:
        w2 = np.random.default_rng(6).permutation(w).astype(np.float32)
        for k, ww in enumerate((w, w2, w)):
            w_eid = torch.from_numpy(ww).cuda()[G.perm.long()]
            G.set_weights(w_eid)
            cost, pred = plan.run()
            sync()
            for i, s in enumerate((0, g.n - 1)):
                ref = oracle_solution(g.n, g.src, g.dst, ww, s, G.effective_scope,
                                      G.effective_relax, G.effective_delta)
                sl = slice(i * g.n, (i + 1) * g.n)
                assert np.array_equal(to_np(cost)[sl], ref["cost"]), (k, i)
                assert np.array_equal(to_np(pred)[sl].astype(np.int64), ref["pred"]), (k, i)
    finally:
        plan.close()
