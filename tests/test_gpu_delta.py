"""GPU parity of the Delta-bucketed label-correcting relax (Section I's
Delta-stepping with the method): an open vertex joins the relax set only
while D < minD + delta.  Against the oracle's round simulator with the same
delta (costs, parents, rounds, relaxed and scanned counts), on the
persistent kernel and on the one-workgroup solver, single and batched;
delta = 0 must reproduce label-setting's counters.
"""
import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_same_solution, oracle_solution, sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def run(sp, g, delta, scope="open", small=True, label=""):
    print("delta case", label, "n=%d delta=%s scope=%s small=%s" % (g.n, delta, scope, small),
          flush=True)
    G = sp.Graph(g.n, g.src, g.dst, g.w, scope=scope, relax="correcting", delta=delta)
    assert G.delta == (None if delta is None else delta)
    ref = oracle_solution(g.n, g.src, g.dst, g.w, g.source, G.effective_scope, "correcting",
                          delta=delta)
    sp.set_launch(None if small else dict(small_n=-1))
    try:
        cost, pred, st = sp.solve(G, g.source, with_pred=True, with_stats=True)
        sync()
    finally:
        sp.set_launch(None)
    assert_same_solution(cost, pred, st, ref, label)
    return st


def workloads():
    rng = np.random.default_rng(611)
    out = [gen.grid_workload(side=48), gen.rmat_workload(scale=12), gen.random_workload()]
    n = 3000
    m = 8 * n
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    w = (rng.integers(1, 2**24, m) * 2.0 ** -24).astype(np.float32)
    out.append(gen.Graph("randf32", n, src, dst, w, 0))
    return out


@pytest.mark.parametrize("small", [True, False])
@pytest.mark.parametrize("scope", ["open", "all"])
def test_delta_against_oracle(sp, scope, small):
    for g in workloads():
        f32 = g.w.dtype == np.float32
        wmean = float(np.mean(g.w))
        for delta in (0, (0.5 * wmean if f32 else int(wmean // 2)),
                      (4.0 * wmean if f32 else int(4 * wmean)), None):
            st = run(sp, g, delta, scope, small, "%s-%s" % (g.name, delta))
            if delta == 0:
                # delta = 0 never relaxes an open vertex: label-setting's counters
                ref = oracle_solution(g.n, g.src, g.dst, g.w, g.source,
                                      "all" if scope == "all" else "open", "setting")
                assert st["relaxed_edges"] == ref["relaxed"]
                assert st["rounds"] == ref["rounds"]


def test_delta_batch_mixed(sp):
    glist = gen.batch_workload(count=3, nmin=1000, nmax=20000)
    deltas = [0.0, 0.05, None]
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w, relax="correcting", delta=d)
              for g, d in zip(glist, deltas)]
    inst_graph = [0, 1, 2, 1]
    inst_source = [glist[gi].source for gi in inst_graph]
    cost, pred, stats = sp.solve_batch(graphs, inst_graph, inst_source, with_pred=True,
                                       with_stats=True)
    sync()
    bases, _ = sp.batch_layout(graphs, inst_graph)
    for i, (gi, s) in enumerate(zip(inst_graph, inst_source)):
        g = glist[gi]
        ref = oracle_solution(g.n, g.src, g.dst, g.w, s, graphs[gi].effective_scope,
                              "correcting", delta=deltas[gi])
        sl = slice(bases[i], bases[i] + g.n)
        assert_same_solution(cost[sl], pred[sl], stats[i], ref, "batch-%d" % i)


def test_delta_validation(sp):
    g = gen.random_workload()
    G = sp.Graph(g.n, g.src, g.dst, g.w, relax="correcting")
    with pytest.raises(ValueError):
        G.delta = -1
    G.delta = 2**40  # clamps to INF: no bound
    assert G.delta is None
