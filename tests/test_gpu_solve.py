"""GPU parity of the builder and the single solve against the CPU oracle.

Every case runs the same seeded arrays through libsssp.so (via the C ABI)
and through the oracle, and compares: the built CSR/CSC arrays exactly,
costs bit-exactly (int32 and float32), pred exactly under the tie rule, and
rounds / settled / relaxed / scanned exactly against the round simulator.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import (assert_same_solution, check_solver_copy, expected_order, oracle_solution,
                      sync, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def check_build(sp, n, src, dst, w, order="auto", scope="auto", relax="auto"):
    G = sp.Graph(n, src, dst, w, order=order, scope=scope, relax=relax)
    want = expected_order(n, src, dst) if order == "auto" else order
    assert G.order == (want if len(src) else "input"), (G.order, want)
    check_solver_copy(G, n, src, dst, w)
    A = {k: to_np(v) for k, v in G.arrays().items()}
    O = oracle.csr(n, src, dst)
    ow, iw, wmin = O.weights(w)
    assert np.array_equal(A["out_off"], O.out_off)
    assert np.array_equal(A["out_dst"], O.out_dst)
    assert np.array_equal(A["in_off"], O.in_off)
    assert np.array_equal(A["in_src"], O.in_src)
    assert np.array_equal(A["in_eid"], O.in_eid)
    assert np.array_equal(to_np(G.perm), O.perm)
    if w.dtype == np.int32:
        assert np.array_equal(A["out_w"], ow) and np.array_equal(A["in_w"], iw)
        assert np.array_equal(A["out_wmin"], wmin)
    else:
        assert np.array_equal(A["out_w"].view(np.int32), ow.view(np.int32))
        assert np.array_equal(A["in_w"].view(np.int32), iw.view(np.int32))
        assert np.array_equal(A["out_wmin"].view(np.int32), wmin.view(np.int32))
    assert G.csr.w_max == float(w.max()) if len(w) else True
    return G


def run_case(sp, n, src, dst, w, source, label, order="auto", scope="auto", relax="auto"):
    print("case", label, "n=%d m=%d order=%s scope=%s relax=%s" % (n, len(src), order, scope,
                                                                  relax), flush=True)
    G = check_build(sp, n, src, dst, w, order, scope, relax)
    cost, pred, st = sp.solve(G, source, with_pred=True, with_stats=True)
    sync()
    ref = oracle_solution(n, src, dst, w, source, G.effective_scope, G.effective_relax,
                          G.effective_delta)
    assert_same_solution(cost, pred, st, ref, label)
    # a second solve on the same graph reuses the workspace
    cost2, pred2, _ = sp.solve(G, source, with_pred=True)
    sync()
    assert np.array_equal(to_np(cost2), to_np(cost)) and np.array_equal(to_np(pred2), to_np(pred))
    return G, st


def test_tiny_worked_example(sp):
    src = np.array([0, 0, 1, 1, 2, 2, 4, 3], np.int32)
    dst = np.array([1, 2, 3, 4, 3, 4, 3, 2], np.int32)
    w = np.array([9, 2, 3, 2, 6, 5, 8, 1], np.int32)
    G, st = run_case(sp, 5, src, dst, w, 0, "worked-example")
    assert st["rounds"] == 3 and to_np(sp.solve(G, 0)[0]).tolist() == [0, 9, 2, 8, 7]


def test_edge_cases(sp):
    # single vertex, no edges
    run_case(sp, 1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), 0,
             "n1")
    # source without out-edges, others unreachable
    run_case(sp, 4, np.array([1, 2], np.int32), np.array([2, 3], np.int32),
             np.array([5, 5], np.int32), 0, "isolated-source")
    # self-loops and duplicates only
    run_case(sp, 3, np.array([0, 0, 0, 1, 1], np.int32), np.array([0, 1, 1, 1, 2], np.int32),
             np.array([1, 7, 3, 2, 4], np.int32), 0, "loops-dups")
    # path: rounds = k + 1
    k = 300
    src = np.arange(k, dtype=np.int32)
    G, st = run_case(sp, k + 1, src, src + 1, np.full(k, 2, np.int32), 0, "path")
    assert st["rounds"] == k + 1
    # star with a hub of 100k leaves (one huge frontier item)
    leaves = 100000
    src = np.zeros(leaves, np.int32)
    dst = np.arange(1, leaves + 1, dtype=np.int32)
    w = gen.weights_int(7, leaves, 1, 1000)
    G, st = run_case(sp, leaves + 1, src, dst, w, 0, "star")
    assert st["rounds"] == 2
    # in-star: a vertex with 200k in-edges from a fan (huge open item)
    fan = 200000
    src = np.concatenate([np.zeros(fan, np.int32), np.arange(1, fan + 1, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, fan + 1, dtype=np.int32),
                          np.full(fan, fan + 1, np.int32)])
    w = gen.weights_int(8, 2 * fan, 1, 1000)
    run_case(sp, fan + 2, src, dst, w, 0, "in-star")


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_builder_gaps_and_long_lists(sp, dtype):
    """Offsets and minimum out-weights where long runs of vertices have no
    edges (before, between and after the used ids) and out-lists cross many
    fixed-size position chunks of the builder, the lightest edge anywhere in
    a list."""
    rng = np.random.default_rng(61)
    n = 300000
    used = np.array([5, 6, 150000, 150001, 299990], np.int32)
    degs = [1000, 3, 700, 1, 257]
    src = np.concatenate([np.full(d, u, np.int32) for u, d in zip(used, degs)])
    dst = used[rng.integers(0, len(used), len(src))].astype(np.int32)
    if dtype == "i32":
        w = rng.integers(2, 1000, len(src)).astype(np.int32)
        w[rng.integers(0, len(src), 4)] = 1
    else:
        w = (rng.integers(2, 2**24, len(src)) * 2.0 ** -24).astype(np.float32)
        w[rng.integers(0, len(src), 4)] = 2.0 ** -24
    for source in (5, 299990):
        run_case(sp, n, src, dst, w, source, "gaps-%s-%d" % (dtype, source))


@pytest.mark.parametrize("order", ["auto", "degree"])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_random_small(sp, dtype, order):
    rng = np.random.default_rng(21)
    for trial in range(30):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 6 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        if dtype == "i32":
            w = rng.integers(1, 50, m).astype(np.int32)
        else:
            w = (rng.integers(1, 2**24, m) * 2.0 ** -24).astype(np.float32)
        run_case(sp, n, src, dst, w, int(rng.integers(0, n)), "rand-%s-%d" % (dtype, trial),
                 order)


def test_unit_weights_bfs(sp):
    g = gen.grid_workload(side=64)
    w = np.ones(g.m, np.int32)
    G, st = run_case(sp, g.n, g.src, g.dst, w, g.source, "grid64-unit")
    hops = oracle.bfs(g.n, g.src, g.dst, g.source)
    assert st["rounds"] == hops.max() + 1


@pytest.mark.parametrize("order", ["input", "degree"])
def test_float_equal_cost_ties(sp, order):
    tiny = np.float32(2.0 ** -30)
    src = np.array([2, 0, 1, 1, 2, 3], np.int32)
    dst = np.array([1, 1, 2, 1, 3, 2], np.int32)
    w = np.array([tiny, 1.0, tiny, tiny, tiny, tiny], np.float32)
    run_case(sp, 4, src, dst, w, 0, "f32-ties", order)
    # many equal-cost tiny edges on a grid of cost-1 vertices
    gr = gen.grid_workload(side=40)
    w = np.full(gr.m, tiny, np.float32)
    src = np.concatenate([gr.src, np.full(1, gr.n, np.int32)])
    dst = np.concatenate([gr.dst, np.full(1, gr.source, np.int32)])
    w = np.concatenate([w, np.ones(1, np.float32)])
    run_case(sp, gr.n + 1, src, dst, w, gr.n, "f32-ties-grid", order)


@pytest.mark.parametrize("order", ["auto", "degree"])
def test_workload_random_4096(sp, order):
    g = gen.random_workload()
    run_case(sp, g.n, g.src, g.dst, g.w, g.source, "random4096", order)


@pytest.mark.parametrize("scale,order", [(10, "auto"), (10, "input"), (14, "auto"),
                                         (14, "input"), (16, "auto")])
def test_rmat_scaled(sp, scale, order):
    g = gen.rmat_workload(scale=scale)
    G, _ = run_case(sp, g.n, g.src, g.dst, g.w, g.source, "rmat%d" % scale, order)
    if order == "auto":
        assert G.order == "degree"


@pytest.mark.parametrize("scope,relax", [("open", "setting"), ("all", "setting"),
                                         ("open", "correcting"), ("all", "correcting")])
def test_scope_and_relax_modes(sp, scope, relax):
    """Each C scope and relax step against the round simulator in the same
    mode, on every workload family and the degenerate shapes."""
    rng = np.random.default_rng(23)
    for trial in range(12):
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 6 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        if trial % 2:
            w = rng.integers(1, 50, m).astype(np.int32)
        else:
            w = (rng.integers(1, 2**24, m) * 2.0 ** -24).astype(np.float32)
        run_case(sp, n, src, dst, w, int(rng.integers(0, n)), "scope-rand-%d" % trial,
                 ["input", "degree"][trial % 3 == 0], scope, relax)
    for order in ("input", "degree"):
        g = gen.rmat_workload(scale=14)
        run_case(sp, g.n, g.src, g.dst, g.w, g.source, "scope-rmat14-" + order, order, scope,
                 relax)
    g = gen.grid_workload(side=48)
    run_case(sp, g.n, g.src, g.dst, g.w, g.source, "scope-grid48", "auto", scope, relax)
    run_case(sp, g.n, g.src, g.dst, np.ones(g.m, np.int32), g.source, "scope-grid48-unit",
             "auto", scope, relax)
    for g in gen.batch_workload(count=2, nmin=1000, nmax=20000):
        run_case(sp, g.n, g.src, g.dst, g.w, g.source, "scope-" + g.name, "auto", scope, relax)
    # one vertex; no edges; a source with no out-edges; unreachable cycles
    run_case(sp, 1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), 0,
             "scope-single", "auto", scope, relax)
    src = np.array([1, 2, 3, 4, 0], np.int32)
    dst = np.array([2, 3, 1, 0, 5], np.int32)
    run_case(sp, 6, src, dst, np.array([3, 4, 5, 6, 7], np.int32), 0, "scope-cycle", "auto",
             scope, relax)
    # a vertex relaxed twice under label-correcting relax (hand-worked in the
    # oracle's pins): 0->1 (10), 0->2 (1), 2->1 (1), 1->3 (1)
    src = np.array([0, 0, 2, 1], np.int32)
    dst = np.array([1, 2, 1, 3], np.int32)
    G, st = run_case(sp, 4, src, dst, np.array([10, 1, 1, 1], np.int32), 0, "relax-twice",
                     "auto", scope, relax)
    assert st["relaxed_edges"] == (5 if relax == "correcting" else 4)


@pytest.mark.parametrize("side", [32, 128])
def test_grid_scaled(sp, side):
    g = gen.grid_workload(side=side)
    run_case(sp, g.n, g.src, g.dst, g.w, g.source, "grid%d" % side)


def test_batch_shape_graphs_single(sp):
    for g in gen.batch_workload(count=3, nmin=1000, nmax=30000):
        run_case(sp, g.n, g.src, g.dst, g.w, g.source, g.name)


@pytest.mark.parametrize("order", ["input", "degree"])
def test_set_weights_then_solve(sp, order):
    g = gen.rmat_workload(scale=12)
    G = sp.Graph(g.n, g.src, g.dst, g.w, order=order)
    w2 = gen.weights_int(77, g.m, 1, 255)
    G.set_weights(torch.from_numpy(w2[to_np(G.perm)]).cuda())
    sync()
    O = oracle.csr(g.n, g.src, g.dst)
    ow, iw, wmin = O.weights(w2)
    A = {k: to_np(v) for k, v in G.arrays().items()}
    assert np.array_equal(A["out_w"], ow) and np.array_equal(A["in_w"], iw)
    assert np.array_equal(A["out_wmin"], wmin)
    check_solver_copy(G, g.n, g.src, g.dst, w2)
    cost, pred, st = sp.solve(G, g.source, with_pred=True, with_stats=True)
    sync()
    ref = oracle_solution(g.n, g.src, g.dst, w2, g.source, G.effective_scope,
                          G.effective_relax, G.effective_delta)
    assert_same_solution(cost, pred, st, ref, "rmat12-reweighted-" + order)
    # invalid weights are refused before anything is written
    bad = torch.from_numpy(w2[to_np(G.perm)]).cuda()
    bad[g.m // 2] = 0
    with pytest.raises(sp.SSSPError) as e:
        G.set_weights(bad)
    assert e.value.status == sp.SSSP_ERR_WEIGHT
    sync()
    check_solver_copy(G, g.n, g.src, g.dst, w2)


def test_weight_and_graph_errors(sp):
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    with pytest.raises(sp.SSSPError) as e:
        sp.Graph(3, src, dst, np.array([1, 0], np.int32))
    assert e.value.status == sp.SSSP_ERR_WEIGHT
    with pytest.raises(sp.SSSPError) as e:
        sp.Graph(3, src, dst, np.array([1.0, np.nan], np.float32))
    assert e.value.status == sp.SSSP_ERR_WEIGHT
    with pytest.raises(sp.SSSPError) as e:
        sp.Graph(3, src, dst, np.array([1.0, -2.0], np.float32))
    assert e.value.status == sp.SSSP_ERR_WEIGHT
    with pytest.raises(sp.SSSPError) as e:
        sp.Graph(2, src, dst, np.array([1, 1], np.int32))
    assert e.value.status == sp.SSSP_ERR_GRAPH
    with pytest.raises(sp.SSSPError) as e:
        sp.Graph(3, src, dst, np.array([1, 2**30], np.int32))
    assert e.value.status == sp.SSSP_ERR_OVERFLOW


def test_workload_grid_1024_full(sp):
    g = gen.grid_workload()
    G, _ = run_case(sp, g.n, g.src, g.dst, g.w, g.source, "grid1024")
    assert G.order == "input"


def test_workload_rmat22_full(sp):
    g = gen.rmat_workload()
    G = sp.Graph(g.n, g.src, g.dst, g.w)
    print("case rmat22 built", G.order, flush=True)
    assert G.order == "degree"
    cost, pred, st = sp.solve(G, g.source, with_pred=True, with_stats=True)
    sync()
    ref = oracle_solution(g.n, g.src, g.dst, g.w, g.source, G.effective_scope,
                          G.effective_relax, G.effective_delta)
    assert_same_solution(cost, pred, st, ref, "rmat22")
    print("rmat22 rounds", st, flush=True)


@pytest.mark.parametrize("relax", ["setting", "correcting"])
def test_active_set_handovers(sp, relax):
    """Many hand-overs between the active block sets of the round kernel:
    small one-block thresholds and work units make the active set grow and
    shrink phase after phase, so parked blocks adopt resume points often (a
    block that took one hand-over's number with the next one's fields once
    ran a phase twice).  Repeated solves must all equal the oracle's."""
    g = gen.rmat_workload(scale=14)
    G = sp.Graph(g.n, g.src, g.dst, g.w, relax=relax, scope="open")
    ref = oracle_solution(g.n, g.src, g.dst, g.w, g.source, G.effective_scope,
                          G.effective_relax, G.effective_delta)
    sp.set_launch(dict(small_n=-1, wg=-1, solo_edges=256, block_units=256))
    try:
        for rep in range(6):
            print("handovers", relax, "solve", rep, flush=True)
            cost, pred, st = sp.solve(G, g.source, with_pred=True, with_stats=True)
            sync()
            assert_same_solution(cost, pred, st, ref, "handovers-%s-%d" % (relax, rep))
    finally:
        sp.set_launch(None)
