"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

Each check compares the oracle with something it does not compute itself:
pure-Python path enumeration (the definition of cost[x] in Section I), the
paper's worked example, closed-form round counts, breadth-first search,
numpy's stable sort, and finite differences for the gradient.
"""
import itertools
import json
import os

import numpy as np
import pytest

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
I32_INF = np.int32(2**31 - 1)


def _inf(dt):
    return I32_INF if np.dtype(dt) == np.int32 else np.dtype(dt).type(np.inf)


def tiny_graph(rng, dtype, n=None, m=None):
    n = int(rng.integers(1, 9)) if n is None else n
    m = int(rng.integers(0, 5 * n + 1)) if m is None else m
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if np.dtype(dtype) == np.int32:
        w = rng.integers(1, 20, m).astype(np.int32)
    else:
        w = (rng.random(m) * 4 + 2.0 ** -20).astype(dtype)
    return n, src, dst, w, int(rng.integers(0, n))


def brute_force_paths(n, src, dst, w, s):
    """min over simple paths of the left-fold path sum in the weight type."""
    dt = w.dtype.type
    out = [None] * n
    out[s] = dt(0)
    adj = [[] for _ in range(n)]
    for i in range(len(src)):
        adj[int(src[i])].append((int(dst[i]), w[i]))

    def walk(v, acc, seen):
        for (y, wy) in adj[v]:
            if y in seen:
                continue
            if np.dtype(dt) == np.int32:
                c = dt(int(acc) + int(wy))
            else:
                c = dt(acc + wy)
            if out[y] is None or c < out[y]:
                out[y] = c
            seen.add(y)
            walk(y, c, seen)
            seen.discard(y)

    walk(s, dt(0), {s})
    res = np.full(n, _inf(w.dtype), dtype=w.dtype)
    for v in range(n):
        if out[v] is not None:
            res[v] = out[v]
    return res


@pytest.mark.parametrize("dtype", [np.int32, np.float32, np.float64])
def test_dijkstra_matches_path_enumeration(dtype):
    rng = np.random.default_rng(11)
    for _ in range(300):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 7)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        bf = brute_force_paths(n, src, dst, w, s)
        assert np.array_equal(c, bf), (n, src, dst, w, s, c, bf)
        assert settles == int(np.sum(c != _inf(dtype)))
        ca, sa = oracle.Adjacency(n, src, dst, w).dijkstra(s)
        assert np.array_equal(ca, bf) and sa == settles


@pytest.mark.parametrize("dtype", [np.int32, np.float32, np.float64])
def test_dijkstra_matches_bellman_ford(dtype):
    rng = np.random.default_rng(12)
    for _ in range(3000):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 13)),
                                       m=int(rng.integers(0, 61)))
        c, _ = oracle.dijkstra(n, src, dst, w, s)
        assert np.array_equal(c, oracle.bellman_ford(n, src, dst, w, s))


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_dijkstra_matches_dag_dp(dtype):
    rng = np.random.default_rng(13)
    for _ in range(300):
        n = int(rng.integers(2, 40))
        order = rng.permutation(n).astype(np.int32)
        m = int(rng.integers(0, 4 * n))
        a = rng.integers(0, n, m)
        b = rng.integers(0, n, m)
        keep = a != b
        lo, hi = np.minimum(a, b)[keep], np.maximum(a, b)[keep]
        src, dst = order[lo], order[hi]
        w = (rng.integers(1, 50, len(src)).astype(np.int32) if dtype == np.int32
             else rng.random(len(src)).astype(np.float32) + np.float32(2.0 ** -20))
        s = int(order[0])
        c, _ = oracle.dijkstra(n, src, dst, w, s)
        assert np.array_equal(c, oracle.dag(n, src, dst, w, s))


def test_unit_weights_are_bfs():
    for side in (1, 5, 17):
        g = gen.grid_workload(side=side)
        w = np.ones(g.m, dtype=np.int32)
        c, _ = oracle.dijkstra(g.n, g.src, g.dst, w, g.source)
        hops = oracle.bfs(g.n, g.src, g.dst, g.source)
        assert np.array_equal(np.where(hops < 0, I32_INF, hops), c)
    g = gen.random_workload(n=500, m=1200)
    w = np.ones(g.m, dtype=np.int32)
    c, _ = oracle.dijkstra(g.n, g.src, g.dst, w, g.source)
    hops = oracle.bfs(g.n, g.src, g.dst, g.source)
    assert np.array_equal(np.where(hops < 0, I32_INF, hops), c)


def _worked_graphs():
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    for extra in ex["edge_into_v2_variants"]:
        e = np.array(ex["edges_common"] + [extra], dtype=np.int64)
        yield ex, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32)


def test_worked_example_costs_pred_rounds():
    for ex, src, dst, w in _worked_graphs():
        n, s = ex["n"], ex["source"]
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        assert c.tolist() == ex["cost"]
        assert settles == 5
        # the paper's inWeight values (min in-weight other than from the
        # vertex that discovered v, SP_2) follow from the weights
        for v, iw in ex["inWeight"].items():
            z = ex["discovered_by"][v]
            assert int(w[(dst == int(v)) & (src != z)].min()) == iw
        g = oracle.csr(n, src, dst)
        p, ties = oracle.pred(g, w, s, c)
        tails = [-1 if e < 0 else int(src[g.perm[e]]) for e in p]
        assert tails == [-1, 0, 0, 2, 2] and ties == 0
        # Hand derivation of the adopted round on this graph:
        # round 1 relaxes v0: D1=9, D2=2; minD=2, thr=min(9+2, 2+5)=7.
        #   v1's only in-edge is from fixed v0 -> C1 = D1 -> fixed; D2=2<=thr -> fixed.
        # round 2 relaxes v1, v2: D3=8, D4=7; minD=7, thr=min(8+1, 7+8)=9 (or
        #   8+inf, 7+1 with the v4->v2 variant: thr=8): both D<=thr -> fixed.
        # round 3 relaxes v3, v4: no open vertex -> stop.  rounds=3, fixed [2,2,0].
        r = oracle.round_sim(n, src, dst, w, s, true_cost=c)
        assert r["cost"].tolist() == ex["cost"]
        assert r["rounds"] == 3 and r["fixed_per_round"].tolist() == [2, 2, 0]
        assert r["violations"] == 0
        # The step-(C) work, counted as every in-edge of every vertex the step
        # covers (in-degrees: v1 1, v2 2, v3 3, v4 2).  Scope OPEN covers
        # O = {v1, v2} in round 1 and O = {v3, v4} in round 2: [3, 5, 0], and
        # 4 open visits.  Scope ALL also covers the undiscovered non-fixed
        # vertices, v3 and v4 in round 1 (their C rises to 5 and 4, which
        # changes no fix here): [8, 5, 0].
        assert r["scanned_per_round"].tolist() == [3, 5, 0]
        assert r["scanned_in_edges"] == 8 and r["open_visits"] == 4
        a = oracle.round_sim(n, src, dst, w, s, mode=oracle.MODE_SCOPE_ALL, true_cost=c)
        assert a["rounds"] == 3 and a["fixed_per_round"].tolist() == [2, 2, 0]
        assert a["scanned_per_round"].tolist() == [8, 5, 0]
        assert a["scanned_in_edges"] == 13 and a["open_visits"] == 4
        assert a["relaxed_edges"] == r["relaxed_edges"] == 8


def test_worked_example_sp12_narratives():
    """The narratives of Sections III and IV run SP_1 and SP_2 on the worked
    example.  SP_1: v0 is removed; v1 is fixed when pred[1] reaches 0; v2 is
    removed next; exploring it fixes v4 (pred 0), and exploring v4 fixes v3
    (pred 0).  SP_2: the same start, but exploring v2 fixes v3 by Lemma
    inWeight (8 <= d + inWeight[3] = 2 + 6) before v4 (pred 0).  Both stop
    with every vertex fixed: two removeMin calls (v0, v2), the stale heap
    entries of v3 and v4 never removed (the overloaded H.empty()), four
    insertions (v0, then v2, v3, v4 from Q), no adjustment."""
    for ex, src, dst, w in _worked_graphs():
        n, s = ex["n"], ex["source"]
        c1, o1, f1 = oracle.sp12(n, src, dst, w, s, 1, sequence=True)
        c2, o2, f2 = oracle.sp12(n, src, dst, w, s, 2, sequence=True)
        assert c1.tolist() == c2.tolist() == ex["cost"]
        assert f1 == [(0, "removeMin"), (1, "pred"), (2, "removeMin"), (4, "pred"), (3, "pred")]
        assert f2 == [(0, "removeMin"), (1, "pred"), (2, "removeMin"), (3, "inWeight"),
                      (4, "pred")]
        for o in (o1, o2):
            assert o == dict(remove_min=2, insert=4, adjust=0, fixed_by_r=3)
        # Dijkstra in the same framework removes all five vertices
        c0, o0 = oracle.sp12(n, src, dst, w, s, 0)
        assert c0.tolist() == ex["cost"] and o0["remove_min"] == 5


def _scope_all_graph():
    """Vertices 0 (source), u = 1, y = 2, a = 3, b = 4, c = 5, z = 6; edges
    0->y (10), u->y (1), 0->a (1), a->b (1), b->c (1), y->z (1).  u has no
    in-edge, so it is never discovered."""
    src = np.array([0, 1, 0, 3, 4, 2], np.int32)
    dst = np.array([2, 2, 3, 4, 5, 6], np.int32)
    w = np.array([10, 1, 1, 1, 1, 1], np.int32)
    return 7, src, dst, w


def test_scope_all_round_semantics():
    """Step 4 of SP_4 raises C of every non-fixed vertex (Section VI); the
    adopted round's scope OPEN raises it for the discovered ones only.
    Worked by hand on _scope_all_graph (D: y 10, a 1, b 2, c 3, z 11):
    OPEN: round 1 fixes a (minD 1; y's in-edge from the undiscovered u holds
      m_y = max(C[u] = 0, minD) + 1 = 2 < 10); round 2 fixes b (C[y] = 3);
      round 3 fixes c and, since c has no out-edge, thr = min(10 + 1, 3 +
      inf) = 11 >= D[y], also y; round 4 fixes z; round 5 relaxes z and finds
      nothing open.  5 rounds, fixed [1, 1, 2, 1, 0].
    ALL: round 1 is the same for O = {y, a}, and the undiscovered vertices
      get C' = max(C, minD, m): u has no in-edge, so C[u] = inf; b, c, z get
      2.  Round 2 reads C[u] = inf, so m_y = inf and C'[y] = D[y] = 10: y is
      fixed with b.  Round 3 relaxes y and b (z: D 11, c: D 3) and fixes both
      (z's only in-edge has a fixed tail; c is the argmin).  Round 4 finds
      nothing open.  4 rounds, fixed [1, 2, 2, 0].
    Scanned in-edges (every in-edge of every covered vertex; in-degrees
    u 0, y 2, a 1, b 1, c 1, z 1): OPEN 3 + 3 + 3 + 1 = 10, one per round
    [3, 3, 3, 1, 0]; ALL (O, then the undiscovered vertices): round 1
    3 + 3, round 2 3 + 2, round 3 2 + 0: [6, 5, 2, 0] = 13.  Open visits:
    OPEN 2 + 2 + 2 + 1 = 7, ALL 2 + 2 + 2 = 6."""
    n, src, dst, w = _scope_all_graph()
    c, settles = oracle.dijkstra(n, src, dst, w, 0)
    assert c.tolist() == [0, I32_INF, 10, 1, 2, 3, 11] and settles == 6
    op = oracle.round_sim(n, src, dst, w, 0, mode=oracle.MODE_ADOPTED, true_cost=c)
    al = oracle.round_sim(n, src, dst, w, 0, mode=oracle.MODE_SCOPE_ALL, true_cost=c)
    for r in (op, al):
        assert np.array_equal(r["cost"], c) and r["violations"] == 0
        assert r["relaxed_edges"] == 5 and r["settled"] == 6
    assert op["rounds"] == 5 and op["fixed_per_round"].tolist() == [1, 1, 2, 1, 0]
    assert al["rounds"] == 4 and al["fixed_per_round"].tolist() == [1, 2, 2, 0]
    assert op["scanned_per_round"].tolist() == [3, 3, 3, 1, 0]
    assert al["scanned_per_round"].tolist() == [6, 5, 2, 0]
    assert op["scanned_in_edges"] == 10 and al["scanned_in_edges"] == 13
    assert op["open_visits"] == 7 and al["open_visits"] == 6


def test_scanned_and_open_visits_closed_forms():
    """Step (C)'s work on shapes where it has a closed form.
    A path 0 -> 1 -> ... -> k: round j (1..k) has O = {j} with in-degree 1,
    so OPEN scans k in-edges with k open visits; ALL also covers the
    undiscovered j+1..k in round j, k - j + 1 vertices of in-degree 1 each,
    so it scans k + (k-1) + ... + 1 = k(k+1)/2.
    A star with L leaves: round 1 has O = all leaves (in-degree 1 each), so
    L scanned and L visits in both scopes (nothing is undiscovered).
    A complete bipartite layer: the source feeds p middle vertices, each
    feeding all q sinks; in round 2 the q sinks have in-degree p each, and a
    sink with a parallel edge counts it twice."""
    for k in (1, 2, 7, 30):
        src = np.arange(k, dtype=np.int32)
        dst = src + 1
        w = np.full(k, 3, np.int32)
        op = oracle.round_sim(k + 1, src, dst, w, 0)
        al = oracle.round_sim(k + 1, src, dst, w, 0, mode=oracle.MODE_SCOPE_ALL)
        assert op["scanned_in_edges"] == k and op["open_visits"] == k
        assert op["scanned_per_round"].tolist() == [1] * k + [0]
        assert al["scanned_in_edges"] == k * (k + 1) // 2 and al["open_visits"] == k
        assert al["scanned_per_round"].tolist() == list(range(k, 0, -1)) + [0]
    for leaves in (1, 5, 100):
        src = np.zeros(leaves, np.int32)
        dst = np.arange(1, leaves + 1, dtype=np.int32)
        w = np.arange(1, leaves + 1, dtype=np.int32)[::-1].copy()
        for mode in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
            r = oracle.round_sim(leaves + 1, src, dst, w, 0, mode=mode)
            assert r["scanned_in_edges"] == leaves and r["open_visits"] == leaves
    p, q = 3, 4
    src = [0] * p + [1 + i for i in range(p) for _ in range(q)] + [1]
    dst = [1 + i for i in range(p)] + [1 + p + j for _ in range(p) for j in range(q)] + [1 + p]
    src, dst = np.array(src, np.int32), np.array(dst, np.int32)
    w = np.full(len(src), 2, np.int32)
    r = oracle.round_sim(1 + p + q, src, dst, w, 0)
    # round 1: the p middles (in-degree 1); round 2: the q sinks (p each, one
    # with an extra parallel edge)
    assert r["scanned_per_round"].tolist() == [p, p * q + 1, 0]
    assert r["open_visits"] == p + q


def test_label_correcting_ending():
    """The loop test follows each run of step (A), as Fig. 6's test follows
    its relax step, and rounds counts the runs of (A).  Worked by hand on
    0->a (1), 0->y (3), u->y (1), a->0 (1) (vertices 0, a = 1, y = 2, u = 3;
    u is never discovered): round 1 relaxes 0 (D[a] = 1, D[y] = 3), minD 1,
    thr = min(1 + 1, 3 + inf) = 2; a is fixed, y survives (m_y = max(C[u],
    1) + 1 = 2 < 3).  Label-correcting: y joins the relax set (D = 3 <
    minD + delta), so round 2 relaxes a (its edge to the fixed 0 changes
    nothing) and y (no out-edge) at D = 3; y is then fixed (minD 3).  Round
    3's relax set is empty (y was relaxed at its final D) and O is empty:
    that run of (A) is the loop test's, and counts.  Label-setting: round 3
    relaxes y.  Both: 3 rounds, fixed [1, 1, 0], relaxed edges 3."""
    src = np.array([0, 0, 3, 1], np.int32)
    dst = np.array([1, 2, 2, 0], np.int32)
    w = np.array([1, 3, 1, 1], np.int32)
    for scope in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
        for lc in (0, oracle.MODE_LC):
            r = oracle.round_sim(4, src, dst, w, 0, mode=scope | lc)
            assert r["cost"].tolist() == [0, 1, 3, I32_INF]
            assert r["rounds"] == 3 and r["fixed_per_round"].tolist() == [1, 1, 0], (scope, lc)
            assert r["relaxed_edges"] == 3


def test_fig5_literal_order_counterexample():
    """Fig. 6 run as printed fixes vertex 2 at 5 in round 2 (threshold is
    inf, since vertex 2 has no out-edge) before vertex 1's out-edge is
    relaxed; the adopted order relaxes first and gets the true cost 2."""
    src = np.array([0, 1, 0], np.int32)
    dst = np.array([1, 2, 2], np.int32)
    for w in (np.array([1, 1, 5], np.int32), np.array([1, 1, 5], np.float32)):
        lit = oracle.round_sim(3, src, dst, w, 0, mode=oracle.MODE_LITERAL_FIG5)
        assert lit["cost"].tolist() == [0, 1, 5]
        ok = oracle.round_sim(3, src, dst, w, 0)
        assert ok["cost"].tolist() == [0, 1, 2] == oracle.dijkstra(3, src, dst, w, 0)[0].tolist()


def test_round_closed_forms():
    # path of k+1 vertices: one vertex per round, plus the final empty relax
    for k in (1, 2, 7, 30):
        src = np.arange(k, dtype=np.int32)
        dst = src + 1
        w = np.full(k, 3, np.int32)
        r = oracle.round_sim(k + 1, src, dst, w, 0)
        assert r["rounds"] == k + 1
    # star: all leaves fixed in round 1 (sole in-edge from the fixed centre)
    for leaves in (1, 5, 100):
        src = np.zeros(leaves, np.int32)
        dst = np.arange(1, leaves + 1, dtype=np.int32)
        w = np.arange(1, leaves + 1, dtype=np.int32)[::-1].copy()
        r = oracle.round_sim(leaves + 1, src, dst, w, 0)
        assert r["rounds"] == 2 and r["fixed_per_round"].tolist() == [leaves, 0]
    # unit weights: one BFS layer per round (SP_2 theorem on unweighted graphs)
    for g in (gen.grid_workload(side=9), gen.random_workload(n=300, m=900)):
        w = np.ones(g.m, np.int32)
        hops = oracle.bfs(g.n, g.src, g.dst, g.source)
        r = oracle.round_sim(g.n, g.src, g.dst, w, g.source)
        assert r["rounds"] == hops.max() + 1
        layer = np.bincount(hops[hops > 0], minlength=hops.max() + 1)[1:]
        assert r["fixed_per_round"].tolist() == layer.tolist() + [0]


def test_round_dag_depth_bound():
    """Acyclic graph whose only root is the source (the SP_1 theorem's
    condition): every vertex is fixed once all its in-neighbours are, so
    rounds <= longest hop depth + 1."""
    rng = np.random.default_rng(14)
    for _ in range(100):
        n = int(rng.integers(2, 60))
        src, dst = [], []
        for v in range(1, n):
            for u in rng.choice(v, size=int(rng.integers(1, min(v, 4) + 1)), replace=False):
                src.append(u)
                dst.append(v)
        src, dst = np.array(src, np.int32), np.array(dst, np.int32)
        w = rng.integers(1, 100, len(src)).astype(np.int32)
        depth = np.zeros(n, np.int64)
        for v in range(1, n):
            depth[v] = 1 + depth[src[dst == v]].max()
        r = oracle.round_sim(n, src, dst, w, 0)
        assert np.array_equal(r["cost"], oracle.dag(n, src, dst, w, 0))
        assert r["rounds"] <= depth.max() + 1


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_round_sim_costs_and_invariants(dtype):
    rng = np.random.default_rng(15)
    for _ in range(400):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 30)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        for mode in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
            r = oracle.round_sim(n, src, dst, w, s, mode=mode, true_cost=c)
            assert np.array_equal(r["cost"], c)
            assert r["violations"] == 0
            assert 1 <= r["rounds"] <= settles
            assert sum(r["fixed_per_round"]) == settles - 1


@pytest.mark.parametrize("family", ["random", "grid", "rmat", "batch"])
def test_round_sim_matches_dijkstra_on_workload_families(family):
    if family == "random":
        g = gen.random_workload()
    elif family == "grid":
        g = gen.grid_workload(side=40)
    elif family == "rmat":
        g = gen.rmat_workload(scale=12)
    else:
        g = gen.batch_workload(count=2, nmin=500, nmax=3000)[1]
    c, settles = oracle.dijkstra(g.n, g.src, g.dst, g.w, g.source)
    r = oracle.round_sim(g.n, g.src, g.dst, g.w, g.source, true_cost=c)
    assert np.array_equal(r["cost"], c)
    assert r["violations"] == 0
    assert r["rounds"] <= settles
    assert r["relaxed_edges"] == int(np.sum(c[g.src] != _inf(g.w.dtype)))


def test_csr_matches_numpy_stable_sort():
    g = gen.rmat_workload(scale=10)
    G = oracle.csr(g.n, g.src, g.dst)
    perm = np.argsort(g.src, kind="stable")
    assert np.array_equal(G.perm, perm)
    assert np.array_equal(G.out_dst, g.dst[perm])
    assert np.array_equal(G.out_off, np.concatenate([[0], np.cumsum(np.bincount(g.src, minlength=g.n))]))
    eids = np.argsort(g.dst[perm], kind="stable")
    assert np.array_equal(G.in_eid, eids)
    assert np.array_equal(G.in_src, g.src[perm][eids])
    ow, iw, wmin = G.weights(g.w)
    assert np.array_equal(ow, g.w[perm]) and np.array_equal(iw, ow[eids])
    ref = np.full(g.n, I32_INF, np.int32)
    np.minimum.at(ref, g.src, g.w)
    assert np.array_equal(wmin, ref)


def brute_pred(n, src, dst, w, s, cost, perm):
    """Tie rule by enumeration: eid = stable CSR position (inverse of perm)."""
    eid_of = np.empty(len(src), np.int64)
    eid_of[perm] = np.arange(len(src))
    inf = _inf(w.dtype)
    dt = w.dtype.type

    def add(a, b):
        if np.dtype(dt) == np.int32:
            return inf if (a == inf or b == inf) else dt(int(a) + int(b))
        return dt(a + b)

    tight = [[] for _ in range(n)]
    for i in range(len(src)):
        u, y = int(src[i]), int(dst[i])
        if cost[u] != inf and cost[y] != inf and add(cost[u], w[i]) == cost[y]:
            tight[y].append((int(eid_of[i]), u))
    pred = np.full(n, -1, np.int64)
    level = {s: 0}
    for y in range(n):
        if y == s or cost[y] == inf:
            continue
        strict = [e for (e, u) in tight[y] if cost[u] < cost[y]]
        if strict:
            pred[y] = min(strict)
            level[y] = 0
    frontier = [v for v in level]
    lv = 0
    while frontier:
        nxt = []
        for y in range(n):
            if y in level or y == s or cost[y] == inf:
                continue
            if any(u in level and level[u] == lv and cost[u] == cost[y] for (_, u) in tight[y]):
                nxt.append(y)
        for y in nxt:
            level[y] = lv + 1
        frontier = nxt
        lv += 1
    for y in range(n):
        if y == s or cost[y] == inf or pred[y] >= 0:
            continue
        pred[y] = min(e for (e, u) in tight[y] if level.get(u) == level[y] - 1 and cost[u] == cost[y])
    return pred


def check_tree(n, s, cost, pred, out_src_of_eid, inf):
    for y in range(n):
        if y == s or cost[y] == inf:
            assert pred[y] == -1
            continue
        assert pred[y] >= 0
        seen = set()
        v = y
        while v != s:
            assert v not in seen
            seen.add(v)
            v = out_src_of_eid[pred[v]]


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_pred_tie_rule_brute_force(dtype):
    rng = np.random.default_rng(16)
    for _ in range(400):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 12)))
        if dtype == np.int32:
            w = rng.integers(1, 4, len(src)).astype(np.int32)  # many ties
        c, _ = oracle.dijkstra(n, src, dst, w, s)
        g = oracle.csr(n, src, dst)
        p, _ = oracle.pred(g, w, s, c)
        assert np.array_equal(p, brute_pred(n, src, dst, w, s, c, g.perm))
        check_tree(n, s, c, p, src[g.perm], _inf(dtype))


def test_pred_equal_cost_float_ties():
    """Edges of weight 2^-30 on cost-1.0 vertices are tight at equal cost
    (1 + 2^-30 rounds to 1 in float32); the level rule keeps a tree."""
    tiny = np.float32(2.0 ** -30)
    # s=0 -> a=1 (1.0); a->b, b->c, c->b, c->a, b->a all tiny; ids chosen so
    # that the smallest tight id into b comes from c (a cycle if taken).
    src = np.array([2, 0, 1, 1, 2, 3], np.int32)
    dst = np.array([1, 1, 2, 1, 3, 2], np.int32)
    w = np.array([tiny, 1.0, tiny, tiny, tiny, tiny], np.float32)
    n, s = 4, 0
    c, _ = oracle.dijkstra(n, src, dst, w, s)
    assert c.tolist() == [0.0, 1.0, 1.0, 1.0]
    g = oracle.csr(n, src, dst)
    p, ties = oracle.pred(g, w, s, c)
    assert ties == 2
    assert np.array_equal(p, brute_pred(n, src, dst, w, s, c, g.perm))
    check_tree(n, s, c, p, src[g.perm], np.float32(np.inf))
    tails = src[g.perm][p[1:]]
    assert tails.tolist() == [0, 1, 2]


def test_gradient_matches_path_sums_and_fd():
    rng = np.random.default_rng(17)
    for trial in range(20):
        n = int(rng.integers(3, 25))
        m = int(rng.integers(n, 5 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        w = rng.random(m) + 0.1
        S = 3
        sources = rng.choice(n, S, replace=False).astype(np.int32)
        gco = rng.standard_normal((S, n))
        G = oracle.csr(n, src, dst)
        preds, costs = [], []
        for s in sources:
            c, _ = oracle.dijkstra(n, src, dst, w, int(s))
            p, ties = oracle.pred(G, w, int(s), c)
            assert ties == 0
            preds.append(p)
            costs.append(c)
        grad = oracle.grad(G, sources, np.array(preds), gco)
        # brute force: each reachable x adds g[s,x] to every edge on its tree path
        tail_of = src[G.perm]
        ref = np.zeros(m)
        for si, s in enumerate(sources):
            for x in range(n):
                if x == s or not np.isfinite(costs[si][x]):
                    continue
                v = x
                while v != s:
                    e = preds[si][v]
                    ref[e] += gco[si, x]
                    v = tail_of[e]
        np.testing.assert_allclose(grad, ref, rtol=1e-12, atol=1e-12)
        # central finite differences in fp64 (paths unique a.s. for random w)
        wcsr = w[G.perm]

        def loss(wc):
            wcoo = np.empty(m)
            wcoo[G.perm] = wc
            tot = 0.0
            for si, s in enumerate(sources):
                c, _ = oracle.dijkstra(n, src, dst, wcoo, int(s))
                fin = np.isfinite(c)
                tot += float(np.sum(gco[si][fin] * c[fin]))
            return tot

        h = 1e-7
        for e in rng.choice(m, min(m, 8), replace=False):
            d = np.zeros(m)
            d[e] = h
            fd = (loss(wcsr + d) - loss(wcsr - d)) / (2 * h)
            assert abs(fd - grad[e]) <= 1e-5 * max(1.0, abs(grad[e]))


def test_generators_deterministic_and_in_range():
    a = gen.random_workload()
    b = gen.random_workload()
    assert np.array_equal(a.src, b.src) and np.array_equal(a.w, b.w)
    assert a.m == 32768 and a.n == 4096 and a.source == 0
    assert not np.any(a.src == a.dst)
    assert a.w.min() >= 1 and a.w.max() <= 100
    gr = gen.grid_workload(side=16)
    assert gr.m == 2 * 2 * 16 * 15 and gr.source == 8 * 16 + 8
    assert gr.w.min() >= 1 and gr.w.max() <= 1000
    r = gen.rmat_workload(scale=10)
    assert r.m == 16 * 1024
    deg = np.bincount(r.src, minlength=r.n)
    assert deg[r.source] == deg.max() and r.source == int(np.argmax(deg))
    assert r.w.min() >= 1 and r.w.max() <= 255
    bl = gen.batch_workload(count=3, nmin=1000, nmax=2000)
    for g in bl:
        assert 1000 <= g.n <= 2000 and g.m == 8 * g.n and 0 <= g.source < g.n
        assert g.w.min() > 0 and g.w.max() <= 1.0
        assert np.all((g.w * np.float32(2 ** 24)) == np.round(g.w * np.float32(2 ** 24)))
    d, gco = gen.diff_workload(side=16, num_sources=5)
    assert len(set(d.sources.tolist())) == 5 and gco.shape == (5, 256)
    assert d.w.min() >= 0.5 and d.w.max() <= 1.5
    assert abs(float(gen.normal_f32(1, 100000).std()) - 1.0) < 0.02


def test_target_closed_forms():
    """Single-destination stop (Section I).  On a path 0 -> 1 -> ... -> k,
    vertex j is fixed in round j, so the rounds stop after j of them with
    0..j exact and j + 1 still undiscovered; the source as target stops
    before round 1.  Dijkstra removes 0..j from its heap."""
    k = 12
    src = np.arange(k, dtype=np.int32)
    dst = src + 1
    w = np.full(k, 5, np.int32)
    for j in range(k + 1):
        r = oracle.round_sim(k + 1, src, dst, w, 0, target=j)
        assert r["rounds"] == j and r["settled"] == j + 1 and r["relaxed_edges"] == j
        assert r["cost"][: j + 1].tolist() == [5 * i for i in range(j + 1)]
        assert all(x == I32_INF for x in r["cost"][j + 1:])
        c, pops = oracle.dijkstra(k + 1, src, dst, w, 0, target=j)
        assert pops == j + 1 and c[j] == 5 * j
    # star: every leaf is fixed in round 1
    src = np.zeros(9, np.int32)
    dst = np.arange(1, 10, dtype=np.int32)
    r = oracle.round_sim(10, src, dst, np.arange(9, 0, -1).astype(np.int32), 0, target=4)
    assert r["rounds"] == 1 and r["settled"] == 10


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_target_stop_against_full_solve(dtype):
    """The stopped rounds are a prefix of the full ones; the target's cost is
    exact and every other entry is an upper bound; an unreachable target
    runs the whole solve."""
    rng = np.random.default_rng(16)
    inf = _inf(dtype)
    for _ in range(300):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 30)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        full = oracle.round_sim(n, src, dst, w, s)
        t = int(rng.integers(0, n))
        r = oracle.round_sim(n, src, dst, w, s, target=t)
        ct, pops = oracle.dijkstra(n, src, dst, w, s, target=t)
        assert r["cost"][t] == c[t] and ct[t] == c[t]
        assert np.all(r["cost"] >= c)
        assert pops <= settles
        if c[t] == inf:
            assert r["rounds"] == full["rounds"] and np.array_equal(r["cost"], full["cost"])
            assert r["settled"] == full["settled"] == settles
            continue
        assert (r["rounds"] == 0) == (t == s)
        assert r["rounds"] <= full["rounds"]
        assert r["fixed_per_round"].tolist() == full["fixed_per_round"][: r["rounds"]].tolist()
        assert r["settled"] == 1 + sum(r["fixed_per_round"])
        assert np.count_nonzero((r["cost"] == c) & (c != inf)) >= r["settled"]
        assert r["relaxed_edges"] <= full["relaxed_edges"]


def test_label_correcting_closed_forms():
    """Label-correcting relax (Fig. 6's step 3 explores every discovered
    vertex).  Worked by hand on 0->1 (10), 0->2 (1), 2->1 (1), 1->3 (1): round
    1 relaxes 0 and fixes 2; round 2 relaxes 2 and, from its tentative D = 10,
    also 1, so D[1] = 2 and D[3] = 11, and 1 is fixed; round 3 relaxes 1 again
    (D fell to 2) and fixes 3; round 4 finds nothing open.  Label-setting
    relaxes each of the four edges once in the same four rounds."""
    src = np.array([0, 0, 2, 1], np.int32)
    dst = np.array([1, 2, 1, 3], np.int32)
    w = np.array([10, 1, 1, 1], np.int32)
    for scope in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
        ls = oracle.round_sim(4, src, dst, w, 0, mode=scope)
        lc = oracle.round_sim(4, src, dst, w, 0, mode=scope | oracle.MODE_LC)
        assert ls["cost"].tolist() == lc["cost"].tolist() == [0, 2, 1, 3]
        assert ls["rounds"] == lc["rounds"] == 4
        assert ls["fixed_per_round"].tolist() == lc["fixed_per_round"].tolist() == [1, 1, 1, 0]
        assert ls["relaxed_edges"] == 4 and lc["relaxed_edges"] == 5
    # a path: every D is final when discovered, so nothing is relaxed twice
    for k in (1, 7, 30):
        src = np.arange(k, dtype=np.int32)
        r = oracle.round_sim(k + 1, src, src + 1, np.full(k, 3, np.int32), 0,
                             mode=oracle.MODE_LC)
        assert r["rounds"] == k + 1 and r["relaxed_edges"] == k


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_label_correcting_costs_and_invariants(dtype):
    rng = np.random.default_rng(17)
    for _ in range(300):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 30)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        for mode in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
            ls = oracle.round_sim(n, src, dst, w, s, mode=mode)
            r = oracle.round_sim(n, src, dst, w, s, mode=mode | oracle.MODE_LC, true_cost=c)
            assert np.array_equal(r["cost"], c)
            assert r["violations"] == 0
            assert 1 <= r["rounds"] <= settles
            assert r["settled"] == settles
            assert r["relaxed_edges"] >= ls["relaxed_edges"]


def test_delta_bucket_closed_forms():
    """Delta-stepping with the method (Section I): an open vertex joins the
    relax set only while D < minD + delta.  On the hand-worked graph above,
    vertex 1 survives round 1 with D = 10 while minD = 1, so it is relaxed
    early (five relaxed edges) iff 10 < 1 + delta, i.e. delta > 9; costs and
    rounds do not change."""
    src = np.array([0, 0, 2, 1], np.int32)
    dst = np.array([1, 2, 1, 3], np.int32)
    w = np.array([10, 1, 1, 1], np.int32)
    for delta, relaxed in ((0, 4), (5, 4), (9, 4), (10, 5), (100, 5), (None, 5),
                           (2**31 - 2, 5)):
        r = oracle.round_sim(4, src, dst, w, 0, mode=oracle.MODE_LC, delta=delta)
        assert r["cost"].tolist() == [0, 2, 1, 3], delta
        assert r["rounds"] == 4 and r["relaxed_edges"] == relaxed, (delta, r)
    # float32: the same boundary at delta = 9 (10 < 1 + delta)
    wf = w.astype(np.float32)
    for delta, relaxed in ((9.0, 4), (9.5, 5), (float("inf"), 5)):
        r = oracle.round_sim(4, src, dst, wf, 0, mode=oracle.MODE_LC, delta=delta)
        assert r["relaxed_edges"] == relaxed, (delta, r)


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_delta_bucket_limits_and_costs(dtype):
    """delta = 0 is label-setting and an unbounded delta (INF, or an int32
    delta whose sum with minD saturates) is full label-correcting, counter
    for counter; every delta reaches Dijkstra's costs with the per-round
    invariants intact."""
    rng = np.random.default_rng(19)
    big = 2**31 - 2 if dtype == np.int32 else np.float32(3e38)
    for _ in range(200):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 30)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        for mode in (oracle.MODE_ADOPTED, oracle.MODE_SCOPE_ALL):
            ls = oracle.round_sim(n, src, dst, w, s, mode=mode)
            lc = oracle.round_sim(n, src, dst, w, s, mode=mode | oracle.MODE_LC)
            z = oracle.round_sim(n, src, dst, w, s, mode=mode | oracle.MODE_LC, delta=0)
            for k in ("rounds", "relaxed_edges", "scanned_in_edges", "settled"):
                assert z[k] == ls[k], (k, z, ls)
            if dtype == np.int32:
                b = oracle.round_sim(n, src, dst, w, s, mode=mode | oracle.MODE_LC, delta=big)
                for k in ("rounds", "relaxed_edges", "scanned_in_edges", "settled"):
                    assert b[k] == lc[k], (k, b, lc)
            for delta in (1, 3, 10) if dtype == np.int32 else (0.05, 0.2, 1.0):
                r = oracle.round_sim(n, src, dst, w, s, mode=mode | oracle.MODE_LC, delta=delta,
                                     true_cost=c)
                assert np.array_equal(r["cost"], c)
                assert r["violations"] == 0
                assert 1 <= r["rounds"] <= settles and r["settled"] == settles
                assert r["relaxed_edges"] >= ls["relaxed_edges"]


def _heap_ops(o):
    return o["remove_min"] + o["insert"] + o["adjust"]


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_sp12_costs(dtype):
    """SP_1 and SP_2 (Figs. 3 and 4) reach Dijkstra's costs; variant 0 is
    Dijkstra in the same framework and removes each reachable vertex once."""
    rng = np.random.default_rng(18)
    for _ in range(400):
        n, src, dst, w, s = tiny_graph(rng, dtype, n=int(rng.integers(1, 30)))
        c, settles = oracle.dijkstra(n, src, dst, w, s)
        c0, o0 = oracle.sp12(n, src, dst, w, s, 0)
        assert np.array_equal(c0, c) and o0["remove_min"] == settles == o0["insert"]
        assert o0["fixed_by_r"] == 0
        for v in (1, 2):
            cv, ov = oracle.sp12(n, src, dst, w, s, v)
            assert np.array_equal(cv, c)
            # every reachable vertex is fixed once: by removeMin or through R
            assert ov["fixed_by_r"] <= settles - 1


def test_sp12_dag_theorem():
    """On a DAG whose only vertex without in-edges is the source, SP_1 and
    SP_2 fix every vertex through R: one insertion and one removeMin (the
    source), no adjustments (the O(e) case of the SP_1 theorem)."""
    rng = np.random.default_rng(19)
    for _ in range(100):
        n = int(rng.integers(2, 80))
        src, dst = [], []
        for v in range(1, n):
            for u in rng.choice(v, size=int(rng.integers(1, min(v, 4) + 1)), replace=False):
                src.append(u)
                dst.append(v)
        src, dst = np.array(src, np.int32), np.array(dst, np.int32)
        w = rng.integers(1, 100, len(src)).astype(np.int32)
        c = oracle.dag(n, src, dst, w, 0)
        for v in (1, 2):
            cv, ov = oracle.sp12(n, src, dst, w, 0, v)
            assert np.array_equal(cv, c)
            assert ov == dict(remove_min=1, insert=1, adjust=0, fixed_by_r=n - 1)


def test_sp12_heap_operations_on_workloads():
    """SP_2 needs no more heap operations than Dijkstra on every workload
    family (Section I's claim; SP_1 can need one more adjustment on a few
    graphs, see the readings), and fixes part of each graph through R."""
    for g in (gen.grid_workload(side=64), gen.rmat_workload(scale=14), gen.random_workload(),
              gen.batch_workload(count=2, nmin=1000, nmax=5000)[1]):
        c, _ = oracle.dijkstra(g.n, g.src, g.dst, g.w, g.source)
        _, o0 = oracle.sp12(g.n, g.src, g.dst, g.w, g.source, 0)
        _, o2 = oracle.sp12(g.n, g.src, g.dst, g.w, g.source, 2)
        assert _heap_ops(o2) <= _heap_ops(o0)
        assert o2["fixed_by_r"] > 0
