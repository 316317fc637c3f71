"""Helpers shared by the GPU tests: build a graph on the device, run the
oracle on the same seeded arrays, and compare."""
import numpy as np
import torch

import oracle


def to_np(t):
    return t.detach().cpu().numpy()


def oracle_mode(scope, relax="setting"):
    """The round simulator's mode for a solve's C scope ("open" or "all") and
    relax step ("setting" or "correcting")."""
    mode = oracle.MODE_SCOPE_ALL if scope == "all" else oracle.MODE_ADOPTED
    return mode | (oracle.MODE_LC if relax == "correcting" else 0)


def oracle_solution(n, src, dst, w, source, scope="open", relax="setting", delta=None):
    """cost, pred (int64), ties (vertices that took the equal-cost level
    rule), settles, and the round counters under the given C scope, relax
    step and label-correcting bucket width, from the oracle."""
    cost, settles = oracle.dijkstra(n, src, dst, w, source)
    O = oracle.csr(n, src, dst)
    pred, ties = oracle.pred(O, w, source, cost)
    sim = oracle.round_sim(n, src, dst, w, source, mode=oracle_mode(scope, relax), delta=delta)
    assert np.array_equal(sim["cost"], cost)
    return dict(cost=cost, pred=pred, ties=ties, settles=settles, rounds=sim["rounds"],
                relaxed=sim["relaxed_edges"], scanned=sim["scanned_in_edges"],
                open_visits=sim["open_visits"], csr=O)


def assert_same_solution(cost, pred, stats, ref, label=""):
    c = to_np(cost)
    assert c.dtype == ref["cost"].dtype
    bad = np.nonzero(c != ref["cost"])[0]
    assert bad.size == 0, "%s cost mismatch at %d vertices, first %s: gpu %s oracle %s" % (
        label, bad.size, bad[:5], c[bad[:5]], ref["cost"][bad[:5]])
    if pred is not None:
        p = to_np(pred).astype(np.int64)
        bad = np.nonzero(p != ref["pred"])[0]
        assert bad.size == 0, "%s pred mismatch at %d vertices, first %s: gpu %s oracle %s" % (
            label, bad.size, bad[:5], p[bad[:5]], ref["pred"][bad[:5]])
    if stats is not None:
        assert stats["rounds"] == ref["rounds"], (label, stats, ref["rounds"])
        assert stats["settled"] == ref["settles"], (label, stats, ref["settles"])
        assert stats["relaxed_edges"] == ref["relaxed"], (label, stats, ref["relaxed"])
        assert stats["scanned_in_edges"] == ref["scanned"], (label, stats, ref["scanned"])
        assert stats["open_visits"] == ref["open_visits"], (label, stats, ref["open_visits"])


def sync():
    torch.cuda.synchronize()


def expected_order(n, src, dst):
    """The builder's automatic choice: degree order iff the largest total
    degree is at least 16 times the mean total degree 2m/n."""
    m = len(src)
    if m == 0:
        return "input"
    deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
    return "degree" if int(deg.max()) * n >= 32 * m else "input"


def check_solver_copy(G, n, src, dst, w):
    """The working copy, rebuilt from its definition.  Degree order: vertices
    by descending total degree (ties by id), out-lists by (tail, head) solver
    id then edge id.  Both orders: in-lists by (head solver id, weight, tail
    solver id, edge id)."""
    O = oracle.csr(n, src, dst)
    ow, _, wmin = O.weights(w)
    S = {k: to_np(v) for k, v in G.solver_arrays().items()}
    if G.order == "degree":
        deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
        vid = np.argsort(-deg, kind="stable")
    else:
        vid = np.arange(n)
    rank = np.empty(n, np.int64)
    rank[vid] = np.arange(n)
    m = len(src)
    eid = np.arange(m)
    tail = np.repeat(np.arange(n), np.diff(O.out_off))
    head = O.out_dst.astype(np.int64)
    bits = lambda a: a.view(np.int32) if a.dtype == np.float32 else a
    wkey = bits(np.ascontiguousarray(ow)).astype(np.int64)  # positive: bits order like values
    sides = {"in": np.lexsort((eid, rank[tail], wkey, rank[head]))}
    if G.order == "degree":
        assert np.array_equal(S["vid"], vid) and np.array_equal(S["rank"], rank)
        sides["out"] = np.lexsort((eid, rank[head], rank[tail]))
        assert np.array_equal(bits(S["out_wmin"]), bits(wmin[vid]))
    # vertex records: out offset and degree, in offset and degree, out_wmin
    so = S["out_off"] if G.order == "degree" else O.out_off
    vr = S["vrec"]
    wmin_s = wmin[vid]
    assert np.array_equal(vr[:, 0], so[:-1]) and np.array_equal(vr[:, 1], np.diff(so))
    in_off_s = np.concatenate([[0], np.cumsum(np.bincount(rank[head], minlength=n))])
    assert np.array_equal(vr[:, 2], in_off_s[:-1]) and np.array_equal(vr[:, 3], np.diff(in_off_s))
    assert np.array_equal(vr[:, 4], bits(np.ascontiguousarray(wmin_s)))
    assert not vr[:, 7].any()
    # the in-side half: in_off, in_degree, the lightest in-edge's tail and weight
    vin = S["vin"]
    assert np.array_equal(vin[:, 0:2], vr[:, 2:4]) and np.array_equal(vin[:, 2:4], vr[:, 5:7])
    for side, order in sides.items():
        key = rank[tail] if side == "out" else rank[head]
        nbr = rank[head] if side == "out" else rank[tail]
        off = np.concatenate([[0], np.cumsum(np.bincount(key, minlength=n))])
        assert np.array_equal(S[side + "_off"], off), side
        assert np.array_equal(S[side + "_eid"], order), side
        nb = S["out_dst"] if side == "out" else S["in_src"]
        assert np.array_equal(nb, nbr[order]), side
        assert np.array_equal(bits(S[side + "_w"]), bits(ow[order])), side
        if side == "in":
            # the record's copy of each in-list's first (lightest) entry
            has = np.diff(off) > 0
            first = off[:-1][has]
            assert np.array_equal(vr[has, 5], nbr[order][first])
            assert np.array_equal(vr[has, 6], bits(np.ascontiguousarray(ow[order]))[first])
            assert not vr[~has, 5:7].any()
            # the same in-lists as (tail, weight) pairs
            assert np.array_equal(S["in_sw"][:, 0], nbr[order])
            assert np.array_equal(S["in_sw"][:, 1], bits(np.ascontiguousarray(ow[order])))
    # out-edge records of the working copy's out-lists (in input order the CSR
    # itself): head solver id, weight, edge id, the head's out_wmin
    oo = sides.get("out", eid)
    rec = S["out_rec"]
    assert np.array_equal(rec[:, 0], rank[head][oo])
    assert np.array_equal(rec[:, 1], bits(np.ascontiguousarray(ow[oo])))
    assert np.array_equal(rec[:, 2], oo)
    assert np.array_equal(rec[:, 3], bits(np.ascontiguousarray(wmin[head[oo]])))


def pool_map(fn, items):
    """fn over items on a thread pool of up to 16 host threads (the oracle's
    C calls release the GIL), results in order."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1, len(items)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))
