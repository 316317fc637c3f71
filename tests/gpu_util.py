"""Helpers shared by the GPU tests: build a graph on the device, run the
oracle on the same seeded arrays, and compare."""
import numpy as np
import torch

import oracle


def to_np(t):
    return t.detach().cpu().numpy()


def oracle_solution(n, src, dst, w, source):
    """(cost, pred (int64), settles, rounds, fixed_per_round, stats) from the oracle."""
    cost, settles = oracle.dijkstra(n, src, dst, w, source)
    O = oracle.csr(n, src, dst)
    pred, _ = oracle.pred(O, w, source, cost)
    sim = oracle.round_sim(n, src, dst, w, source)
    assert np.array_equal(sim["cost"], cost)
    return dict(cost=cost, pred=pred, settles=settles, rounds=sim["rounds"],
                relaxed=sim["relaxed_edges"], scanned=sim["scanned_in_edges"], csr=O)


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


def sync():
    torch.cuda.synchronize()
