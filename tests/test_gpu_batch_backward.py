"""GPU parity of the batched solve and of the backward pass.

Batch: one persistent launch over many instances (several graphs, several
sources per graph) must give, instance by instance, the same cost, pred and
stats as single solves and as the oracle.  Backward: the weight gradient of
L = sum g * cost must match the oracle's fp64 subtree sums (relative-norm
error <= 1e-5) and fp64 finite differences on sampled edges.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import oracle_solution, sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def check_batch(sp, graphs, glist, inst_graph, inst_source, label):
    print("batch", label, "instances", len(inst_graph), flush=True)
    cost, pred, stats = sp.solve_batch(graphs, inst_graph, inst_source, with_pred=True,
                                       with_stats=True)
    sync()
    bases, total = sp.batch_layout(graphs, inst_graph)
    assert cost.numel() == total
    c, p = to_np(cost), to_np(pred).astype(np.int64)
    for i, (gi, s) in enumerate(zip(inst_graph, inst_source)):
        g = glist[gi]
        # each instance runs its graph's C scope and relax step
        ref = oracle_solution(g.n, g.src, g.dst, g.w, s, graphs[gi].effective_scope,
                              graphs[gi].effective_relax, graphs[gi].effective_delta)
        sl = slice(bases[i], bases[i] + g.n)
        assert np.array_equal(c[sl], ref["cost"]), (label, i)
        assert np.array_equal(p[sl], ref["pred"]), (label, i)
        st = stats[i]
        assert st["rounds"] == ref["rounds"], (label, i, st, ref["rounds"])
        assert st["settled"] == ref["settles"], (label, i)
        assert st["relaxed_edges"] == ref["relaxed"], (label, i)
        assert st["scanned_in_edges"] == ref["scanned"], (label, i)
        assert st["open_visits"] == ref["open_visits"], (label, i)
        # identical to the single solve of the same instance
        c1, p1, st1 = sp.solve(graphs[gi], s, with_pred=True, with_stats=True)
        sync()
        assert np.array_equal(to_np(c1), c[sl]) and np.array_equal(to_np(p1), to_np(pred)[sl])
        assert st1["rounds"] == st["rounds"] and st1["open_visits"] == st["open_visits"]
        assert st1["scanned_in_edges"] == st["scanned_in_edges"]
    return cost, pred


def test_batch_mixed_small(sp):
    rng = np.random.default_rng(31)
    glist = []
    for k in range(5):
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 8 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        w = (rng.integers(1, 2**24, m) * 2.0 ** -24).astype(np.float32)
        glist.append(gen.Graph("g%d" % k, n, src, dst, w, 0))
    # one batch mixes graphs in both numberings
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w, order=("degree" if k % 2 else "input"))
              for k, g in enumerate(glist)]
    inst_graph = [0, 1, 2, 3, 4, 2, 2, 0]
    inst_source = [int(rng.integers(0, glist[g].n)) for g in inst_graph]
    check_batch(sp, graphs, glist, inst_graph, inst_source, "mixed-small")


def test_batch_label_correcting(sp):
    # per-graph relax steps in one launch: label-correcting and label-setting
    glist = gen.batch_workload(count=6, nmin=1000, nmax=20000)
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w, relax=("correcting" if k % 3 else "setting"))
              for k, g in enumerate(glist)]
    check_batch(sp, graphs, glist, [0, 1, 2, 3, 4, 5, 1, 2], [g.source for g in glist] +
                [int(glist[1].n // 2), int(glist[2].n // 3)], "batch-lc")
    d, _ = gen.diff_workload(side=48, num_sources=8)
    G = sp.Graph(d.n, d.src, d.dst, d.w, relax="correcting")
    check_batch(sp, [G], [d], [0] * 8, [int(s) for s in d.sources], "grid48x8-lc")


@pytest.mark.parametrize("scope", ["open", "all"])
def test_batch_scopes(sp, scope):
    # every instance in one C scope, mixed numberings, plus a skewed graph
    glist = gen.batch_workload(count=5, nmin=1000, nmax=20000)
    glist.append(gen.rmat_workload(scale=12))
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w.astype(np.float32) if g.w.dtype != np.float32
                       else g.w, order=("degree" if k % 2 else "input"), scope=scope)
              for k, g in enumerate(glist)]
    glist = [gen.Graph(g.name, g.n, g.src, g.dst,
                       g.w.astype(np.float32) if g.w.dtype != np.float32 else g.w, g.source)
             for g in glist]
    check_batch(sp, graphs, glist, [0, 1, 2, 3, 4, 5, 5, 0],
                [g.source for g in glist] + [int(glist[5].n // 3), 7], "batch-" + scope)


def test_batch_workload_shape(sp):
    glist = gen.batch_workload(count=12, nmin=1000, nmax=20000)
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w) for g in glist]
    check_batch(sp, graphs, glist, list(range(12)), [g.source for g in glist], "batch12")


def test_batch_same_graph_many_sources(sp):
    d, _ = gen.diff_workload(side=48, num_sources=16)
    G = sp.Graph(d.n, d.src, d.dst, d.w)
    srcs = [int(s) for s in d.sources]
    check_batch(sp, [G], [d], [0] * len(srcs), srcs, "grid48x16")


def test_batch_int32(sp):
    glist = [gen.random_workload(n=3000, m=20000), gen.rmat_workload(scale=11),
             gen.grid_workload(side=40)]
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w) for g in glist]
    check_batch(sp, graphs, glist, [0, 1, 2, 1], [0, glist[1].source, glist[2].source, 5],
                "i32-mix")


def test_batch_more_instances_than_lds_slots(sp):
    # 2100 instances: more than the per-block LDS slots (2048), so the
    # per-instance minima go straight to device atomics
    rng = np.random.default_rng(41)
    glist = []
    for k in range(3):
        n = int(rng.integers(20, 60))
        m = 4 * n
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        w = rng.integers(1, 30, m).astype(np.int32)
        glist.append(gen.Graph("s%d" % k, n, src, dst, w, 0))
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w) for g in glist]
    inst_graph = [int(x) for x in rng.integers(0, 3, 2100)]
    inst_source = [int(rng.integers(0, glist[g].n)) for g in inst_graph]
    cost, pred, stats = sp.solve_batch(graphs, inst_graph, inst_source, with_pred=True,
                                       with_stats=True)
    sync()
    bases, _ = sp.batch_layout(graphs, inst_graph)
    c, p = to_np(cost), to_np(pred).astype(np.int64)
    refs = {}
    for i, (gi, s) in enumerate(zip(inst_graph, inst_source)):
        if (gi, s) not in refs:
            g = glist[gi]
            refs[(gi, s)] = oracle_solution(g.n, g.src, g.dst, g.w, s,
                                            graphs[gi].effective_scope,
                                            graphs[gi].effective_relax, graphs[gi].effective_delta)
        ref = refs[(gi, s)]
        sl = slice(bases[i], bases[i] + glist[gi].n)
        assert np.array_equal(c[sl], ref["cost"]), i
        assert np.array_equal(p[sl], ref["pred"]), i
        assert stats[i]["rounds"] == ref["rounds"], i
        assert stats[i]["scanned_in_edges"] == ref["scanned"], i
        assert stats[i]["open_visits"] == ref["open_visits"], i


def grad_reference(glist, graphs_np_csr, inst_graph, inst_source, preds, gco, bases):
    out = []
    for gi, g in enumerate(glist):
        O = graphs_np_csr[gi]
        ins = [i for i, x in enumerate(inst_graph) if x == gi]
        if not ins:
            out.append(np.zeros(g.m))
            continue
        P = np.stack([preds[bases[i]:bases[i] + g.n] for i in ins]).astype(np.int64)
        Gc = np.stack([gco[bases[i]:bases[i] + g.n] for i in ins]).astype(np.float64)
        reach = np.stack([True for _ in ins])
        del reach
        out.append(oracle.grad(O, [inst_source[i] for i in ins], P, Gc))
    return np.concatenate(out)


@pytest.mark.parametrize("order", ["auto", "degree"])
def test_backward_matches_oracle_gradient(sp, order):
    d, gco_full = gen.diff_workload(side=64, num_sources=8)
    G = sp.Graph(d.n, d.src, d.dst, d.w, order=order)
    srcs = [int(s) for s in d.sources]
    cost, pred, _ = sp.solve_batch([G], [0] * len(srcs), srcs)
    gcost = torch.from_numpy(gco_full.reshape(-1)).cuda()
    gw = sp.backward([G], [0] * len(srcs), srcs, pred, gcost)
    sync()
    O = oracle.csr(d.n, d.src, d.dst)
    p = to_np(pred).astype(np.int64).reshape(len(srcs), d.n)
    ref = oracle.grad(O, srcs, p, gco_full.astype(np.float64))
    got = to_np(gw).astype(np.float64)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("backward rel-norm err", err, flush=True)
    assert err <= 1e-5
    # deterministic: a second call gives the same bits
    gw2 = sp.backward([G], [0] * len(srcs), srcs, pred, gcost)
    sync()
    assert np.array_equal(to_np(gw2), to_np(gw))


def test_backward_multi_graph(sp):
    glist = gen.batch_workload(count=4, nmin=500, nmax=3000)
    graphs = [sp.Graph(g.n, g.src, g.dst, g.w, order=("degree" if k in (1, 2) else "auto"))
              for k, g in enumerate(glist)]
    inst_graph = [0, 1, 1, 2, 3, 3, 3]
    rng = np.random.default_rng(5)
    inst_source = [int(rng.integers(0, glist[g].n)) for g in inst_graph]
    cost, pred, _ = sp.solve_batch(graphs, inst_graph, inst_source)
    bases, total = sp.batch_layout(graphs, inst_graph)
    gco = gen.normal_f32(9, total)
    gw = sp.backward(graphs, inst_graph, inst_source, pred, torch.from_numpy(gco).cuda())
    sync()
    csrs = [oracle.csr(g.n, g.src, g.dst) for g in glist]
    ref = grad_reference(glist, csrs, inst_graph, inst_source, to_np(pred), gco, bases)
    got = to_np(gw).astype(np.float64)
    err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
    assert err <= 1e-5, err


def test_backward_finite_differences_fp64(sp):
    """Central differences of the fp64 oracle at h=1e-3 on sampled edges whose
    pred trees at w-h, w, w+h agree (no near-ties), against the GPU gradient."""
    d, gco = gen.diff_workload(side=24, num_sources=3)
    G = sp.Graph(d.n, d.src, d.dst, d.w)
    srcs = [int(s) for s in d.sources]
    cost, pred, _ = sp.solve_batch([G], [0] * 3, srcs)
    gw = to_np(sp.backward([G], [0] * 3, srcs, pred,
                           torch.from_numpy(gco.reshape(-1)).cuda())).astype(np.float64)
    O = oracle.csr(d.n, d.src, d.dst)
    w64 = d.w.astype(np.float64)

    def solve64(wc):
        costs, preds = [], []
        for s in srcs:
            c, _ = oracle.dijkstra(d.n, d.src, d.dst, wc, s)
            p, _ = oracle.pred(O, wc, s, c)
            costs.append(c)
            preds.append(p)
        return costs, preds

    def loss(costs):
        return sum(float(np.sum(gco[i].astype(np.float64) * c)) for i, c in enumerate(costs))

    base_c, base_p = solve64(w64)
    p32 = to_np(pred).astype(np.int64).reshape(3, d.n)
    rng = np.random.default_rng(3)
    h, checked = 1e-3, 0
    for e in rng.choice(d.m, 48, replace=False):
        coo = int(O.perm[e])
        wp, wm = w64.copy(), w64.copy()
        wp[coo] += h
        wm[coo] -= h
        cp, pp = solve64(wp)
        cm, pm = solve64(wm)
        if not all(np.array_equal(a, b) and np.array_equal(a, c)
                   for a, b, c in zip(base_p, pp, pm)):
            continue
        if not all(np.array_equal(base_p[i], p32[i]) for i in range(3)):
            continue
        fd = (loss(cp) - loss(cm)) / (2 * h)
        assert abs(fd - gw[e]) <= 1e-3 * max(1.0, abs(fd)), (e, fd, gw[e])
        checked += 1
    print("fd edges checked", checked, flush=True)
    assert checked >= 10


@pytest.mark.parametrize("order", ["auto", "degree"])
def test_autograd_function(sp, order):
    d, gco = gen.diff_workload(side=20, num_sources=4)
    G = sp.Graph(d.n, d.src, d.dst, d.w, order=order)
    w_eid = torch.from_numpy(d.w[to_np(G.perm)]).cuda().requires_grad_(True)
    srcs = [int(s) for s in d.sources]
    cost = sp.shortest_paths(w_eid, G, srcs)
    g = torch.from_numpy(gco).cuda()
    reach = torch.isfinite(cost)
    loss = (torch.where(reach, cost, torch.zeros_like(cost)) * g).sum()
    loss.backward()
    sync()
    O = oracle.csr(d.n, d.src, d.dst)
    _, pred, _ = sp.solve_batch([G], [0] * 4, srcs)
    ref = oracle.grad(O, srcs, to_np(pred).astype(np.int64).reshape(4, d.n),
                      gco.astype(np.float64))
    got = to_np(w_eid.grad).astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


@pytest.mark.gpu
@pytest.mark.parametrize("order", ["input", "degree"])
def test_autograd_coo_order(sp, order):
    """Weights and gradient in the input (COO) order: the library permutes
    them through the builder's perm both ways.  Costs equal the edge-id
    order's bit for bit, the gradient is the edge-id gradient scattered to
    COO positions (bit for bit), and it matches the CPU gradient."""
    d, gco = gen.diff_workload(side=20, num_sources=4)
    G = sp.Graph(d.n, d.src, d.dst, d.w, order=order)
    perm = to_np(G.perm).astype(np.int64)
    assert sorted(perm.tolist()) == list(range(d.m))
    srcs = [int(s) for s in d.sources]
    g = torch.from_numpy(gco).cuda()

    def run(w, o):
        w = w.clone().requires_grad_(True)
        cost = sp.shortest_paths(w, G, srcs, order=o)
        reach = torch.isfinite(cost)
        (torch.where(reach, cost, torch.zeros_like(cost)) * g).sum().backward()
        sync()
        return cost.detach(), w.grad

    w_coo = torch.from_numpy(d.w).cuda()
    c_coo, g_coo = run(w_coo, "coo")
    c_eid, g_eid = run(torch.from_numpy(d.w[perm]).cuda(), "eid")
    assert torch.equal(c_coo, c_eid)
    gc, ge = to_np(g_coo), to_np(g_eid)
    assert np.array_equal(gc[perm], ge)
    O = oracle.csr(d.n, d.src, d.dst)
    _, pred, _ = sp.solve_batch([G], [0] * 4, srcs)
    ref = oracle.grad(O, srcs, to_np(pred).astype(np.int64).reshape(4, d.n),
                      gco.astype(np.float64))
    got = ge.astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


@pytest.mark.gpu
def test_permute_edges_both_ways(sp):
    """sssp_permute_edges against indexing by perm, on int32 and float32
    values of an RMAT graph in degree order (a non-trivial permutation)."""
    g = gen.rmat_workload(scale=12)
    G = sp.Graph(g.n, g.src, g.dst, g.w, order="degree")
    perm = G.perm.long()
    vi = torch.arange(g.m, dtype=torch.int32, device="cuda") * 7 + 3
    vf = torch.rand(g.m, dtype=torch.float32, device="cuda")
    for v in (vi, vf):
        e = G.to_edge_order(v)
        assert torch.equal(e, v[perm])
        back = G.to_coo_order(e)
        assert torch.equal(back, v)
    sync()
