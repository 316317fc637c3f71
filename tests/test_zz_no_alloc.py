"""The allocation-free solve (sssp_solve_noalloc) against sssp_solve.

Called through the C ABI on the same built graphs, it must give the same
costs and parents bit for bit and the same counters, with and without stats,
on consecutive calls whose graphs shrink (the static region keeps the
previous call's contents), on every round-kernel path; a graph whose state
does not fit the region is refused with SSSP_ERR_CAPACITY and leaves the
next call unaffected.
"""
import numpy as np
import pytest
import torch

import gen
from gpu_util import sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def _both(sp, G, source, label):
    print("noalloc", label, "n=%d m=%d kernel=%s" % (G.n, G.m, G.kernel), flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    for fn in (sp.sssp_solve, sp.sssp_solve_noalloc, sp.sssp_solve_noalloc):
        c = torch.full((G.n,), 7, dtype=G.value_dtype, device="cuda")
        p = torch.full((G.n,), -7, dtype=torch.int32, device="cuda")
        st = sp.Stats() if len(out) < 2 else None  # the last call: no stats, asynchronous
        fn(G.csr, int(source), c.data_ptr(), p.data_ptr(), st, stream)
        out.append((c, p, st.as_dict() if st is not None else None))
    sync()
    sp.check()
    (c0, p0, s0), (c1, p1, s1), (c2, p2, _) = out
    for c, p in ((c1, p1), (c2, p2)):
        assert np.array_equal(to_np(c).view(np.int32), to_np(c0).view(np.int32)), label
        assert np.array_equal(to_np(p), to_np(p0)), label
    assert s1 == s0, (label, s0, s1)


def test_noalloc_matches_solve_on_shrinking_graphs(sp):
    # every kernel path, each graph smaller than the one before
    r18 = gen.rmat_workload(scale=18)
    G = sp.Graph(r18.n, r18.src, r18.dst, r18.w)
    assert G.kernel == "rounds_kernel"
    _both(sp, G, r18.source, "rmat18")
    d, _ = gen.diff_workload(side=300, num_sources=2)
    G = sp.Graph(d.n, d.src, d.dst, d.w)
    assert G.kernel == "wg_rounds_kernel"
    _both(sp, G, int(d.sources[0]), "grid300 f32")
    g = gen.grid_workload(side=200)
    G = sp.Graph(g.n, g.src, g.dst, g.w)
    assert G.kernel == "wg_rounds_kernel" and G.effective_relax == "correcting"
    _both(sp, G, g.source, "grid200 i32 label-correcting")
    r12 = gen.rmat_workload(scale=12)
    G = sp.Graph(r12.n, r12.src, r12.dst, r12.w, scope="all", relax="correcting")
    _both(sp, G, r12.source, "rmat12 all correcting")
    g = gen.random_workload(n=3000, m=24000)
    G = sp.Graph(g.n, g.src, g.dst, g.w)
    assert G.kernel == "small_rounds_kernel"
    _both(sp, G, g.source, "random3000")


def test_noalloc_holds_its_stated_capacity(sp):
    # the header's promise: every graph with n <= 450,000 fits, whatever its
    # scope and relax step (scope ALL and label-correcting relax need the
    # most state)
    g = gen.random_workload(n=450000, m=1800000)
    G = sp.Graph(g.n, g.src, g.dst, g.w, scope="all", relax="correcting")
    _both(sp, G, g.source, "random450000 all correcting")


def test_noalloc_refuses_a_graph_beyond_its_region(sp):
    n = 600000
    src = np.arange(n - 1, dtype=np.int32)
    G = sp.Graph(n, src, src + 1, np.ones(n - 1, np.int32))
    c = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(sp.SSSPError) as e:
        sp.sssp_solve_noalloc(G.csr, 0, c.data_ptr(), None, None,
                              torch.cuda.current_stream().cuda_stream)
    assert e.value.status == sp.SSSP_ERR_CAPACITY
    # a graph that fits, right after
    r = gen.rmat_workload(scale=14)
    _both(sp, sp.Graph(r.n, r.src, r.dst, r.w), r.source, "rmat14 after a refusal")
