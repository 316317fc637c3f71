"""Fault status without stats, and the backward pass on a parent array that
names an in-edge of the source.

The round watchdog is forced from the host: sssp_set_round_limit caps the
rounds below what the solve needs, so every kernel path stops at the cap and
exits normally; the status must then reach the caller through sssp_check
(and through the call itself when it asks for stats).
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import sync, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    assert torch.cuda.is_available()
    return sp


def _path(k, dtype=np.int32):
    src = np.arange(k, dtype=np.int32)
    return k + 1, src, src + 1, np.full(k, 3, dtype)


@pytest.mark.parametrize("kernel", ["small_rounds_kernel", "wg_rounds_kernel", "rounds_kernel"])
def test_watchdog_reaches_the_caller(sp, kernel):
    # a 5000-vertex path: 5000 rounds; scope OPEN keeps it on the workgroup
    # kernel by default, scope ALL on the persistent one; small_n covers the
    # LDS kernel
    n, src, dst, w = _path(4999 if kernel != "small_rounds_kernel" else 3000)
    G = sp.Graph(n, src, dst, w, scope=("all" if kernel == "rounds_kernel" else "open"))
    assert G.kernel == kernel, G.policy()
    sp.check()  # nothing pending
    try:
        sp.set_round_limit(40)
        print("watchdog", kernel, "no stats", flush=True)
        sp.solve(G, 0, with_pred=True, with_stats=False)
        with pytest.raises(sp.SSSPError) as e:
            sp.check()
        assert e.value.status == sp.SSSP_ERR_INTERNAL
        sp.check()  # cleared by the first check
        print("watchdog", kernel, "with stats", flush=True)
        with pytest.raises(sp.SSSPError) as e:
            sp.solve(G, 0, with_pred=True, with_stats=True)
        assert e.value.status == sp.SSSP_ERR_INTERNAL
        # sssp_check reports every fault since the previous check, this one too
        with pytest.raises(sp.SSSPError):
            sp.check()
        sp.check()
    finally:
        sp.set_round_limit(0)
        try:
            sp.check()
        except sp.SSSPError:
            pass
    # back to normal: the full solve is exact and reports no fault
    cost, pred, st = sp.solve(G, 0, with_pred=True, with_stats=True)
    sync()
    sp.check()
    assert to_np(cost).tolist() == [3 * i for i in range(n)]
    assert st["rounds"] == n


def test_watchdog_in_plans_and_batches(sp):
    n, src, dst, w = _path(6000)
    G = sp.Graph(n, src, dst, w)
    try:
        sp.set_round_limit(25)
        plan = sp.Plan([G, G], [0, 1], [0, 0], kind="batch")
        sp.set_round_limit(0)
        plan.run()
        with pytest.raises(sp.SSSPError) as e:
            sp.check()
        assert e.value.status == sp.SSSP_ERR_INTERNAL
        plan.close()
        sp.set_round_limit(25)
        sp.solve_batch([G], [0, 0], [0, 5], with_pred=False, with_stats=False)
        with pytest.raises(sp.SSSPError):
            sp.check()
    finally:
        sp.set_round_limit(0)
    plan = sp.Plan([G], [0], [0], kind="batch")
    c, _ = plan.run()
    sync()
    sp.check()
    assert to_np(c)[-1] == 3 * (n - 1)
    plan.close()


@pytest.mark.parametrize("wg", [1, -1])
@pytest.mark.parametrize("num_sources", [1, 3])
def test_backward_ignores_a_parent_of_the_source(sp, wg, num_sources):
    """pred[source] set to an in-edge of the source whose tail is in the
    source's own tree: the source stays the root and the gradients are those
    of the well-formed pred array, bit for bit.  With one source that edge
    (its head is the source) gets gradient 0; with several it may still be a
    tree edge of another source's tree."""
    d, gco = gen.diff_workload(side=32, num_sources=3)
    G = sp.Graph(d.n, d.src, d.dst, d.w)
    srcs = [int(s) for s in d.sources][:num_sources]
    S = len(srcs)
    gco = gco[:S]
    _, pred, _ = sp.solve_batch([G], [0] * S, srcs)
    sync()
    gcost = torch.from_numpy(np.ascontiguousarray(gco).reshape(-1)).cuda()
    O = oracle.csr(d.n, d.src, d.dst)
    bad = pred.clone()
    into = []
    for i, s in enumerate(srcs):
        # an in-edge of the source (O.in_eid lists edge ids by head)
        e = int(O.in_eid[O.in_off[s]])
        into.append(e)
        bad[i * d.n + s] = e
    print("backward root test: wg", wg, "sources", S, flush=True)
    try:
        sp.set_launch({"wg": wg})
        ref = to_np(sp.backward([G], [0] * S, srcs, pred, gcost))
        got = to_np(sp.backward([G], [0] * S, srcs, bad, gcost))
        sync()
    finally:
        sp.set_launch(None)
    p = to_np(pred).astype(np.int64).reshape(S, d.n)
    want = oracle.grad(O, srcs, p, gco.astype(np.float64))
    assert np.linalg.norm(ref - want) / np.linalg.norm(want) <= 1e-5
    assert np.array_equal(got, ref)
    if S == 1:
        assert got[into[0]] == 0.0
