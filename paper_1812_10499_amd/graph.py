"""PyTorch-facing helpers over the C ABI: device memory, streams and shapes.

PyTorch only allocates device memory and supplies the current stream; every
step of the method runs in libsssp.so.  Nothing here computes a shortest
path.
"""
from __future__ import annotations

import ctypes
import weakref
from typing import Sequence

import numpy as np
import torch

from . import _abi
from ._abi import (Csr, SSSP_F32, SSSP_I32, SSSP_ORDER_AUTO, SSSP_ORDER_DEGREE,
                   SSSP_SCOPE_ALL, SSSP_SCOPE_AUTO, SSSP_SCOPE_OPEN, SSSP_RELAX_AUTO,
                   SSSP_RELAX_CORRECTING, SSSP_RELAX_SETTING,
                   SSSP_ORDER_INPUT, Stats)

I32_INF = 2**31 - 1
ORDERS = {"auto": SSSP_ORDER_AUTO, "input": SSSP_ORDER_INPUT, "degree": SSSP_ORDER_DEGREE}
SCOPES = {"auto": SSSP_SCOPE_AUTO, "open": SSSP_SCOPE_OPEN, "all": SSSP_SCOPE_ALL}
RELAXES = {"auto": SSSP_RELAX_AUTO, "setting": SSSP_RELAX_SETTING,
           "correcting": SSSP_RELAX_CORRECTING}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_i32(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)


class Graph:
    """A directed graph built on the GPU (CSR by tail + CSC by head).

    Edge ids are positions in the CSR; ``perm[k]`` is the input (COO) index
    of edge id ``k``.  Weights are int32 (>= 1) or float32 (> 0).  ``order``
    picks the vertex numbering of the solver's working copy ("auto",
    "input" or "degree"); ``scope`` the C scope of single solves ("auto",
    "open" or "all"; see :attr:`scope`), ``relax`` the relax step ("auto",
    "setting" or "correcting"; see :attr:`relax`), ``delta`` the bucket
    width of label-correcting relax (see :attr:`delta`).  Results never
    depend on any of them.
    """

    def __init__(self, n: int, src, dst, w, device="cuda", order: str = "auto",
                 scope: str = "auto", relax: str = "auto", delta=None):
        device = torch.device(device)
        if isinstance(w, torch.Tensor):
            wt = w.to(device).contiguous()
        else:
            wt = torch.from_numpy(np.ascontiguousarray(w)).to(device)
        if wt.dtype == torch.int32:
            self.dtype = SSSP_I32
        elif wt.dtype == torch.float32:
            self.dtype = SSSP_F32
        else:
            raise TypeError("weights must be int32 or float32, got %s" % wt.dtype)
        s = _dev_i32(src, device)
        d = _dev_i32(dst, device)
        m = int(s.numel())
        if d.numel() != m or wt.numel() != m:
            raise ValueError("src, dst and w must have the same length")
        self.n, self.m, self.device = int(n), m, device
        if order not in ORDERS:
            raise ValueError("order must be one of %s" % sorted(ORDERS))
        nbytes = _abi.sssp_build_csr_bytes(self.n, m, self.dtype, ORDERS[order])
        if nbytes == 0:
            raise ValueError("invalid graph size n=%d m=%d" % (n, m))
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.perm = torch.empty(max(m, 1), dtype=torch.int32, device=device)
        self.csr = Csr()
        _abi.sssp_build_csr(self.n, m, self.dtype, ORDERS[order], s.data_ptr(), d.data_ptr(),
                            wt.data_ptr(), self.buffer.data_ptr(), nbytes, self.csr,
                            self.perm.data_ptr(), _stream())
        self.perm = self.perm[:m]
        self.scope = scope
        self.relax = relax
        self.delta = delta

    @property
    def scope(self) -> str:
        """C scope of the solves as set: "auto", "open" or "all"."""
        return {v: k for k, v in SCOPES.items()}[self.csr.scope]

    @scope.setter
    def scope(self, value: str):
        if value not in SCOPES:
            raise ValueError("scope must be one of %s" % sorted(SCOPES))
        self.csr.scope = SCOPES[value]

    def policy(self) -> dict:
        """What the library resolves this graph's AUTO settings to (asked of
        the library: sssp_policy_of): scope, relax, delta (None: no bound,
        or label-setting) and the round kernel of a single solve under the
        device's current default launch geometry."""
        p = _abi.sssp_policy_of(self.csr)
        if p.relax != SSSP_RELAX_CORRECTING or p.delta == (
                0x7f800000 if self.dtype == SSSP_F32 else I32_INF):
            delta = None
        elif self.dtype == SSSP_F32:
            delta = float(np.array([p.delta], np.int32).view(np.float32)[0])
        else:
            delta = int(p.delta)
        return dict(scope="all" if p.scope == SSSP_SCOPE_ALL else "open",
                    relax="correcting" if p.relax == SSSP_RELAX_CORRECTING else "setting",
                    delta=delta, kernel=_abi.KERNELS[p.kernel])

    @property
    def effective_scope(self) -> str:
        """The scope solves run ("auto" resolved by the library)."""
        return self.policy()["scope"]

    @property
    def relax(self) -> str:
        """Relax step of every solve as set: "auto", "setting" or "correcting"."""
        return {v: k for k, v in RELAXES.items()}[self.csr.relax]

    @relax.setter
    def relax(self, value: str):
        if value not in RELAXES:
            raise ValueError("relax must be one of %s" % sorted(RELAXES))
        self.csr.relax = RELAXES[value]

    @property
    def effective_relax(self) -> str:
        """The relax step solves run ("auto" resolved by the library)."""
        return self.policy()["relax"]

    @property
    def effective_delta(self):
        """The bucket width label-correcting solves use (None: no bound, or
        label-setting), as the library resolves it."""
        return self.policy()["delta"]

    @property
    def kernel(self) -> str:
        """The round kernel a single solve of this graph runs now."""
        return self.policy()["kernel"]

    @property
    def delta(self):
        """Bucket width of label-correcting relax (an open vertex joins the
        relax set only while D < minD + delta), or None for no bound."""
        if self.dtype == SSSP_F32:
            v = float(np.array([self.csr.delta], np.int32).view(np.float32)[0])
            return None if v == float("inf") else v
        return None if self.csr.delta == I32_INF else int(self.csr.delta)

    @delta.setter
    def delta(self, value):
        if value is None:
            self.csr.delta = 0x7f800000 if self.dtype == SSSP_F32 else I32_INF
            return
        if self.dtype == SSSP_F32:
            v = np.float32(value)
            if not (v >= 0):
                raise ValueError("delta must be >= 0")
            self.csr.delta = int(np.array([v], np.float32).view(np.int32)[0])
        else:
            v = int(value)
            if v < 0:
                raise ValueError("delta must be >= 0")
            self.csr.delta = min(v, I32_INF)

    @property
    def order(self) -> str:
        """The numbering the builder applied: "input" or "degree"."""
        return "degree" if self.csr.order == SSSP_ORDER_DEGREE else "input"

    @property
    def value_dtype(self):
        return torch.float32 if self.dtype == SSSP_F32 else torch.int32

    def _view(self, ptr, count, dtype=torch.int32):
        off = ptr - self.buffer.data_ptr()
        return self.buffer[off:off + 4 * count].view(dtype)

    def arrays(self) -> dict:
        """Views of the built arrays (out_off, out_dst, out_w, in_off, in_src,
        in_eid, in_w, out_wmin)."""
        c, n, m, vt = self.csr, self.n, self.m, self.value_dtype
        return dict(out_off=self._view(c.out_off, n + 1), out_dst=self._view(c.out_dst, m),
                    out_w=self._view(c.out_w, m, vt), in_off=self._view(c.in_off, n + 1),
                    in_src=self._view(c.in_src, m), in_eid=self._view(c.in_eid, m),
                    in_w=self._view(c.in_w, m, vt), out_wmin=self._view(c.out_wmin, n, vt))

    def solver_arrays(self) -> dict:
        """Views of the solver's working copy: the weight-ordered in-lists (also
        as (tail, weight-bits) pairs), the out-edge records (head, weight bits,
        edge id, the head's out_wmin bits), the vertex records and their
        in-side halves, and in degree
        order also vid, rank and the renumbered out-lists."""
        c, n, m, vt = self.csr, self.n, self.m, self.value_dtype
        out = dict(in_off=self._view(c.s_in_off, n + 1), in_src=self._view(c.s_in_src, m),
                   in_eid=self._view(c.s_in_eid, m), in_w=self._view(c.s_in_w, m, vt),
                   in_sw=self._view(c.s_in_sw, 2 * m).view(m, 2),
                   out_rec=self._view(c.s_out_rec, 4 * m).view(m, 4),
                   vrec=self._view(c.s_vrec, 8 * n).view(n, 8),
                   vin=self._view(c.s_vin, 4 * n).view(n, 4))
        if self.csr.order == SSSP_ORDER_DEGREE:
            out.update(vid=self._view(c.vid, n), rank=self._view(c.rank, n),
                       out_off=self._view(c.s_out_off, n + 1),
                       out_dst=self._view(c.s_out_dst, m), out_w=self._view(c.s_out_w, m, vt),
                       out_eid=self._view(c.s_out_eid, m),
                       out_wmin=self._view(c.s_out_wmin, n, vt))
        return out

    def to_edge_order(self, values_coo: torch.Tensor) -> torch.Tensor:
        """Per-edge values given in the input (COO) order, in edge-id order
        (sssp_permute_edges through the builder's permutation)."""
        return self._permute(values_coo, to_coo=False)

    def to_coo_order(self, values_eid: torch.Tensor) -> torch.Tensor:
        """Per-edge values given in edge-id order, in the input (COO) order."""
        return self._permute(values_eid, to_coo=True)

    def _permute(self, v: torch.Tensor, to_coo: bool) -> torch.Tensor:
        if v.numel() != self.m:
            raise ValueError("expected %d per-edge values" % self.m)
        if v.element_size() != 4:
            raise ValueError("per-edge values must be 4-byte (float32 or int32)")
        v = v.to(self.device).contiguous()
        out = torch.empty_like(v)
        _abi.sssp_permute_edges(self.perm.data_ptr(), self.m, v.data_ptr(), out.data_ptr(),
                                to_coo, _stream())
        return out

    def set_weights(self, w_eid: torch.Tensor):
        """Replace the weights; w_eid is given in edge-id order."""
        w_eid = w_eid.to(device=self.device, dtype=self.value_dtype).contiguous()
        if w_eid.numel() != self.m:
            raise ValueError("expected %d weights" % self.m)
        _abi.sssp_set_weights(self.csr, w_eid.data_ptr(), _stream())


def solve(g: Graph, source: int, with_pred: bool = True, with_stats: bool = False):
    """Returns (cost[n], pred[n] or None, stats dict or None)."""
    cost = torch.empty(g.n, dtype=g.value_dtype, device=g.device)
    pred = torch.empty(g.n, dtype=torch.int32, device=g.device) if with_pred else None
    st = Stats() if with_stats else None
    _abi.sssp_solve(g.csr, int(source), cost.data_ptr(), pred.data_ptr() if with_pred else None,
                    st, _stream())
    return cost, pred, (st.as_dict() if st is not None else None)


def solve_target(g: Graph, source: int, target: int, with_stats: bool = False):
    """Rounds until `target` is fixed.  Returns (cost[n], stats dict or None):
    cost is exact for every vertex fixed by then, the target among them."""
    cost = torch.empty(g.n, dtype=g.value_dtype, device=g.device)
    st = Stats() if with_stats else None
    _abi.sssp_solve_target(g.csr, int(source), int(target), cost.data_ptr(), st, _stream())
    return cost, (st.as_dict() if st is not None else None)


def batch_layout(graphs: Sequence[Graph], inst_graph: Sequence[int]):
    bases, b = [], 0
    for gi in inst_graph:
        bases.append(b)
        b += graphs[gi].n
    return bases, b


def solve_batch(graphs: Sequence[Graph], inst_graph: Sequence[int], inst_source: Sequence[int],
                with_pred: bool = True, with_stats: bool = False):
    """Returns (cost[total], pred[total] or None, list of stats dicts or None);
    instance i occupies [base_i, base_i + n_i)."""
    _, total = batch_layout(graphs, inst_graph)
    dev = graphs[0].device
    cost = torch.empty(total, dtype=graphs[0].value_dtype, device=dev)
    pred = torch.empty(total, dtype=torch.int32, device=dev) if with_pred else None
    st = (Stats * len(inst_graph))() if with_stats else None
    _abi.sssp_solve_batch([g.csr for g in graphs], inst_graph, inst_source, cost.data_ptr(),
                          pred.data_ptr() if with_pred else None, st, _stream())
    stats = [s.as_dict() for s in st] if st is not None else None
    return cost, pred, stats


PLAN_KINDS = {"batch": _abi.SSSP_PLAN_BATCH, "sequence": _abi.SSSP_PLAN_SEQUENCE}
_live_plans = weakref.WeakSet()


def close_plans():
    """Destroys every plan still open (called at process exit)."""
    for p in list(_live_plans):
        p.close()


def _launch(launch):
    if launch is None or isinstance(launch, _abi.Launch):
        return launch
    return _abi.Launch(int(launch.get("blocks", 0)), int(launch.get("solo_edges", 0)),
                       int(launch.get("block_units", 0)), int(launch.get("small_n", 0)),
                       int(launch.get("wg", 0)))


class Plan:
    """Solves recorded once into a HIP graph and replayed by :meth:`run`.

    kind "batch": one persistent launch for all instances (as
    :func:`solve_batch`); "sequence": one single solve per instance, back
    to back.  ``cost`` and ``pred`` (the latter optional) are allocated here
    in the batch layout and rewritten by every run.  ``launch`` is a dict
    (blocks, solo_edges, block_units, small_n, wg) or None for the defaults.
    """

    def __init__(self, graphs: Sequence[Graph], inst_graph: Sequence[int],
                 inst_source: Sequence[int], kind: str = "batch", with_pred: bool = True,
                 with_stats: bool = False, launch=None):
        _, total = batch_layout(graphs, inst_graph)
        dev = graphs[0].device
        self.graphs = list(graphs)  # keeps the graph buffers alive
        self.num_inst = len(inst_graph)
        self.cost = torch.empty(total, dtype=graphs[0].value_dtype, device=dev)
        self.pred = torch.empty(total, dtype=torch.int32, device=dev) if with_pred else None
        self.handle = None
        self.handle = _abi.sssp_plan_create(
            [g.csr for g in graphs], inst_graph, inst_source, PLAN_KINDS[kind],
            self.cost.data_ptr(), self.pred.data_ptr() if with_pred else None, with_stats,
            _launch(launch))
        _live_plans.add(self)

    def run(self):
        """Replays the recorded solves on the current stream (asynchronous)."""
        _abi.sssp_plan_run(self.handle, _stream())
        return self.cost, self.pred

    def stats(self):
        st = (Stats * self.num_inst)()
        _abi.sssp_plan_stats(self.handle, st, _stream())
        return [s.as_dict() for s in st]

    def close(self):
        if self.handle:
            _abi.sssp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(graphs: Sequence[Graph], inst_graph: Sequence[int], inst_source: Sequence[int],
             kind: str = "batch", reps: int = 2):
    """Times replays under candidate launch geometries; returns (launch dict,
    mean ms per run).  Pass the dict to :class:`Plan` or :func:`set_launch`."""
    _, total = batch_layout(graphs, inst_graph)
    dev = graphs[0].device
    cost = torch.empty(total, dtype=graphs[0].value_dtype, device=dev)
    pred = torch.empty(total, dtype=torch.int32, device=dev)
    best, ms = _abi.sssp_autotune([g.csr for g in graphs], inst_graph, inst_source,
                                  PLAN_KINDS[kind], cost.data_ptr(), pred.data_ptr(), reps,
                                  _stream())
    return best.as_dict(), ms


def check():
    """Waits for the current stream; raises SSSPError (SSSP_ERR_INTERNAL) if
    a solve since the last check on this device hit the round watchdog."""
    _abi.sssp_check(_stream())


def set_round_limit(limit: int = 0):
    """Diagnostics: cap the round watchdog of later solves (0: the default)."""
    _abi.sssp_set_round_limit(limit)


def set_launch(launch=None):
    """Default launch geometry of this device's direct solves (None: defaults)."""
    _abi.sssp_set_launch(_launch(launch))


def backward(graphs: Sequence[Graph], inst_graph: Sequence[int], inst_source: Sequence[int],
             pred: torch.Tensor, grad_cost: torch.Tensor) -> torch.Tensor:
    """dL/dw for L = sum grad_cost * cost over the pred trees; returns
    float32[sum of m] with graph g's edges (edge-id order) at its offset."""
    total_m = sum(g.m for g in graphs)
    dev = graphs[0].device
    grad_w = torch.empty(max(total_m, 1), dtype=torch.float32, device=dev)
    gc = grad_cost.to(device=dev, dtype=torch.float32).contiguous()
    pr = pred.to(device=dev, dtype=torch.int32).contiguous()
    _abi.sssp_backward([g.csr for g in graphs], inst_graph, inst_source, pr.data_ptr(),
                       gc.data_ptr(), grad_w.data_ptr(), _stream())
    return grad_w[:total_m]


class SSSPFunction(torch.autograd.Function):
    """cost[S, n] = shortest-path costs from S sources on one float32 graph,
    differentiable in the edge weights.  order "eid": the weights (and their
    gradient) are in edge-id order; "coo": in the order of the edges the
    graph was built from (the library permutes them both ways)."""

    @staticmethod
    def forward(ctx, w: torch.Tensor, graph: Graph, sources: Sequence[int], order: str = "eid"):
        if order not in ("eid", "coo"):
            raise ValueError("order must be 'eid' or 'coo'")
        w = w.detach()
        graph.set_weights(graph.to_edge_order(w) if order == "coo" else w)
        S = len(sources)
        cost, pred, _ = solve_batch([graph], [0] * S, list(sources), with_pred=True)
        ctx.graph, ctx.sources, ctx.order = graph, list(sources), order
        ctx.save_for_backward(pred)
        return cost.view(S, graph.n)

    @staticmethod
    def backward(ctx, grad_cost):
        (pred,) = ctx.saved_tensors
        g = ctx.graph
        gw = backward([g], [0] * len(ctx.sources), ctx.sources, pred,
                      grad_cost.reshape(-1))
        if ctx.order == "coo":
            gw = g.to_coo_order(gw)
        return gw, None, None, None


def shortest_paths(w: torch.Tensor, graph: Graph, sources: Sequence[int],
                   order: str = "eid") -> torch.Tensor:
    """Differentiable costs from `sources`; `w` in edge-id ("eid") or input
    ("coo") order (see SSSPFunction)."""
    return SSSPFunction.apply(w, graph, sources, order)
