"""CPU oracle for the lower/upper-bound SSSP method (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The GPU library never
imports, links or calls anything here, and nothing here imports the GPU
library.  The arithmetic lives in plain C (``oracle.c``, ``oracle_typed.inc``);
this module only marshals numpy arrays through ctypes.

Functions and the passages they follow:

* :func:`dijkstra` -- Fig. 1 (binary-heap Dijkstra); the definition of
  ``cost[x]`` in Section I.
* :func:`sp12` -- SP_1 and SP_2 (Figs. 3 and 4; Sections III and IV), the
  sequential algorithms, with their heap operations counted.
* :func:`bellman_ford` -- brute-force relaxation to a fixpoint (tiny graphs).
* :func:`dag` -- topological-order DP, the O(e) behaviour the SP_1/SP_2
  theorems give on acyclic graphs.
* :func:`bfs` -- hop distances; the SP_2 theorem on unweighted graphs.
* :func:`csr` / :func:`csr_weights` -- stable CSR by tail and CSC by head
  (incoming-edge access, Section I) and ``outWeight`` (Figs. 5 and 6).
* :func:`pred` -- parent pointers (Section I) under the smallest-tight-edge
  tie rule, with the equal-cost level rule for float ties.
* :func:`round_sim` -- the method's rounds (Eq. 1, Lemmas crule2 and crauser,
  Fig. 6's steps in the adopted sound order; mode 2 is Fig. 6 as printed;
  MODE_LC relaxes every discovered vertex whose D fell, as Fig. 6's step 3).
* :func:`grad` -- fp64 subtree-sum gradient of ``sum g * cost`` over the
  pred tree.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_typed.inc")]
_lib = None

TYPES = {np.dtype(np.int32): "i32", np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}
INF = {"i32": np.int32(2**31 - 1), "f32": np.float32(np.inf), "f64": np.float64(np.inf)}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain SSE float math, no fast-math)."""
    stale = not os.path.exists(_SO) or any(
        os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRCS)
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-msse2", "-mfpmath=sse", "-o", tmp,
             os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _kind(w):
    w = np.asarray(w)
    if w.dtype not in TYPES:
        raise TypeError("weights must be int32, float32 or float64, got %s" % w.dtype)
    return TYPES[w.dtype], np.ascontiguousarray(w)


def _call(name, *args):
    f = getattr(_L(), name)
    f.restype = ctypes.c_int
    return f(*args)


def dijkstra(n, src, dst, w, source, target=None):
    """Return (cost, settles): binary-heap Dijkstra (Fig. 1).  With a target,
    it stops once the target leaves the heap; settles counts the removals up
    to and including it."""
    k, w = _kind(w)
    src, dst = _i32(src), _i32(dst)
    cost = np.empty(n, dtype=w.dtype)
    settles = ctypes.c_int64(0)
    t = -1 if target is None else int(target)
    rc = _call("oracle_dijkstra_target_" + k, ctypes.c_int32(n), ctypes.c_int64(len(src)),
               _p(src), _p(dst), _p(w), ctypes.c_int32(source), ctypes.c_int32(t), _p(cost),
               ctypes.byref(settles))
    if rc != 0:
        raise ValueError("oracle_dijkstra failed: %d" % rc)
    return cost, settles.value


SP12_HOW = {0: "removeMin", 1: "pred", 2: "inWeight"}


class Adjacency:
    """A graph's out-adjacency built once (the COO indices of each tail's
    edges), so that :meth:`dijkstra` times the search alone."""

    def __init__(self, n, src, dst, w):
        k, self.w = _kind(w)
        self.kind = k
        self.n = int(n)
        src = _i32(src)
        self.dst = _i32(dst)
        self.off = np.empty(self.n + 1, dtype=np.int64)
        self.adj = np.empty(max(len(src), 1), dtype=np.int32)
        rc = _call("oracle_out_adjacency", ctypes.c_int32(self.n), ctypes.c_int64(len(src)),
                   _p(src), _p(self.off), _p(self.adj))
        if rc != 0:
            raise ValueError("oracle_out_adjacency failed: %d" % rc)

    def dijkstra(self, source, target=None):
        """(cost, settles) of Fig. 1's algorithm from `source`, as :func:`dijkstra`."""
        cost = np.empty(self.n, dtype=self.w.dtype)
        settles = ctypes.c_int64(0)
        t = -1 if target is None else int(target)
        rc = _call("oracle_dijkstra_adj_" + self.kind, ctypes.c_int32(self.n), _p(self.off),
                   _p(self.adj), _p(self.dst), _p(self.w), ctypes.c_int32(source),
                   ctypes.c_int32(t), _p(cost), ctypes.byref(settles))
        if rc != 0:
            raise ValueError("oracle_dijkstra_adj failed: %d" % rc)
        return cost, settles.value


def sp12(n, src, dst, w, source, variant, sequence=False):
    """SP_1 (variant 1, Fig. 3) or SP_2 (variant 2, Fig. 4), or Dijkstra in
    the same framework (variant 0); the outer loop ends once the heap holds
    no non-fixed vertex (the overloaded H.empty() of Section III).  Returns
    (cost, ops) with ops a dict of remove_min, insert, adjust and fixed_by_r
    counts; with sequence=True also the fix sequence as a list of
    (vertex, how) pairs, how one of SP12_HOW's names."""
    k, w = _kind(w)
    src, dst = _i32(src), _i32(dst)
    cost = np.empty(n, dtype=w.dtype)
    ops = np.zeros(4, dtype=np.int64)
    seq = np.empty(n, dtype=np.int32)
    how = np.empty(n, dtype=np.int32)
    rc = _call("oracle_sp12_" + k, ctypes.c_int32(n), ctypes.c_int64(len(src)), _p(src),
               _p(dst), _p(w), ctypes.c_int32(source), ctypes.c_int(variant), _p(cost), _p(ops),
               _p(seq), _p(how))
    if rc != 0:
        raise ValueError("oracle_sp12 failed: %d" % rc)
    o = dict(remove_min=int(ops[0]), insert=int(ops[1]), adjust=int(ops[2]),
             fixed_by_r=int(ops[3]))
    if not sequence:
        return cost, o
    fixes = [(int(v), SP12_HOW[int(h)]) for v, h in zip(seq, how) if v >= 0]
    return cost, o, fixes


def bellman_ford(n, src, dst, w, source):
    k, w = _kind(w)
    src, dst = _i32(src), _i32(dst)
    cost = np.empty(n, dtype=w.dtype)
    rc = _call("oracle_bellman_ford_" + k, ctypes.c_int32(n), ctypes.c_int64(len(src)), _p(src),
               _p(dst), _p(w), ctypes.c_int32(source), _p(cost))
    if rc != 0:
        raise ValueError("oracle_bellman_ford failed: %d" % rc)
    return cost


def dag(n, src, dst, w, source):
    """Topological-order DP; raises if the graph has a cycle."""
    k, w = _kind(w)
    src, dst = _i32(src), _i32(dst)
    cost = np.empty(n, dtype=w.dtype)
    rc = _call("oracle_dag_" + k, ctypes.c_int32(n), ctypes.c_int64(len(src)), _p(src), _p(dst),
               _p(w), ctypes.c_int32(source), _p(cost))
    if rc != 0:
        raise ValueError("oracle_dag failed: %d" % rc)
    return cost


def bfs(n, src, dst, source):
    src, dst = _i32(src), _i32(dst)
    hops = np.empty(n, dtype=np.int32)
    rc = _call("oracle_bfs", ctypes.c_int32(n), ctypes.c_int64(len(src)), _p(src), _p(dst),
               ctypes.c_int32(source), _p(hops))
    if rc != 0:
        raise ValueError("oracle_bfs failed: %d" % rc)
    return hops


class CSR:
    """Stable CSR by tail + CSC by head (arrays as numpy, ids int64)."""

    def __init__(self, n, src, dst):
        src, dst = _i32(src), _i32(dst)
        m = len(src)
        self.n, self.m = n, m
        self.out_off = np.empty(n + 1, dtype=np.int64)
        self.out_dst = np.empty(m, dtype=np.int32)
        self.perm = np.empty(m, dtype=np.int64)
        self.in_off = np.empty(n + 1, dtype=np.int64)
        self.in_src = np.empty(m, dtype=np.int32)
        self.in_eid = np.empty(m, dtype=np.int64)
        rc = _call("oracle_csr", ctypes.c_int32(n), ctypes.c_int64(m), _p(src), _p(dst),
                   _p(self.out_off), _p(self.out_dst), _p(self.perm), _p(self.in_off),
                   _p(self.in_src), _p(self.in_eid))
        if rc != 0:
            raise ValueError("oracle_csr failed: %d" % rc)

    def weights(self, w):
        """Return (out_w, in_w, out_wmin) for COO weights w."""
        k, w = _kind(w)
        out_w = np.empty(self.m, dtype=w.dtype)
        in_w = np.empty(self.m, dtype=w.dtype)
        wmin = np.empty(self.n, dtype=w.dtype)
        f = getattr(_L(), "oracle_csr_weights_" + k)
        f.restype = None
        f(
            ctypes.c_int32(self.n), ctypes.c_int64(self.m), _p(self.out_off), _p(self.perm),
            _p(self.in_eid), _p(w), _p(out_w), _p(in_w), _p(wmin))
        return out_w, in_w, wmin


def csr(n, src, dst):
    return CSR(n, src, dst)


def pred(g: CSR, w, source, cost):
    """Parent edge ids (stable CSR positions) under the tie rule; -1 for the
    source and unreachable vertices.  Returns (pred, n_equal_cost_ties)."""
    k, w = _kind(w)
    _, in_w, _ = g.weights(w)
    cost = np.ascontiguousarray(cost, dtype=w.dtype)
    out = np.empty(g.n, dtype=np.int64)
    rc = _call("oracle_pred_" + k, ctypes.c_int32(g.n), ctypes.c_int32(source), _p(cost),
               _p(g.in_off), _p(g.in_src), _p(g.in_eid), _p(in_w), _p(out))
    if rc < 0:
        raise ValueError("oracle_pred failed: %d" % rc)
    return out, rc


MODE_ADOPTED, MODE_SCOPE_ALL, MODE_LITERAL_FIG5 = 0, 1, 2
MODE_LC = 4  # or-ed with MODE_ADOPTED / MODE_SCOPE_ALL: label-correcting relax


def round_sim(n, src, dst, w, source, mode=MODE_ADOPTED, true_cost=None, target=None,
              delta=None):
    """Run the round simulator.  Returns dict(cost, rounds, fixed_per_round,
    scanned_per_round, relaxed_edges, scanned_in_edges, open_visits, settled,
    violations).  With a target
    (modes 0 and 1) the rounds stop once the target is fixed.  delta (with
    MODE_LC): an open vertex joins the relax set only while D < minD + delta
    (None: no bound)."""
    k, w = _kind(w)
    if delta is None:
        dl = {"i32": ctypes.c_int32(2**31 - 1), "f32": ctypes.c_float(np.inf),
              "f64": ctypes.c_double(np.inf)}[k]
    else:
        dl = {"i32": ctypes.c_int32, "f32": ctypes.c_float, "f64": ctypes.c_double}[k](delta)
    src, dst = _i32(src), _i32(dst)
    cost = np.empty(n, dtype=w.dtype)
    cap = 4 * n + 8
    fpr = np.zeros(cap, dtype=np.int64)
    spr = np.zeros(cap, dtype=np.int64)
    stats = np.zeros(4, dtype=np.int64)
    t = -1 if target is None else int(target)
    rounds = ctypes.c_int64(0)
    viol = ctypes.c_int64(0)
    tc = None
    if true_cost is not None:
        tc = np.ascontiguousarray(true_cost, dtype=w.dtype)
    rc = _call("oracle_round_sim_" + k, ctypes.c_int32(n), ctypes.c_int64(len(src)), _p(src),
               _p(dst), _p(w), ctypes.c_int32(source), ctypes.c_int32(t), ctypes.c_int(mode),
               dl, _p(cost),
               ctypes.byref(rounds), _p(fpr), _p(spr), ctypes.c_int64(cap), _p(stats),
               _p(tc) if tc is not None else None, ctypes.byref(viol))
    if rc != 0:
        raise ValueError("oracle_round_sim failed: %d" % rc)
    r = rounds.value
    return dict(cost=cost, rounds=r, fixed_per_round=fpr[:r].copy(),
                scanned_per_round=spr[:r].copy(), relaxed_edges=int(stats[0]),
                scanned_in_edges=int(stats[1]), settled=int(stats[2]),
                open_visits=int(stats[3]), violations=viol.value)


def grad(g: CSR, sources, preds, gcoef):
    """fp64 dL/dw per edge (CSR order) for L = sum_s sum_x gcoef[s,x]*cost_s[x]."""
    sources = _i32(np.atleast_1d(sources))
    preds = np.ascontiguousarray(np.atleast_2d(preds), dtype=np.int64)
    gc = np.ascontiguousarray(np.atleast_2d(gcoef), dtype=np.float64)
    assert preds.shape == (len(sources), g.n) and gc.shape == preds.shape
    out = np.empty(g.m, dtype=np.float64)
    rc = _call("oracle_grad", ctypes.c_int32(g.n), ctypes.c_int64(g.m), _p(g.out_off),
               _p(g.out_dst), ctypes.c_int32(len(sources)), _p(sources), _p(preds), _p(gc),
               _p(out))
    if rc != 0:
        raise ValueError("oracle_grad failed: %d" % rc)
    return out
