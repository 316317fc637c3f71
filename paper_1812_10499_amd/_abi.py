"""ctypes binding of the C ABI declared in include/sssp.h.

Argument marshalling only: every function here forwards to the function of
the same name in libsssp.so and raises :class:`SSSPError` on a non-zero
status.  Pointers are passed as Python ints (device addresses, e.g.
``tensor.data_ptr()``), streams as the raw HIP stream handle.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import torch  # noqa: F401  (load PyTorch's HIP runtime first: one runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsssp.so")

SSSP_I32, SSSP_F32 = 0, 1
SSSP_ORDER_AUTO, SSSP_ORDER_INPUT, SSSP_ORDER_DEGREE = 0, 1, 2
SSSP_SCOPE_AUTO, SSSP_SCOPE_OPEN, SSSP_SCOPE_ALL = 0, 1, 2
SSSP_RELAX_AUTO, SSSP_RELAX_SETTING, SSSP_RELAX_CORRECTING = 0, 1, 2
(SSSP_OK, SSSP_ERR_ARG, SSSP_ERR_GRAPH, SSSP_ERR_WEIGHT, SSSP_ERR_OVERFLOW, SSSP_ERR_NOMEM,
 SSSP_ERR_HIP, SSSP_ERR_INTERNAL, SSSP_ERR_CAPACITY) = range(9)

SSSP_PLAN_BATCH, SSSP_PLAN_SEQUENCE = 0, 1

EXPORTS = ("sssp_build_csr_bytes", "sssp_build_csr", "sssp_set_weights", "sssp_solve",
           "sssp_solve_target", "sssp_solve_batch", "sssp_backward", "sssp_set_launch",
           "sssp_plan_create", "sssp_plan_run", "sssp_plan_stats", "sssp_plan_destroy",
           "sssp_autotune", "sssp_release_workspace", "sssp_strerror",
           "sssp_profile_enable", "sssp_profile_read", "sssp_check", "sssp_set_round_limit",
           "sssp_policy_of", "sssp_solve_noalloc", "sssp_permute_edges")
KERNELS = {0: "rounds_kernel", 1: "wg_rounds_kernel", 2: "small_rounds_kernel"}


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("order", ctypes.c_int32), ("scope", ctypes.c_int32),
                ("relax", ctypes.c_int32), ("deg_max", ctypes.c_int32),
                ("delta", ctypes.c_int32),
                ("out_off", ctypes.c_void_p), ("out_dst", ctypes.c_void_p),
                ("out_w", ctypes.c_void_p), ("in_off", ctypes.c_void_p),
                ("in_src", ctypes.c_void_p), ("in_eid", ctypes.c_void_p),
                ("in_w", ctypes.c_void_p), ("out_wmin", ctypes.c_void_p),
                ("w_max", ctypes.c_double), ("w_min", ctypes.c_double),
                ("vid", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("s_out_off", ctypes.c_void_p), ("s_out_dst", ctypes.c_void_p),
                ("s_out_w", ctypes.c_void_p), ("s_out_eid", ctypes.c_void_p),
                ("s_in_off", ctypes.c_void_p), ("s_in_src", ctypes.c_void_p),
                ("s_in_eid", ctypes.c_void_p), ("s_in_w", ctypes.c_void_p),
                ("s_out_wmin", ctypes.c_void_p), ("s_vrec", ctypes.c_void_p),
                ("s_in_sw", ctypes.c_void_p), ("s_out_rec", ctypes.c_void_p),
                ("s_vin", ctypes.c_void_p)]


class Policy(ctypes.Structure):
    _fields_ = [("scope", ctypes.c_int32), ("relax", ctypes.c_int32),
                ("delta", ctypes.c_int32), ("kernel", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("settled", ctypes.c_int32),
                ("relaxed_edges", ctypes.c_int64), ("scanned_in_edges", ctypes.c_int64),
                ("open_visits", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Launch(ctypes.Structure):
    """Launch geometry of the round kernel (0 in a field: the default)."""
    _fields_ = [("blocks", ctypes.c_int32), ("solo_edges", ctypes.c_int32),
                ("block_units", ctypes.c_int32), ("small_n", ctypes.c_int32),
                ("wg", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SSSPError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, sssp_strerror(status), status))


_lib = None


def lib():
    """Load libsssp.so; fails loudly if the HIP library was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsssp.so is not built; run paper_1812_10499_amd.build.build() "
                              "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
        L.sssp_build_csr_bytes.argtypes = [i32, i32, ctypes.c_int, ctypes.c_int]
        L.sssp_build_csr_bytes.restype = ctypes.c_size_t
        L.sssp_build_csr.argtypes = [i32, i32, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp,
                                     ctypes.c_size_t, ctypes.POINTER(Csr), vp, vp]
        L.sssp_build_csr.restype = ctypes.c_int
        L.sssp_set_weights.argtypes = [ctypes.POINTER(Csr), vp, vp]
        L.sssp_set_weights.restype = ctypes.c_int
        L.sssp_permute_edges.argtypes = [vp, ctypes.c_int64, vp, vp, i32, vp]
        L.sssp_permute_edges.restype = ctypes.c_int
        L.sssp_solve.argtypes = [ctypes.POINTER(Csr), i32, vp, vp, ctypes.POINTER(Stats), vp]
        L.sssp_solve.restype = ctypes.c_int
        L.sssp_solve_noalloc.argtypes = [ctypes.POINTER(Csr), i32, vp, vp,
                                         ctypes.POINTER(Stats), vp]
        L.sssp_solve_noalloc.restype = ctypes.c_int
        L.sssp_solve_target.argtypes = [ctypes.POINTER(Csr), i32, i32, vp,
                                        ctypes.POINTER(Stats), vp]
        L.sssp_solve_target.restype = ctypes.c_int
        L.sssp_solve_batch.argtypes = [ctypes.POINTER(Csr), i32, vp, vp, i32, vp, vp,
                                       ctypes.POINTER(Stats), vp]
        L.sssp_solve_batch.restype = ctypes.c_int
        L.sssp_backward.argtypes = [ctypes.POINTER(Csr), i32, vp, vp, i32, vp, vp, vp, vp]
        L.sssp_backward.restype = ctypes.c_int
        L.sssp_set_launch.argtypes = [ctypes.POINTER(Launch)]
        L.sssp_set_launch.restype = ctypes.c_int
        L.sssp_plan_create.argtypes = [ctypes.POINTER(Csr), i32, vp, vp, i32, ctypes.c_int, vp,
                                       vp, i32, ctypes.POINTER(Launch),
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.sssp_plan_create.restype = ctypes.c_int
        L.sssp_plan_run.argtypes = [vp, vp]
        L.sssp_plan_run.restype = ctypes.c_int
        L.sssp_plan_stats.argtypes = [vp, ctypes.POINTER(Stats), vp]
        L.sssp_plan_stats.restype = ctypes.c_int
        L.sssp_plan_destroy.argtypes = [vp]
        L.sssp_plan_destroy.restype = ctypes.c_int
        L.sssp_autotune.argtypes = [ctypes.POINTER(Csr), i32, vp, vp, i32, ctypes.c_int, vp, vp,
                                    i32, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_double),
                                    vp]
        L.sssp_autotune.restype = ctypes.c_int
        L.sssp_release_workspace.argtypes = []
        L.sssp_release_workspace.restype = ctypes.c_int
        L.sssp_profile_enable.argtypes = [ctypes.c_int]
        L.sssp_profile_enable.restype = ctypes.c_int
        L.sssp_profile_read.argtypes = [ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
        L.sssp_profile_read.restype = ctypes.c_int
        L.sssp_policy_of.argtypes = [ctypes.POINTER(Csr), ctypes.POINTER(Policy)]
        L.sssp_policy_of.restype = ctypes.c_int
        L.sssp_check.argtypes = [vp]
        L.sssp_check.restype = ctypes.c_int
        L.sssp_set_round_limit.argtypes = [i32]
        L.sssp_set_round_limit.restype = ctypes.c_int
        L.sssp_strerror.argtypes = [ctypes.c_int]
        L.sssp_strerror.restype = ctypes.c_char_p
        del i64p
        _lib = L
    return _lib


def _release_at_exit():
    """Frees the library's device resources before the process ends, while
    the HIP runtime is still up: live plans, then the workspace and events."""
    if _lib is None:
        return
    try:
        from . import graph
        graph.close_plans()
        _lib.sssp_release_workspace()
    except Exception:
        pass


atexit.register(_release_at_exit)


def _check(status: int, where: str):
    if status != SSSP_OK:
        raise SSSPError(status, where)


def _arr(ctype, values):
    values = [int(v) for v in values]
    return (ctype * len(values))(*values)


def sssp_strerror(status: int) -> str:
    return lib().sssp_strerror(int(status)).decode()


def sssp_build_csr_bytes(n: int, m: int, dtype: int, order: int) -> int:
    return int(lib().sssp_build_csr_bytes(n, m, dtype, order))


def sssp_build_csr(n, m, dtype, order, src, dst, w, buffer, buffer_bytes, out: Csr, perm,
                   stream):
    _check(lib().sssp_build_csr(n, m, dtype, order, src, dst, w, buffer, buffer_bytes,
                                ctypes.byref(out), perm, stream), "sssp_build_csr")


def sssp_set_weights(g: Csr, w, stream):
    _check(lib().sssp_set_weights(ctypes.byref(g), w, stream), "sssp_set_weights")


def sssp_permute_edges(perm, m, src, dst, to_coo, stream):
    _check(lib().sssp_permute_edges(perm, m, src, dst, 1 if to_coo else 0, stream),
           "sssp_permute_edges")


def sssp_solve(g: Csr, source, cost, pred, stats, stream):
    _check(lib().sssp_solve(ctypes.byref(g), source, cost, pred,
                            ctypes.byref(stats) if stats is not None else None, stream),
           "sssp_solve")


def sssp_solve_noalloc(g: Csr, source, cost, pred, stats, stream):
    _check(lib().sssp_solve_noalloc(ctypes.byref(g), source, cost, pred,
                                    ctypes.byref(stats) if stats is not None else None, stream),
           "sssp_solve_noalloc")


def sssp_solve_target(g: Csr, source, target, cost, stats, stream):
    _check(lib().sssp_solve_target(ctypes.byref(g), source, target, cost,
                                   ctypes.byref(stats) if stats is not None else None, stream),
           "sssp_solve_target")


def sssp_solve_batch(graphs, inst_graph, inst_source, cost, pred, stats, stream):
    ga = (Csr * len(graphs))(*graphs)
    ig = _arr(ctypes.c_int32, inst_graph)
    isrc = _arr(ctypes.c_int32, inst_source)
    _check(lib().sssp_solve_batch(ga, len(graphs), ctypes.cast(ig, ctypes.c_void_p),
                                  ctypes.cast(isrc, ctypes.c_void_p), len(ig), cost, pred,
                                  stats, stream), "sssp_solve_batch")


def sssp_backward(graphs, inst_graph, inst_source, pred, grad_cost, grad_w, stream):
    ga = (Csr * len(graphs))(*graphs)
    ig = _arr(ctypes.c_int32, inst_graph)
    isrc = _arr(ctypes.c_int32, inst_source)
    _check(lib().sssp_backward(ga, len(graphs), ctypes.cast(ig, ctypes.c_void_p),
                               ctypes.cast(isrc, ctypes.c_void_p), len(ig), pred, grad_cost,
                               grad_w, stream), "sssp_backward")


def sssp_profile_enable(on: bool):
    _check(lib().sssp_profile_enable(1 if on else 0), "sssp_profile_enable")


def sssp_profile_read():
    """(timed round-kernel launches, their summed milliseconds) since the last read."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib().sssp_profile_read(ctypes.byref(n), ctypes.byref(ms)), "sssp_profile_read")
    return n.value, ms.value


def sssp_policy_of(g: Csr) -> Policy:
    p = Policy()
    _check(lib().sssp_policy_of(ctypes.byref(g), ctypes.byref(p)), "sssp_policy_of")
    return p


def sssp_check(stream):
    _check(lib().sssp_check(stream), "sssp_check")


def sssp_set_round_limit(limit: int):
    _check(lib().sssp_set_round_limit(int(limit)), "sssp_set_round_limit")


def sssp_release_workspace():
    _check(lib().sssp_release_workspace(), "sssp_release_workspace")


def sssp_set_launch(launch):
    """launch: a Launch, or None for the defaults."""
    _check(lib().sssp_set_launch(ctypes.byref(launch) if launch is not None else None),
           "sssp_set_launch")


def _batch_args(graphs, inst_graph, inst_source):
    ga = (Csr * len(graphs))(*graphs)
    ig = _arr(ctypes.c_int32, inst_graph)
    isrc = _arr(ctypes.c_int32, inst_source)
    return ga, ig, isrc


def sssp_plan_create(graphs, inst_graph, inst_source, kind, cost, pred, with_stats, launch):
    """Returns the plan handle (an int)."""
    ga, ig, isrc = _batch_args(graphs, inst_graph, inst_source)
    h = ctypes.c_void_p(0)
    _check(lib().sssp_plan_create(ga, len(graphs), ctypes.cast(ig, ctypes.c_void_p),
                                  ctypes.cast(isrc, ctypes.c_void_p), len(ig), kind, cost, pred,
                                  1 if with_stats else 0,
                                  ctypes.byref(launch) if launch is not None else None,
                                  ctypes.byref(h)), "sssp_plan_create")
    return h.value


def sssp_plan_run(plan, stream):
    _check(lib().sssp_plan_run(plan, stream), "sssp_plan_run")


def sssp_plan_stats(plan, stats, stream):
    _check(lib().sssp_plan_stats(plan, stats, stream), "sssp_plan_stats")


def sssp_plan_destroy(plan):
    _check(lib().sssp_plan_destroy(plan), "sssp_plan_destroy")


def sssp_autotune(graphs, inst_graph, inst_source, kind, cost, pred, reps, stream):
    """Returns (Launch, mean milliseconds per run under it)."""
    ga, ig, isrc = _batch_args(graphs, inst_graph, inst_source)
    best = Launch()
    ms = ctypes.c_double(0.0)
    _check(lib().sssp_autotune(ga, len(graphs), ctypes.cast(ig, ctypes.c_void_p),
                               ctypes.cast(isrc, ctypes.c_void_p), len(ig), kind, cost, pred,
                               int(reps), ctypes.byref(best), ctypes.byref(ms), stream),
           "sssp_autotune")
    return best, ms.value
