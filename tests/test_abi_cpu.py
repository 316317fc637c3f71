"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/sssp.h declares, and
reject host-checkable bad arguments before touching the GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sssp.h")


@pytest.fixture(scope="module")
def sp():
    import paper_1812_10499_amd as sp
    if not os.path.exists(sp.LIB_PATH):
        from paper_1812_10499_amd import build
        build.build()
    return sp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sssp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert names == sorted(["sssp_build_csr_bytes", "sssp_build_csr", "sssp_set_weights",
                            "sssp_solve", "sssp_solve_target", "sssp_solve_batch",
                            "sssp_backward", "sssp_set_launch", "sssp_plan_create",
                            "sssp_plan_run", "sssp_plan_stats", "sssp_plan_destroy",
                            "sssp_autotune",
                            "sssp_release_workspace", "sssp_strerror",
                            "sssp_profile_enable", "sssp_profile_read", "sssp_check",
                            "sssp_set_round_limit", "sssp_policy_of",
                            "sssp_solve_noalloc", "sssp_permute_edges"])


def test_library_exports_every_declared_symbol(sp):
    L = ctypes.CDLL(sp.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(sp.EXPORTS) == set(declared_functions())


def test_strerror_and_sizes(sp):
    assert sp.sssp_strerror(0) == "ok"
    for s in range(1, 9):
        assert sp.sssp_strerror(s) and sp.sssp_strerror(s) != "unknown status"
    I, A, D = sp.SSSP_ORDER_INPUT, sp.SSSP_ORDER_AUTO, sp.SSSP_ORDER_DEGREE
    assert sp.sssp_build_csr_bytes(0, 10, sp.SSSP_I32, I) == 0
    assert sp.sssp_build_csr_bytes(10, -1, sp.SSSP_I32, I) == 0
    assert sp.sssp_build_csr_bytes(10, 10, 7, I) == 0
    assert sp.sssp_build_csr_bytes(10, 10, sp.SSSP_I32, 3) == 0
    b = sp.sssp_build_csr_bytes(1000, 5000, sp.SSSP_F32, I)
    # CSR/CSC (2 offset arrays, 5 edge arrays, out_wmin) + the weight-ordered
    # in-lists of the working copy (offsets, 3 edge arrays) + 32-byte vertex records
    assert b >= 4 * (3 * 1001 + 8 * 5000 + 1000) + 32 * 1000
    # degree order adds vid, rank, out_wmin (n), offsets (n+1), 3 edge arrays
    bd = sp.sssp_build_csr_bytes(1000, 5000, sp.SSSP_F32, D)
    assert bd >= b + 4 * (3 * 1000 + 1001 + 3 * 5000)
    assert sp.sssp_build_csr_bytes(1000, 5000, sp.SSSP_F32, A) == bd


def _fake_csr(sp, n=10, m=20, dtype=0, w_max=5.0):
    c = sp.Csr()
    c.n, c.m, c.dtype, c.w_max, c.order = n, m, dtype, w_max, sp.SSSP_ORDER_INPUT
    for f in ("out_off", "out_dst", "out_w", "in_off", "in_src", "in_eid", "in_w", "out_wmin",
              "s_out_off", "s_out_dst", "s_out_w", "s_in_off", "s_in_src", "s_in_eid", "s_in_w",
              "s_out_wmin", "s_vrec", "s_in_sw", "s_out_rec", "s_vin"):
        setattr(c, f, 0x1000)  # never dereferenced: every call below fails its host checks
    return c


def _status(fn):
    try:
        fn()
    except Exception as e:  # SSSPError
        return e.status
    return 0


def test_round_limit_argument(sp):
    with pytest.raises(sp.SSSPError) as e:
        sp.sssp_set_round_limit(-1)
    assert e.value.status == sp.SSSP_ERR_ARG
    sp.sssp_set_round_limit(0)


def test_permute_argument_errors(sp):
    """Argument errors of sssp_permute_edges, returned before any GPU work;
    an empty permutation is a no-op."""
    S = sp.SSSP_ERR_ARG
    assert _status(lambda: sp.sssp_permute_edges(0x1000, -1, 0x2000, 0x3000, 0, None)) == S
    assert _status(lambda: sp.sssp_permute_edges(None, 4, 0x2000, 0x3000, 0, None)) == S
    assert _status(lambda: sp.sssp_permute_edges(0x1000, 4, None, 0x3000, 1, None)) == S
    assert _status(lambda: sp.sssp_permute_edges(0x1000, 4, 0x2000, None, 1, None)) == S
    assert _status(lambda: sp.sssp_permute_edges(0x1000, 4, 0x2000, 0x2000, 0, None)) == S
    sp.sssp_permute_edges(None, 0, None, None, 0, None)


def test_host_argument_errors(sp):
    c = _fake_csr(sp)
    S = sp.SSSP_ERR_ARG
    assert _status(lambda: sp.sssp_solve(c, -1, 0x1000, None, None, None)) == S
    assert _status(lambda: sp.sssp_solve(c, 10, 0x1000, None, None, None)) == S
    assert _status(lambda: sp.sssp_solve(c, 0, None, None, None, None)) == S
    bad = _fake_csr(sp, n=0)
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad = _fake_csr(sp, dtype=5)
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad = _fake_csr(sp)
    bad.in_src = None
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    # a built graph records INPUT or DEGREE; DEGREE needs the working copy
    bad = _fake_csr(sp)
    bad.order = sp.SSSP_ORDER_AUTO
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad.order = sp.SSSP_ORDER_DEGREE  # without vid, rank, s_out_eid
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad = _fake_csr(sp)
    bad.s_in_w = None  # the in-list copy is required in every order
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    # so are the paired in-lists, the out-edge records and the in-records
    for f in ("s_in_sw", "s_out_rec", "s_vin"):
        bad = _fake_csr(sp)
        setattr(bad, f, None)
        assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S, f
    # an edgeless graph needs no per-edge arrays, but still its in-records
    bad = _fake_csr(sp, m=0)
    bad.s_in_sw = bad.s_out_rec = None
    bad.s_vin = None
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad = _fake_csr(sp)
    bad.scope = 3  # not an sssp_scope
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    # the bucket width is a key in [0, INF]: negative, or a float32 NaN
    bad = _fake_csr(sp)
    bad.delta = -1
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    bad = _fake_csr(sp, dtype=1)
    bad.delta = 0x7fc00000
    assert _status(lambda: sp.sssp_solve(bad, 0, 0x1000, None, None, None)) == S
    # single-target solve: the target must be a vertex
    assert _status(lambda: sp.sssp_solve_target(c, 0, -1, 0x1000, None, None)) == S
    assert _status(lambda: sp.sssp_solve_target(c, 0, 10, 0x1000, None, None)) == S
    # int32 overflow precondition: (n-1) * w_max >= INT32_MAX
    big = _fake_csr(sp, n=1 << 22, w_max=1000.0)
    assert _status(lambda: sp.sssp_solve(big, 0, 0x1000, None, None, None)) == \
        sp._abi.SSSP_ERR_OVERFLOW
    ok_f32 = _fake_csr(sp, n=1 << 22, w_max=1000.0, dtype=1)
    # float32 graphs have no overflow precondition: this fails only on the
    # source range check
    assert _status(lambda: sp.sssp_solve(ok_f32, -5, 0x1000, None, None, None)) == S
    # batch: instance graph / source out of range, mixed dtypes
    assert _status(lambda: sp.sssp_solve_batch([c], [1], [0], 0x1000, None, None, None)) == S
    assert _status(lambda: sp.sssp_solve_batch([c], [0], [10], 0x1000, None, None, None)) == S
    f = _fake_csr(sp, dtype=1)
    assert _status(lambda: sp.sssp_solve_batch([c, f], [0, 1], [0, 0], 0x1000, None, None,
                                               None)) == S
    assert _status(lambda: sp.sssp_backward([c], [0], [10], 0x1000, 0x1000, 0x1000, None)) == S
    assert _status(lambda: sp.sssp_backward([c], [0], [0], None, 0x1000, 0x1000, None)) == S
    # plans and the autotuner check their batch like sssp_solve_batch
    B, Q = sp.SSSP_PLAN_BATCH, sp.SSSP_PLAN_SEQUENCE
    assert _status(lambda: sp.sssp_plan_create([c], [1], [0], B, 0x1000, None, 0, None)) == S
    assert _status(lambda: sp.sssp_plan_create([c], [0], [10], Q, 0x1000, None, 0, None)) == S
    assert _status(lambda: sp.sssp_plan_create([c], [0], [0], 2, 0x1000, None, 0, None)) == S
    assert _status(lambda: sp.sssp_plan_create([c], [0], [0], B, None, None, 0, None)) == S
    assert _status(lambda: sp.sssp_plan_create([c, f], [0, 1], [0, 0], B, 0x1000, None, 0,
                                               None)) == S
    assert _status(lambda: sp.sssp_plan_run(None, None)) == S
    assert _status(lambda: sp.sssp_plan_stats(None, sp.Stats(), None)) == S
    assert _status(lambda: sp.sssp_plan_destroy(None)) == 0
    assert _status(lambda: sp.sssp_autotune([c], [0], [0], B, 0x1000, None, 0, None)) == S
    assert _status(lambda: sp.sssp_autotune([c], [0], [0], B, 0x1000, None, 101, None)) == S
    assert _status(lambda: sp.sssp_autotune([c], [0], [11], B, 0x1000, None, 2, None)) == S
    # builder: bad sizes, missing pointers, short buffer
    out = sp.Csr()
    I = sp.SSSP_ORDER_INPUT
    assert _status(lambda: sp.sssp_build_csr(0, 5, 0, I, 0x1000, 0x1000, 0x1000, 0x1000,
                                             1 << 20, out, None, None)) == S
    assert _status(lambda: sp.sssp_build_csr(5, 5, 0, I, None, 0x1000, 0x1000, 0x1000,
                                             1 << 20, out, None, None)) == S
    assert _status(lambda: sp.sssp_build_csr(5, 5, 0, I, 0x1000, 0x1000, 0x1000, 0x1000, 16,
                                             out, None, None)) == S
    assert _status(lambda: sp.sssp_build_csr(5, 5, 0, 9, 0x1000, 0x1000, 0x1000, 0x1000,
                                             1 << 20, out, None, None)) == S
    # a buffer large enough for the input order but not for the working copy
    small = sp.sssp_build_csr_bytes(5, 5, 0, I)
    assert _status(lambda: sp.sssp_build_csr(5, 5, 0, sp.SSSP_ORDER_DEGREE, 0x1000, 0x1000,
                                             0x1000, 0x1000, small, out, None, None)) == S


def test_probe_library_exports(sp):
    """The measurement library (access rates and barrier costs the bench's
    latency bound uses) loads and exports its entry points."""
    from paper_1812_10499_amd.build import PROBE_SO
    if not os.path.exists(PROBE_SO):
        from paper_1812_10499_amd import build
        build.build()
    L = ctypes.CDLL(PROBE_SO)
    for name in ("probe_gather", "probe_gather_atomic", "probe_gather_atomic_every",
                 "probe_gather_part", "probe_chase", "probe_sync", "probe_grid_sync",
                 "probe_cu_access"):
        assert hasattr(L, name), name
