"""Access rates, latencies and barrier costs of MI355X that bound the round
kernels (measurement only; csrc/probe.hip, built into libsssp_probe.so).

    python -m paper_1812_10499_amd.probe --out FILE.md

Measures, on device 0:
  * random gathers: 8-byte values from a 2^22-entry array (the size of the
    RMAT-22 key array) at uniform indices and along the RMAT-22 graph's
    out-edge heads in CSR order (the relax step's pattern), and 4-byte
    values along its in-edge tails (the bound step's pattern), with 8
    independent gathers in flight per thread;
  * the relax step's update: gather, then 64-bit atomicMin where smaller,
    and with a set share of the edges issuing the atomic (1 in 1, 4, 16,
    64);
  * gathers folded into eighths of the array, one eighth per XCD or every
    eighth from every XCD (what L2 locality per XCD would buy);
  * dependent-load latency: the 64 lanes of one wave each following a
    random cycle through arrays of 2 MB (fits a 4 MB L2), 64 MB (fits the
    256 MB Infinity Cache, not an L2) and 1 GB (HBM);
  * a block barrier pair in one 1024-thread workgroup, and the round
    kernel's grid barrier over 8, 64 and 256 cooperative blocks;
  * one CU (one 1024-thread workgroup): the cost per wave instruction of
    random 4-byte gathers over 2 MB and 64 MB, and of coalesced 4- and
    16-byte loads and stores;
  * a 1 GiB device copy for reference.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from .build import PROBE_SO
    if not os.path.exists(PROBE_SO):
        raise ImportError("libsssp_probe.so is not built; run paper_1812_10499_amd.build.build()")
    L = ctypes.CDLL(PROBE_SO)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.probe_gather.argtypes = [ctypes.c_int, vp, vp, i64, vp, ctypes.c_int, vp]
    L.probe_gather_atomic.argtypes = [vp, vp, i64, vp, ctypes.c_int, vp]
    L.probe_gather_part.argtypes = [ctypes.c_int, vp, vp, i64, vp, ctypes.c_int, ctypes.c_uint32,
                                    ctypes.c_int, ctypes.c_int, vp]
    L.probe_gather_atomic_every.argtypes = [vp, vp, i64, vp, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_uint32, vp]
    L.probe_chase.argtypes = [vp, vp, i64, vp, vp]
    L.probe_sync.argtypes = [ctypes.c_int, vp, vp]
    L.probe_grid_sync.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.probe_cu_access.argtypes = [ctypes.c_int, vp, ctypes.c_uint32, ctypes.c_int, vp, vp]
    return L


def _time_ms(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def block_barrier_us(iters: int = 20000) -> float:
    """One block barrier in a 1024-thread workgroup (with an LDS store and
    load between barriers), on the current device, in microseconds."""
    import torch
    L = _lib()
    o = torch.empty(1024, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    ms = _time_ms(torch, lambda: L.probe_sync(iters, o.data_ptr(), st))
    return ms * 1e3 / (2 * iters)


def grid_barrier_us(blocks: int, iters: int = 2000) -> float:
    """The round kernel's grid barrier over `blocks` cooperative blocks, in
    microseconds."""
    import torch
    L = _lib()
    flags = torch.zeros(4096 * 16 + 64, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    tot = 0.0
    for _ in range(3):
        flags.zero_()
        tot += _time_ms(torch, lambda: L.probe_grid_sync(flags.data_ptr(),
                                                         flags[4096 * 16:].data_ptr(), iters,
                                                         blocks, st), reps=1)
    return tot / 3 * 1e3 / iters


def dependent_load_ns(nbytes: int, steps: int = 20000, seed: int = 1) -> float:
    """One step of 64 lanes each following a random cycle through an array
    of nbytes (vector loads), in nanoseconds."""
    import numpy as np
    import torch
    L = _lib()
    n = nbytes // 4
    perm = np.random.default_rng(seed).permutation(n).astype(np.int64)
    nxt = np.empty(n, dtype=np.uint32)
    nxt[perm] = np.roll(perm, -1)
    nd = torch.from_numpy(nxt.view(np.int32)).to("cuda")
    starts = torch.from_numpy(perm[:: max(1, n // 64)][:64].astype(np.int32)).to("cuda")
    o = torch.empty(64, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    ms = _time_ms(torch, lambda: L.probe_chase(nd.data_ptr(), starts.data_ptr(), steps,
                                               o.data_ptr(), st))
    return ms * 1e6 / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    import gen
    import paper_1812_10499_amd as sp

    L = _lib()
    dev = "cuda:0"
    torch.cuda.set_device(0)
    st = torch.cuda.current_stream().cuda_stream

    def timed(fn, reps=10, pre=None):
        if pre:
            pre()
        fn()
        torch.cuda.synchronize()
        tot = 0.0
        for _ in range(reps):
            if pre:
                pre()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        return tot / reps

    def ok(rc):
        if rc != 0:
            raise RuntimeError("probe launch failed: %d" % rc)

    rows = []
    g = gen.rmat_workload()
    G = sp.Graph(g.n, g.src, g.dst, g.w, device=dev)
    S = G.solver_arrays()
    heads = S["out_dst"].contiguous()
    tails = S["in_src"].contiguous()
    N, M = g.n, g.m
    rng = np.random.default_rng(1)
    uni = torch.from_numpy(rng.integers(0, N, M).astype(np.int32)).to(dev)
    blocks = 4096
    out = torch.empty(blocks * 256, dtype=torch.int64, device=dev)
    a64 = torch.zeros(N, dtype=torch.int64, device=dev)
    a32 = torch.zeros(N, dtype=torch.int32, device=dev)
    for name, w, arr, idx in (("8-byte gather, uniform indices", 8, a64, uni),
                              ("8-byte gather, RMAT-22 out-edge heads (CSR order)", 8, a64, heads),
                              ("4-byte gather, uniform indices", 4, a32, uni),
                              ("4-byte gather, RMAT-22 in-edge tails (CSC order)", 4, a32, tails)):
        ms = timed(lambda: ok(L.probe_gather(w, arr.data_ptr(), idx.data_ptr(), M,
                                             out.data_ptr(), blocks, st)))
        rows.append((name, "%.1f G gathers/s" % (M / ms / 1e6), "%.3f ms for 2^26" % ms))
    fill = lambda: a64.fill_(-1)  # every key starts at its maximum
    t_fill = timed(fill)
    ms = timed(lambda: ok(L.probe_gather_atomic(a64.data_ptr(), heads.data_ptr(), M,
                                                out.data_ptr(), blocks, st)), pre=fill)
    rows.append(("gather + 64-bit atomicMin where smaller, RMAT-22 heads",
                 "%.1f G edges/s" % (M / ms / 1e6), "%.3f ms for 2^26" % ms))
    # the same with a set share of atomics, kept off the hubs (the relax
    # step issues one for about 7 % of its edges, nearly none into the 4096
    # heaviest vertices); the atomics' share is counted on the host
    fill_lo = lambda: a64.fill_(1 << 40)
    h = heads.cpu().numpy()
    pos = np.arange(M)
    for every, cut in ((64, 65536), (16, 65536), (8, 65536), (4, 65536), (1, 65536),
                       (16, 0)):
        share = float(((pos % every == 0) & (h >= cut)).mean())
        ms = timed(lambda: ok(L.probe_gather_atomic_every(a64.data_ptr(), heads.data_ptr(), M,
                                                          out.data_ptr(), blocks, every, cut,
                                                          st)),
                   pre=fill_lo)
        rows.append(("gather + 64-bit atomicMin on %.1f %% of the edges (1 in %d, heads >= %d)"
                     ", RMAT-22 heads" % (100 * share, every, cut),
                     "%.1f G edges/s, %.2f G atomics/s" % (M / ms / 1e6, share * M / ms / 1e6),
                     "%.3f ms for 2^26" % ms))
    del h, pos
    # L2 locality: gathers folded into eighths of the array, one eighth per
    # XCD (blocks round-robin over the XCDs) or every eighth from every XCD
    span = N // 8
    for label, div in (("one eighth per XCD", 1), ("each eighth from all XCDs", 8)):
        for name, idx in (("uniform indices", uni), ("RMAT-22 heads", heads)):
            ms = timed(lambda: ok(L.probe_gather_part(8, a64.data_ptr(), idx.data_ptr(), M,
                                                      out.data_ptr(), blocks, span, 8, div, st)))
            rows.append(("8-byte gather folded into eighths, %s, %s" % (label, name),
                         "%.1f G gathers/s" % (M / ms / 1e6), "%.3f ms for 2^26" % ms))
    del uni
    for label, nbytes in (("2 MB (L2)", 2 << 20), ("64 MB (Infinity Cache)", 64 << 20),
                          ("1 GB (HBM)", 1 << 30)):
        rows.append(("dependent load (64 lanes, vector loads), random cycle over %s" % label,
                     "%.0f ns per step" % dependent_load_ns(nbytes), "20000 steps"))
    rows.append(("block barrier (1024 threads, with an LDS store and load)",
                 "%.0f ns per barrier" % (block_barrier_us() * 1e3), "20000 pairs"))
    for nb in (8, 64, 256):
        rows.append(("grid barrier of the round kernel over %d blocks" % nb,
                     "%.2f us per barrier" % grid_barrier_us(nb), "2000 barriers"))
    # one CU: 64 iterations x 8 accesses x 16 waves
    cu_out = torch.empty(1024, dtype=torch.int32, device=dev)
    for mode, label, nbytes in ((0, "random 4-byte gather over 2 MB", 2 << 20),
                                (0, "random 4-byte gather over 64 MB", 64 << 20),
                                (1, "coalesced 4-byte load", 2 << 20),
                                (2, "coalesced 16-byte load", 2 << 20),
                                (3, "coalesced 4-byte store", 2 << 20),
                                (4, "coalesced 16-byte store", 2 << 20)):
        arr = torch.zeros(nbytes // 4, dtype=torch.int32, device=dev)
        ms = timed(lambda: ok(L.probe_cu_access(mode, arr.data_ptr(), nbytes // 4 - 1, 64,
                                                cu_out.data_ptr(), st)))
        rows.append(("one CU (1024 threads): %s" % label,
                     "%.1f ns per wave instruction" % (ms * 1e6 / (64 * 8 * 16)),
                     "8192 instructions"))
        del arr
    x = torch.empty(1 << 28, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    ms = timed(lambda: y.copy_(x))
    rows.append(("device copy 1 GiB -> 1 GiB", "%.0f GB/s (read + write)" %
                 (2 * x.numel() * 4 / ms / 1e6), "%.3f ms" % ms))
    lines = ["# Access rates, latencies and barriers on MI355X", "",
             "Command (from the repository root):", "", "```",
             "python -m paper_1812_10499_amd.probe --out %s" % args.out, "```", "",
             "Kernels: `paper_1812_10499_amd/csrc/probe.hip` (gathers: 4096 blocks of 256 "
             "threads, 8 gathers in flight per thread; mean of 10 launches).  The fill of the "
             "key array before each atomic launch (%.3f ms) is outside the timed launch." % t_fill,
             "", "| probe | rate / latency | size |", "|---|---|---|"]
    lines += ["| %s | %s | %s |" % r for r in rows]
    text = "\n".join(lines) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
