"""Per-round, per-phase breakdown of one solve of the persistent round kernel.

    python -m paper_1812_10499_amd.tracesum [--workload rmat22] --out FILE.md

Runs the workload's solve once untraced (for its kernel time) and once with
the library's round trace switched on (the SSSP_TRACE environment variable:
block 0 stamps the device clock, 100 MHz, at each phase start, barrier
arrival and barrier release, and every block stamps its phase end), then
writes a Markdown table: per round and phase, the list sizes, the active
blocks, block 0's work time and barrier wait, and the spread of the blocks'
phase ends (the last block's end minus the first's: the imbalance).  The
trace itself costs a few stores per block and phase.
"""
from __future__ import annotations

import argparse
import csv
import os
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TICK_US = 0.01  # device wall clock: 100 MHz


def _read_trace(path):
    with open(path) as fh:
        rows = [r for r in csv.DictReader(fh)]
    blk = {}
    if os.path.exists(path + ".blk"):
        with open(path + ".blk") as fh:
            for line in fh:
                r, ph, b, end, win, first, units, mid = (int(x) for x in line.split(","))
                if end:
                    blk.setdefault((r, ph), []).append((end, mid))
    return rows, blk


def _blocks(recs, start):
    """Mean over the blocks that ran a phase of the time to the end of their
    list windows and from there to their phase end, and max minus mean of
    the phase ends: what a perfect balance of the phase would save."""
    if not recs:
        return "-"
    ends = [(e - start) * TICK_US for e, _ in recs]
    mids = [(m - start) * TICK_US for _, m in recs]
    mean_end = sum(ends) / len(ends)
    mean_mid = sum(mids) / len(mids)
    return "%.1f / %.1f / %.1f" % (mean_mid, mean_end - mean_mid, max(ends) - mean_end)


def summarize(rows, blk, kernel_ms, title, cmd):
    out = ["# %s" % title, "", "Command (from the repository root):", "", "```", cmd, "```", "",
           "Untraced round-kernel time: %.3f ms (mean of the timed launches)." % kernel_ms, "",
           "Columns: F = relax items (newly fixed), EF = their out-edges; O = open items, EO = "
           "their useful in-edges (weight prefix); L = live undiscovered vertices (scope ALL); "
           "act = active blocks (relax/bound); work = block 0 from phase start to barrier "
           "arrival; wait = block 0 at the barrier; spread = last minus first block's phase "
           "end (blocks that ran the phase). The blocks columns are means over the blocks that "
           "ran the phase: time in list windows / time after them (relax: the flush of first "
           "discoveries with their in-edge counts; bound: the list flushes and the live pass) / "
           "the last block's phase end minus the mean (what perfect balance would save). Times "
           "in microseconds.", "",
           "| round | F | EF | O | EO | L | act | relax work | relax wait | relax spread | "
           "relax blocks | bound work | bound wait | bound spread | bound blocks |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    tot = dict(rw=0.0, rwa=0.0, bw=0.0, bwa=0.0)
    t_first = t_last = None
    for r in rows:
        rd = int(r["round"])
        st, ar, er = int(r["start"]), int(r["arr_relax"]), int(r["end_relax"])
        af, ef = int(r["arr_fused"]), int(r["end_fused"])
        mode = int(r["mode"])
        act_r, act_b = mode & 0xffff, (mode >> 16) & 0xffff
        rw = (ar - st) * TICK_US
        rwa = (er - ar) * TICK_US
        bw = (af - er) * TICK_US if af else 0.0
        bwa = (ef - af) * TICK_US if af else 0.0
        t_first = st if t_first is None else t_first
        t_last = max(ef, er)
        sp, bk = [], []
        for ph in (0, 1):
            recs = blk.get((rd, ph))
            ends = [e for e, _ in recs] if recs else None
            sp.append("%.1f" % ((max(ends) - min(ends)) * TICK_US) if ends and len(ends) > 1
                      else "-")
            bk.append(_blocks(recs, st if ph == 0 else er))
        tot["rw"] += rw
        tot["rwa"] += rwa
        tot["bw"] += bw
        tot["bwa"] += bwa
        out.append("| %d | %s | %s | %s | %s | %s | %d/%d | %.1f | %.1f | %s | %s | %.1f | %.1f | "
                   "%s | %s |"
                   % (rd, r["nf"], r["ef"], r["no"], r["eo"], r["nl"], act_r, act_b, rw, rwa,
                      sp[0], bk[0], bw, bwa, sp[1], bk[1]))
    span = (t_last - t_first) * TICK_US if t_first is not None else 0.0
    out += ["", "Totals over %d rounds (block 0): relax work %.1f us, relax barrier wait %.1f us,"
            " bound work %.1f us, bound barrier wait %.1f us; first phase start to last "
            "release %.1f us." % (len(rows), tot["rw"], tot["rwa"], tot["bw"], tot["bwa"], span),
            ""]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    import gen
    import paper_1812_10499_amd as sp

    if args.workload == "rmat22":
        g = gen.rmat_workload()
    elif args.workload.startswith("rmat"):
        g = gen.rmat_workload(scale=int(args.workload[4:]))
    elif args.workload == "grid1024":
        g = gen.grid_workload()
    else:
        raise SystemExit("unknown workload %s" % args.workload)
    torch.cuda.set_device(0)
    G = sp.Graph(g.n, g.src, g.dst, g.w, device="cuda:0")
    cost = torch.empty(g.n, dtype=G.value_dtype, device="cuda:0")
    pred = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(2):
        sp.sssp_solve(G.csr, g.source, cost.data_ptr(), pred.data_ptr(), None, stream)
    torch.cuda.synchronize()
    sp.sssp_profile_enable(True)
    sp.sssp_profile_read()
    for _ in range(args.reps):
        sp.sssp_solve(G.csr, g.source, cost.data_ptr(), pred.data_ptr(), None, stream)
    n, ms = sp.sssp_profile_read()
    sp.sssp_profile_enable(False)
    kernel_ms = ms / max(n, 1)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "trace.csv")
        os.environ["SSSP_TRACE"] = path
        try:
            sp.sssp_solve(G.csr, g.source, cost.data_ptr(), pred.data_ptr(), None, stream)
            torch.cuda.synchronize()
        finally:
            del os.environ["SSSP_TRACE"]
        rows, blk = _read_trace(path)
    sp.check()
    title = "Round trace: %s on %s (n=%d, m=%d), kernel %s" % (
        "sssp_solve", g.name, g.n, g.m, G.kernel)
    cmd = "python -m paper_1812_10499_amd.tracesum --workload %s --out %s" % (args.workload,
                                                                              args.out)
    text = summarize(rows, blk, kernel_ms, title, cmd)
    with open(args.out, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
