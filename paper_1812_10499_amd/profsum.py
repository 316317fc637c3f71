"""Summaries of rocprofv3 result databases (the SQLite ``*_results.db`` files).

    python -m paper_1812_10499_amd.profsum stats DB --title T --cmd C --out FILE.md
        per-kernel dispatch count and durations from a --kernel-trace run

    python -m paper_1812_10499_amd.profsum traffic --fetch DB --write DB
        --copy-fetch DB --copy-write DB --copy-mib N --kernel NAME
        --title T --cmd C --out FILE.md --json FILE.json
        per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of one kernel, scaled to
        bytes by the same counters read on a plain copy of known size

    python -m paper_1812_10499_amd.profsum counters DB [DB ...] --kernel NAME
        --title T --cmd C --out FILE.md
        per-dispatch means of every counter the --pmc runs took on one kernel,
        and the ratios they give (wait and issue shares of wave time, memory
        latencies, L2 hit rate, LDS bank conflicts)

The JSON carries the hash of the round kernel's sources so that a reader can
tell whether the counters still describe the built kernel.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import statistics

from .build import kernel_source_hash


def _short(name: str) -> str:
    name = name.replace(".kd", "")
    for key in ("small_rounds_kernel", "wg_rounds_kernel", "bw_wg_kernel", "rounds_kernel",
                "emit_kernel", "pred_degen_kernel", "init_fill_kernel",
                "init_seed_kernel", "bw_levels_kernel", "bw_grad_kernel", "bw_init_kernel",
                "bitwise_not"):
        if key in name:
            tmpl = ""
            if "KeyI32" in name:
                tmpl = "<i32%s>" % (", batch" if "Lb1E" in name else "")
            elif "KeyF32" in name:
                tmpl = "<f32%s>" % (", batch" if "Lb1E" in name else "")
            return key + tmpl
    return name[:60]


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    by = {}
    for name, dur in rows:
        by.setdefault(_short(name), []).append(dur / 1000.0)  # ns -> us
    total = sum(sum(v) for v in by.values())
    out = []
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append(dict(kernel=k, calls=len(v), total_us=sum(v), avg_us=statistics.mean(v),
                        min_us=min(v), max_us=max(v), pct=100.0 * sum(v) / total))
    return out


def counter_per_dispatch(db: str, counter: str, kernel: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                       "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    vals = [v for name, _, v in rows if kernel in name]
    if not vals:
        raise SystemExit("no %s dispatches of %s in %s" % (counter, kernel, db))
    return vals


def cmd_stats(a):
    st = kernel_stats(a.db)
    lines = ["# %s" % a.title, "", "Command (from the repository root):", "", "```",
             a.cmd, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in st:
        lines.append("| %s | %d | %.3f | %.1f | %.1f | %.1f | %.1f |" % (
            r["kernel"], r["calls"], r["total_us"] / 1e3, r["avg_us"], r["min_us"], r["max_us"],
            r["pct"]))
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_traffic(a):
    fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    write = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    cf = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", "bitwise_not")
    cw = counter_per_dispatch(a.copy_write, "WRITE_SIZE", "bitwise_not")
    copy_bytes = a.copy_mib * float(1 << 20)
    # the counters report KiB; the copy reads and writes copy_bytes each
    f_factor = copy_bytes / (statistics.mean(cf) * 1024.0)
    w_factor = copy_bytes / (statistics.mean(cw) * 1024.0)
    fb = statistics.mean(fetch) * 1024.0 * f_factor
    wb = statistics.mean(write) * 1024.0 * w_factor
    d = dict(kernel=a.kernel, source_sha=kernel_source_hash(),
             fetch_kib_per_dispatch=statistics.mean(fetch),
             write_kib_per_dispatch=statistics.mean(write), dispatches=[len(fetch), len(write)],
             copy_mib=a.copy_mib, copy_fetch_kib=statistics.mean(cf),
             copy_write_kib=statistics.mean(cw), fetch_factor=f_factor, write_factor=w_factor,
             hbm_read_bytes_per_launch=fb, hbm_write_bytes_per_launch=wb,
             hbm_bytes_per_launch=fb + wb)
    json.dump(d, open(a.json, "w"), indent=1)
    lines = ["# %s" % a.title, "", "Commands (from the repository root):", "", "```", a.cmd,
             "```", "",
             "FETCH_SIZE and WRITE_SIZE count the L2's requests to the fabric. The Infinity",
             "Cache can serve them before HBM does, so the scaled figures bound HBM traffic",
             "from above.", "",
             "| quantity | value |", "|---|---|",
             "| %s dispatches (FETCH, WRITE runs) | %d, %d |" % (a.kernel, len(fetch), len(write)),
             "| FETCH_SIZE per dispatch (KiB) | %.1f |" % d["fetch_kib_per_dispatch"],
             "| WRITE_SIZE per dispatch (KiB) | %.1f |" % d["write_kib_per_dispatch"],
             "| copy probe: %d MiB read + written; FETCH_SIZE, WRITE_SIZE (KiB) | %.1f, %.1f |"
             % (a.copy_mib, d["copy_fetch_kib"], d["copy_write_kib"]),
             "| scale factors (bytes per counted KiB / 1024): fetch, write | %.4f, %.4f |"
             % (f_factor, w_factor),
             "| HBM bytes per launch: read, written, total (GB) | %.3f, %.3f, %.3f |"
             % (fb / 1e9, wb / 1e9, (fb + wb) / 1e9),
             "| round-kernel source hash | %s |" % d["source_sha"]]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(db: str, kernel: str):
    """{counter: mean value per dispatch} and the mean dispatch duration (ns)
    of the dispatches of `kernel` in one --pmc database."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, counter_name, sum(value), "
                       "max(duration) from counters_collection "
                       "group by dispatch_id, counter_name").fetchall()
    vals, durs = {}, {}
    for name, did, counter, v, dur in rows:
        if _short(name) != kernel and not _short(name).startswith(kernel + "<"):
            continue
        vals.setdefault(counter, []).append(v)
        durs[did] = dur
    if not vals:
        raise SystemExit("no dispatches of %s in %s" % (kernel, db))
    return ({c: statistics.mean(v) for c, v in vals.items()}, len(durs),
            statistics.mean(durs.values()))


def cmd_counters(a):
    c, lines_in = {}, []
    for db in a.db:
        vals, n, dur = _per_dispatch(db, a.kernel)
        lines_in.append("| %s | %d | %.1f |" % (", ".join(sorted(vals)), n, dur / 1e3))
        c.update(vals)
        c.setdefault("_dur_ns", []).append(dur)
    dur_s = statistics.mean(c.pop("_dur_ns")) / 1e9

    def ratio(num, den):
        if num in c and den in c and c[den]:
            return "%.3f" % (c[num] / c[den])
        return "—"

    def rate(num):
        return "%.3g" % (c[num] / dur_s) if num in c else "—"

    derived = [
        ("waiting share of wave time (SQ_WAIT_ANY / SQ_WAVE_CYCLES)",
         ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES")),
        ("issuing share of wave time (SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES)",
         ratio("SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES")),
        ("waiting for an instruction to issue (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES)",
         ratio("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")),
        ("mean L1-to-L2 read latency, cycles (TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ)",
         ratio("TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum")),
        ("L1-to-L2 read requests per second", rate("TCP_TCC_READ_REQ_sum")),
        ("L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS))",
         "%.3f" % (c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"]))
         if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c else "—"),
        ("share of L2-to-fabric reads that went to DRAM (TCC_EA0_RDREQ_DRAM / TCC_EA0_RDREQ)",
         ratio("TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_RDREQ_sum")),
        ("LDS bank-conflict cycles per LDS-active cycle (SQ_LDS_BANK_CONFLICT / "
         "SQ_ACTIVE_INST_LDS)", ratio("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS")),
        ("waiting on LDS share of wave time (SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES)",
         ratio("SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES")),
    ]
    lines = ["# %s" % a.title, "", "Commands (from the repository root):", "", "```", a.cmd,
             "```", "",
             "SQ cycle counters count quad-cycles (4 clocks) per wave, so their ratios are",
             "shares of wave time. Each run took one group of counters; every pass ran the",
             "same bench command. TCC_EA0_RDREQ_DRAM counts every L2-to-fabric read, whether",
             "the Infinity Cache or HBM then serves it.", "",
             "| counters of the run | dispatches | mean duration (µs) |", "|---|---|---|"]
    lines += lines_in
    lines += ["", "| counter | per dispatch |", "|---|---|"]
    lines += ["| %s | %.4g |" % (k, v) for k, v in sorted(c.items())]
    lines += ["", "| derived | value |", "|---|---|"]
    lines += ["| %s | %s |" % kv for kv in derived]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--kernel", "--title",
              "--cmd", "--out", "--json"):
        t.add_argument(k, required=True)
    t.add_argument("--copy-mib", type=int, default=1024)
    c = sub.add_parser("counters")
    c.add_argument("db", nargs="+")
    for k in ("--kernel", "--title", "--cmd", "--out"):
        c.add_argument(k, required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
