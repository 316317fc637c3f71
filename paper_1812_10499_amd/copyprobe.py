"""Calibration load for HBM traffic counters: a plain device copy of known size.

    python -m paper_1812_10499_amd.copyprobe [--mib 1024] [--reps 3]

Under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE) the elementwise copy
kernel reads and writes exactly ``mib`` MiB per dispatch; the ratio of that
size to what the counter reports scales the counters of the round kernel to
bytes.  Prints one line when done.
"""
from __future__ import annotations

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        torch.bitwise_not(src, out=dst)  # one read and one write of every element
    torch.cuda.synchronize()
    assert int(dst[12345]) == ~12345
    print("copyprobe done: %d dispatches of %d MiB read + %d MiB written"
          % (args.reps, args.mib, args.mib), flush=True)


if __name__ == "__main__":
    main()
