"""Compile the gfx950 HIP library libsssp.so in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SO = os.path.join(PKG, "libsssp.so")
SOURCES = ["api.hip", "solve.hip", "small.hip", "wg.hip", "pred.hip", "build_csr.hip",
           "backward.hip"]
HEADERS = ["sssp_dev.h", "sssp_kernels.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the process may run on PyTorch's bundled HIP runtime; v5 code objects
    # load on every ROCm runtime this package meets
    "-mcode-object-version=5",
    # packed fp32 instructions stay off (the compiler would otherwise form
    # v_pk_* ops from float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def kernel_source_hash() -> str:
    """Hash of the round kernel's sources (identifies which kernel a set of
    profiler counters describes)."""
    h = hashlib.sha256()
    for f in ("solve.hip", "sssp_dev.h", "sssp_kernels.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PROBE_SO = os.path.join(PKG, "libsssp_probe.so")


def _hipcc(out: str, srcs, verbose: bool):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp] \
        + list(srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Always recompiles (the caller asked for a build): the library and the
    measurement probes (libsssp_probe.so, csrc/probe.hip)."""
    _hipcc(SO, sources(), verbose)
    _hipcc(PROBE_SO, [os.path.join(CSRC, "probe.hip")], verbose)
    return SO


if __name__ == "__main__":
    build(verbose=True)
