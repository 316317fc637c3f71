"""Seeded synthetic workloads (no shortest-path arithmetic).

The arrays built here feed both the CPU oracle and the GPU library, bit for
bit.  The generators themselves are in ``gen.c`` (counter-based splitmix64;
see its header for the exact streams); this module marshals them and names
the five benchmark workloads:

* ``random_workload``  -- random directed graph, n=4096, m=32768, int32
  weights uniform in [1,100], source 0 (seed 0x5EED0001).
* ``grid_workload``    -- 1024x1024 4-neighbour grid, int32 weights uniform in
  [1,1000], source at the centre (seed 0x5EED0002).
* ``rmat_workload``    -- R-MAT scale 22, edge factor 16, (a,b,c,d) =
  (.57,.19,.19,.05), relabelled, duplicates and self-loops kept, int32
  weights uniform in [1,255], source = highest out-degree vertex (seed
  0x5EED0003).
* ``batch_workload``   -- 256 random graphs, n_i uniform in [1000,200000],
  m_i = 8 n_i, float32 weights (k+1)*2^-24, random source (seed 0x5EED0004).
* ``diff_workload``    -- 512x512 grid, float32 weights 0.5 + k*2^-23 in
  [0.5,1.5], 64 distinct sources, loss coefficients g ~ N(0,1) in float32
  (seed 0x5EED0005).

Every builder takes size parameters so that tests can use scaled-down
instances of the same families.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsssp_gen.so")
_SRC = os.path.join(_HERE, "gen.c")
_lib = None

SEED_RANDOM, SEED_GRID, SEED_RMAT, SEED_BATCH, SEED_DIFF = (
    0x5EED0001, 0x5EED0002, 0x5EED0003, 0x5EED0004, 0x5EED0005)


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SRC) > os.path.getmtime(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
        _lib.gen_draw.restype = ctypes.c_uint64
        _lib.gen_draw.argtypes = [ctypes.c_uint64] * 3
        _lib.gen_uniform_below.restype = ctypes.c_uint64
        _lib.gen_uniform_below.argtypes = [ctypes.c_uint64] * 4
        _lib.gen_grid_edge_count.restype = ctypes.c_int64
        _lib.gen_max_out_degree_vertex.restype = ctypes.c_int32
        _lib.gen_distinct_vertices.restype = ctypes.c_int
        for name in ("gen_random_edges", "gen_grid_edges", "gen_rmat_edges", "gen_weights_int",
                     "gen_weights_unit24", "gen_weights_half23", "gen_normal_f32"):
            getattr(_lib, name).restype = None
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


U64 = ctypes.c_uint64


def draw(seed, stream, ctr) -> int:
    return int(_L().gen_draw(seed, stream, ctr))


def uniform_below(seed, stream, idx, rng) -> int:
    return int(_L().gen_uniform_below(seed, stream, idx, rng))


def random_edges(seed, n, m):
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _L().gen_random_edges(U64(seed), ctypes.c_int32(n), ctypes.c_int64(m), _p(src), _p(dst))
    return src, dst


def grid_edges(rows, cols):
    m = int(_L().gen_grid_edge_count(ctypes.c_int32(rows), ctypes.c_int32(cols)))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _L().gen_grid_edges(ctypes.c_int32(rows), ctypes.c_int32(cols), _p(src), _p(dst))
    return src, dst


def rmat_edges(seed, scale, m, a=0.57, b=0.19, c=0.19, permute=True):
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    work = np.empty(1 << scale, dtype=np.int32)
    _L().gen_rmat_edges(U64(seed), ctypes.c_int32(scale), ctypes.c_int64(m), ctypes.c_double(a),
                        ctypes.c_double(b), ctypes.c_double(c), ctypes.c_int(1 if permute else 0),
                        _p(src), _p(dst), _p(work))
    return src, dst


def weights_int(seed, m, lo, hi):
    w = np.empty(m, dtype=np.int32)
    _L().gen_weights_int(U64(seed), ctypes.c_int64(m), ctypes.c_int32(lo), ctypes.c_int32(hi), _p(w))
    return w


def weights_unit24(seed, m):
    w = np.empty(m, dtype=np.float32)
    _L().gen_weights_unit24(U64(seed), ctypes.c_int64(m), _p(w))
    return w


def weights_half23(seed, m):
    w = np.empty(m, dtype=np.float32)
    _L().gen_weights_half23(U64(seed), ctypes.c_int64(m), _p(w))
    return w


def distinct_vertices(seed, n, count):
    out = np.empty(count, dtype=np.int32)
    if _L().gen_distinct_vertices(U64(seed), ctypes.c_int32(n), ctypes.c_int32(count), _p(out)):
        raise ValueError("more distinct vertices requested than exist")
    return out


def normal_f32(seed, count):
    out = np.empty(count, dtype=np.float32)
    _L().gen_normal_f32(U64(seed), ctypes.c_int64(count), _p(out))
    return out


def max_out_degree_vertex(n, src):
    src = np.ascontiguousarray(src, dtype=np.int32)
    work = np.empty(n, dtype=np.int32)
    return int(_L().gen_max_out_degree_vertex(ctypes.c_int32(n), ctypes.c_int64(len(src)),
                                              _p(src), _p(work)))


@dataclass
class Graph:
    """One COO graph plus its source(s).  w dtype is int32 or float32."""
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    w: np.ndarray
    source: int = 0
    sources: np.ndarray = field(default=None)

    @property
    def m(self) -> int:
        return int(len(self.src))


def random_workload(n=4096, m=32768, seed=SEED_RANDOM, wlo=1, whi=100) -> Graph:
    src, dst = random_edges(seed, n, m)
    return Graph("random%d_%d" % (n, m), n, src, dst, weights_int(seed, m, wlo, whi), 0)


def grid_workload(side=1024, seed=SEED_GRID, wlo=1, whi=1000) -> Graph:
    src, dst = grid_edges(side, side)
    centre = (side // 2) * side + side // 2
    return Graph("grid%dx%d" % (side, side), side * side, src, dst,
                 weights_int(seed, len(src), wlo, whi), centre)


def rmat_workload(scale=22, edge_factor=16, seed=SEED_RMAT, wlo=1, whi=255) -> Graph:
    n = 1 << scale
    m = edge_factor * n
    src, dst = rmat_edges(seed, scale, m)
    w = weights_int(seed, m, wlo, whi)
    return Graph("rmat%d_ef%d" % (scale, edge_factor), n, src, dst, w,
                 max_out_degree_vertex(n, src))


def batch_workload(count=256, nmin=1000, nmax=200000, degree=8, seed=SEED_BATCH):
    """List of Graphs, one instance each (own graph, own source)."""
    out = []
    for i in range(count):
        n = nmin + uniform_below(seed, 100, i, nmax - nmin + 1)
        gseed = draw(seed, 101, i)
        m = degree * n
        src, dst = random_edges(gseed, n, m)
        w = weights_unit24(gseed, m)
        s = uniform_below(seed, 102, i, n)
        out.append(Graph("batch%d_%d" % (count, i), n, src, dst, w, s))
    return out


def diff_workload(side=512, num_sources=64, seed=SEED_DIFF):
    """(Graph with .sources, g[num_sources, n] float32 loss coefficients)."""
    src, dst = grid_edges(side, side)
    w = weights_half23(seed, len(src))
    n = side * side
    sources = distinct_vertices(seed, n, num_sources)
    g = normal_f32(seed, num_sources * n).reshape(num_sources, n)
    gr = Graph("grid%dx%d_f32" % (side, side), n, src, dst, w, int(sources[0]), sources)
    return gr, g
