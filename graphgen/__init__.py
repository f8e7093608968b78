"""Seeded synthetic graph generators (inputs only).

This module holds none of the community-detection arithmetic.  It builds the
symmetric CSR graphs that both the oracle and the GPU library consume:

* ``sbm``       stochastic block model / planted partition (contiguous blocks)
* ``rmat``      R-MAT (Chakrabarti, Zhan & Faloutsos 2004), symmetrised, loops and
                duplicates removed, optional integer weights in [1, 100]
* ``rmat_gpu``  the same R-MAT graph built directly in device memory
* small closed-form families used by the pins: cliques, rings of cliques,
  disjoint edges, and random weighted graphs with self-loops.

CSR convention: ``off`` int64[n+1], ``col`` int32[nnz] with each row strictly
ascending, ``w`` int32[nnz] or ``None`` (unit weights).  Every undirected
non-loop edge {u,v} is stored as (u,v,w) and (v,u,w); a self-loop (u,u,w) is
stored once with its own weight.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_CPU_SO = os.path.join(_HERE, "libgraphgen.so")
_GPU_SO = os.path.join(_HERE, "libgraphgen_gpu.so")

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("off", ctypes.POINTER(ctypes.c_int64)), ("col", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_int32))]


@dataclass
class Graph:
    """Host CSR graph."""
    off: np.ndarray
    col: np.ndarray
    w: np.ndarray | None

    @property
    def n(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def weights64(self) -> np.ndarray:
        if self.w is None:
            return np.ones(self.nnz, dtype=np.int64)
        return self.w.astype(np.int64)

    def undirected_edges(self) -> int:
        """m: undirected edges, a self-loop counted once."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.off))
        loops = int(np.count_nonzero(rows == self.col))
        return (self.nnz - loops) // 2 + loops


def build(force: bool = True) -> None:
    """Compile the host generator (gcc) and the device generator (hipcc, gfx950)."""
    if force or not os.path.exists(_CPU_SO):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               os.path.join(_HERE, "graphgen.c"), "-o", _CPU_SO, "-lm"])
    if force or not os.path.exists(_GPU_SO):
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               os.path.join(_HERE, "graphgen_gpu.hip"), "-o", _GPU_SO])


_cpu = None
_gpu = None


def _cpu_lib():
    global _cpu
    if _cpu is None:
        if not os.path.exists(_CPU_SO):
            build(force=False)
        lib = ctypes.CDLL(_CPU_SO)
        lib.gg_sbm.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64, ctypes.POINTER(_CSR)]
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_CSR)]
        lib.gg_free.argtypes = [ctypes.POINTER(_CSR)]
        lib.gg_draw_export.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_draw_export.restype = ctypes.c_uint64
        lib.gg_rmat_perm.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
        lib.gg_rmat_perm.restype = ctypes.c_uint64
        p64 = ctypes.POINTER(ctypes.c_int64)
        pd = ctypes.POINTER(ctypes.c_double)
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        lib.gg_batch_params.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        p64, p64, pd, pd, pu64]
        _cpu = lib
    return _cpu


def _take(c: _CSR) -> Graph:
    n, nnz = int(c.n), int(c.nnz)
    off = np.ctypeslib.as_array(c.off, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(c.col, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int32)
    w = None
    if bool(c.w):
        w = np.ctypeslib.as_array(c.w, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int32)
    return Graph(off, col, w)


def sbm(n: int, k: int, p_in: float, p_out: float, seed: int) -> Graph:
    """SBM with k contiguous near-equal blocks, unit weights."""
    lib = _cpu_lib()
    c = _CSR()
    if lib.gg_sbm(n, k, p_in, p_out, seed, ctypes.byref(c)) != 0:
        raise MemoryError("gg_sbm failed")
    try:
        return _take(c)
    finally:
        lib.gg_free(ctypes.byref(c))


def rmat(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = 2, weighted: bool = False) -> Graph:
    """R-MAT graph on the host (see graphgen.c for the exact recipe)."""
    lib = _cpu_lib()
    c = _CSR()
    a, b, cc, _ = abcd
    if lib.gg_rmat(scale, edge_factor, a, b, cc, seed, 1 if weighted else 0, ctypes.byref(c)) != 0:
        raise MemoryError("gg_rmat failed")
    try:
        return _take(c)
    finally:
        lib.gg_free(ctypes.byref(c))


def draw(seed: int, stream: int, counter: int) -> int:
    return int(_cpu_lib().gg_draw_export(seed, stream, counter))


def rmat_perm(x: int, scale: int, seed: int) -> int:
    return int(_cpu_lib().gg_rmat_perm(x, scale, seed))


def batch_params(seed: int, count: int, n_lo: float = 100.0, n_hi: float = 100000.0):
    """Per-graph (n, k, p_in, p_out, seed) of the SBM batch."""
    lib = _cpu_lib()
    n = np.zeros(count, np.int64); k = np.zeros(count, np.int64)
    pin = np.zeros(count, np.float64); pout = np.zeros(count, np.float64); gs = np.zeros(count, np.uint64)
    lib.gg_batch_params(seed, count, n_lo, n_hi, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        pin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        pout.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        gs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return n, k, pin, pout, gs


def serve_params(seed: int, count: int, rate: float, scale_lo: int = 12, scale_hi: int = 22):
    """Requests of the served workload: Poisson arrivals at `rate` per second
    (exponential gaps), R-MAT scale uniform in [scale_lo, scale_hi] and a
    per-request graph seed, all from counter-based draws of `seed`.
    Returns (arrival times in s, scales, graph seeds)."""
    arrivals = np.zeros(count, np.float64)
    scales = np.zeros(count, np.int64)
    seeds = np.zeros(count, np.uint64)
    t = 0.0
    for i in range(count):
        u = ((draw(seed, 2, i) >> 11) + 1) * (1.0 / 9007199254740993.0)   # (0, 1]
        t += -np.log(u) / rate
        arrivals[i] = t
        scales[i] = scale_lo + draw(seed, 1, i) % (scale_hi - scale_lo + 1)
        seeds[i] = draw(seed, 3, i) & 0xFFFFFFFF
    return arrivals, scales, seeds


def sbm_batch(seed: int, count: int, n_lo: float = 100.0, n_hi: float = 100000.0) -> list[Graph]:
    n, k, pin, pout, gs = batch_params(seed, count, n_lo, n_hi)
    return [sbm(int(n[i]), int(k[i]), float(pin[i]), float(pout[i]), int(gs[i])) for i in range(count)]


# ---------------------------------------------------------------- named workloads
def planted_partition_1000(seed: int = 1) -> Graph:
    """n=1000, 10 blocks of 100, p_in=0.1, p_out=0.005, unit weights."""
    return sbm(1000, 10, 0.1, 0.005, seed)


def rmat20(seed: int = 2) -> Graph:
    return rmat(20, 16, RMAT_ABCD, seed, weighted=False)


# ---------------------------------------------------------------- device R-MAT
class DeviceGraph:
    """R-MAT graph held in device memory (hipMalloc'ed by the generator)."""

    def __init__(self, n, nnz, off_ptr, col_ptr, w_ptr):
        self.n, self.nnz = n, nnz
        self.off_ptr, self.col_ptr, self.w_ptr = off_ptr, col_ptr, w_ptr

    def free(self):
        lib = _gpu_lib()
        for p in (self.off_ptr, self.col_ptr, self.w_ptr):
            if p:
                lib.ggpu_free(ctypes.c_void_p(p))
        self.off_ptr = self.col_ptr = self.w_ptr = 0

    def to_host(self) -> Graph:
        lib = _gpu_lib()
        off = np.zeros(self.n + 1, np.int64)
        col = np.zeros(self.nnz, np.int32)
        lib.ggpu_copy_to_host(off.ctypes.data, ctypes.c_void_p(self.off_ptr), off.nbytes)
        lib.ggpu_copy_to_host(col.ctypes.data, ctypes.c_void_p(self.col_ptr), col.nbytes)
        w = None
        if self.w_ptr:
            w = np.zeros(self.nnz, np.int32)
            lib.ggpu_copy_to_host(w.ctypes.data, ctypes.c_void_p(self.w_ptr), w.nbytes)
        return Graph(off, col, w)

    def rows_to_host(self, rows: np.ndarray):
        """(off of the given rows, their concatenated cols, weights) copied one range at a time."""
        lib = _gpu_lib()
        off = np.zeros(self.n + 1, np.int64)
        lib.ggpu_copy_to_host(off.ctypes.data, ctypes.c_void_p(self.off_ptr), off.nbytes)
        return off


def _gpu_lib():
    global _gpu
    if _gpu is None:
        import torch  # noqa: F401  (share torch's HIP runtime, loaded first)
        if not os.path.exists(_GPU_SO):
            build(force=False)
        lib = ctypes.CDLL(_GPU_SO)
        pp64 = ctypes.POINTER(ctypes.c_void_p)
        lib.ggpu_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_uint64, ctypes.c_int, pp64, pp64, pp64]
        lib.ggpu_rmat.restype = ctypes.c_int64
        lib.ggpu_free.argtypes = [ctypes.c_void_p]
        lib.ggpu_copy_to_host.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        _gpu = lib
    return _gpu


def rmat_gpu(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = 3, weighted: bool = True) -> DeviceGraph:
    lib = _gpu_lib()
    o, c, w = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    a, b, cc, _ = abcd
    nnz = lib.ggpu_rmat(scale, edge_factor, a, b, cc, seed, 1 if weighted else 0,
                        ctypes.byref(o), ctypes.byref(c), ctypes.byref(w))
    if nnz < 0:
        raise RuntimeError("ggpu_rmat failed")
    return DeviceGraph(1 << scale, int(nnz), o.value or 0, c.value or 0, w.value or 0)


# ---------------------------------------------------------------- small families
def from_edges(n: int, edges, weights=None, loops=None) -> Graph:
    """CSR from undirected non-loop edges [(u,v)], optional weights, optional {u: w} self-loops."""
    rows, cols, ws = [], [], []
    for i, (u, v) in enumerate(edges):
        if u == v:
            raise ValueError("use loops= for self-loops")
        wt = 1 if weights is None else int(weights[i])
        rows += [u, v]; cols += [v, u]; ws += [wt, wt]
    for u, wt in (loops or {}).items():
        rows.append(u); cols.append(u); ws.append(int(wt))
    rows = np.asarray(rows, np.int64); cols = np.asarray(cols, np.int64); ws = np.asarray(ws, np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    key = rows * (n + 1) + cols
    if len(key) and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate edge")
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, rows + 1, 1)
    off = np.cumsum(off)
    unit = weights is None and not loops
    return Graph(off.astype(np.int64), cols.astype(np.int32), None if unit else ws.astype(np.int32))


def clique_edges(nodes):
    nodes = list(nodes)
    return [(nodes[i], nodes[j]) for i in range(len(nodes)) for j in range(i + 1, len(nodes))]


def disjoint_cliques(c: int, k: int) -> Graph:
    edges = []
    for b in range(c):
        edges += clique_edges(range(b * k, (b + 1) * k))
    return from_edges(c * k, edges)


def ring_of_cliques(c: int, k: int) -> Graph:
    """c cliques K_k; clique b's last node joined to clique b+1's first node (cyclically)."""
    edges = []
    for b in range(c):
        edges += clique_edges(range(b * k, (b + 1) * k))
        edges.append(((b * k + k - 1), ((b + 1) % c) * k))
    edges = [(min(u, v), max(u, v)) for u, v in edges]
    return from_edges(c * k, sorted(set(edges)))


def disjoint_edges(c: int) -> Graph:
    return from_edges(2 * c, [(2 * i, 2 * i + 1) for i in range(c)])


def random_graph(n: int, p: float, seed: int, weighted: bool = True, loops: float = 0.0, wmax: int = 9) -> Graph:
    """Erdos-Renyi-style test graph with optional weights and self-loops (numpy PCG64, seeded)."""
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.append((u, v)); ws.append(int(rng.integers(1, wmax + 1)))
    lp = {u: int(rng.integers(1, wmax + 1)) for u in range(n) if rng.random() < loops}
    if not weighted:
        ws = [1] * len(edges)
        lp = {u: 1 for u in lp}
    g = from_edges(n, edges, ws, lp)
    if g.w is None:
        g = Graph(g.off, g.col, np.ones(g.nnz, np.int32))
    return g
