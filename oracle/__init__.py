"""The oracle: a plain single-threaded CPU reference of PLM under the
colour-class schedule (see plm_oracle.c for what it computes and where in the
paper each step comes from).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The GPU library never uses it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plm_oracle.c")
_SO = os.path.join(_HERE, "liborc.so")

MAX_LEVELS = 64
MAX_SWEEPS = 64


class _Options(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("refine", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("gamma_num", ctypes.c_int64), ("gamma_den", ctypes.c_int64)]


class _Trace(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n", ctypes.c_int64 * MAX_LEVELS), ("nnz", ctypes.c_int64 * MAX_LEVELS),
                ("colours", ctypes.c_int64 * MAX_LEVELS), ("sweeps", ctypes.c_int64 * MAX_LEVELS),
                ("communities", ctypes.c_int64 * MAX_LEVELS),
                ("moves", (ctypes.c_int64 * MAX_SWEEPS) * MAX_LEVELS),
                ("ref_sweeps", ctypes.c_int64 * MAX_LEVELS), ("ref_moves", ctypes.c_int64 * MAX_LEVELS),
                ("S", ctypes.c_int64)]


def build(force: bool = True) -> None:
    """Compile the oracle (gcc -O2; OpenMP only for the optional threads of orc_sweep_mt)."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _SO])


_lib = None


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        P64, PU64, P32 = ctypes.POINTER(i64), ctypes.POINTER(u64), ctypes.POINTER(i32)
        L.orc_splitmix64.argtypes = [u64]; L.orc_splitmix64.restype = u64
        L.orc_priority.argtypes = [u64, i32, i64]; L.orc_priority.restype = u64
        L.orc_double_diagonal.argtypes = [i64, P64, P32, P64, P64]
        L.orc_volumes.argtypes = [i64, P64, P64, P64]; L.orc_volumes.restype = i64
        L.orc_priority_order.argtypes = [i64, u64, i32, P32]
        L.orc_colour.argtypes = [i64, P64, P32, u64, i32, i32, P32]; L.orc_colour.restype = i64
        L.orc_decide.argtypes = [i64, i64, P64, P32, P64, P32, P64, P64, i64, i64, i64, P64, PU64]
        L.orc_decide.restype = i32
        L.orc_decide_many.argtypes = [i64, i64, P32, P64, P32, P64, P32, P64, P64, i64, i64, i64, P32]
        L.orc_class_step.argtypes = [i64, P64, P32, P64, P64, i64, i64, i64, P32, i32, P32, P64]
        L.orc_class_step.restype = i64
        L.orc_sweep.argtypes = [i64, P64, P32, P64, P64, i64, i64, i64, P32, i64, P32, P64]
        L.orc_sweep.restype = i64
        L.orc_sweep_mt.argtypes = [i64, P64, P32, P64, P64, i64, i64, i64, P32, i64, P32, P64, i32]
        L.orc_sweep_mt.restype = i64
        L.orc_relabel.argtypes = [i64, P32, P32]; L.orc_relabel.restype = i64
        L.orc_contract.argtypes = [i64, P64, P32, P64, P32, i64, P64, P32, P64]; L.orc_contract.restype = i64
        L.orc_modularity.argtypes = [i64, P64, P32, P64, P32, P64, PU64, P64, PU64]
        L.orc_modularity.restype = dbl
        L.orc_canonical.argtypes = [i64, P32, P32]
        L.orc_run.argtypes = [i64, P64, P32, P64, ctypes.POINTER(_Options), P32, ctypes.POINTER(dbl),
                              ctypes.POINTER(_Trace)]
        L.orc_run.restype = ctypes.c_int
        L.orc_plp_run.argtypes = [i64, P64, P32, P64, u64, i32, P32, ctypes.POINTER(dbl), P64, P32]
        L.orc_plp_run.restype = ctypes.c_int
        L.orc_epp.argtypes = [i64, P64, P32, P64, i32, i32, ctypes.POINTER(_Options), P32, ctypes.POINTER(dbl),
                              P64, P32, ctypes.POINTER(_Trace)]
        L.orc_epp.restype = ctypes.c_int
        _lib = L
    return _lib


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u128(hi: int, lo: int) -> int:
    return (int(hi) << 64) | int(lo)


# ----------------------------------------------------------------- steps
def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x))


def priority(seed: int, level: int, u: int) -> int:
    return int(lib().orc_priority(seed, level, u))


def priority_order(n: int, seed: int, level: int) -> np.ndarray:
    out = np.zeros(max(n, 1), np.int32)
    lib().orc_priority_order(n, seed, level, _p(out, ctypes.c_int32))
    return out[:n]


def double_diagonal(off, col, w=None) -> np.ndarray:
    """Entry weights with every self-loop doubled (int64); w None = unit."""
    off, col = _i64(off), _i32(col)
    n = off.shape[0] - 1
    out = np.zeros(max(col.shape[0], 1), np.int64)
    wp = None
    if w is not None:
        w = _i64(w)
        wp = _p(w, ctypes.c_int64)
    lib().orc_double_diagonal(n, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), wp, _p(out, ctypes.c_int64))
    return out[: col.shape[0]]


def volumes(off, w2):
    off, w2 = _i64(off), _i64(w2)
    n = off.shape[0] - 1
    vol = np.zeros(max(n, 1), np.int64)
    S = lib().orc_volumes(n, _p(off, ctypes.c_int64), _p(w2, ctypes.c_int64), _p(vol, ctypes.c_int64))
    return vol[:n], int(S)


def colour(off, col, seed: int = 0, level: int = 0, schedule: int = 0):
    off, col = _i64(off), _i32(col)
    n = off.shape[0] - 1
    out = np.zeros(max(n, 1), np.int32)
    C = lib().orc_colour(n, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), seed, level, schedule,
                         _p(out, ctypes.c_int32))
    return out[:n], int(C)


def decide(u, off, col, w2, zeta, volC, vol, S, gamma=(1, 1)):
    """(target or -1, exact 128-bit gain) of one node; gamma = (num, den)."""
    off, col, w2, zeta, volC, vol = _i64(off), _i32(col), _i64(w2), _i32(zeta), _i64(volC), _i64(vol)
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    x = lib().orc_decide(off.shape[0] - 1, u, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                         _p(w2, ctypes.c_int64), _p(zeta, ctypes.c_int32), _p(volC, ctypes.c_int64),
                         _p(vol, ctypes.c_int64), S, gamma[0], gamma[1], ctypes.byref(hi), ctypes.byref(lo))
    g = _u128(hi.value, lo.value)
    if g >= 1 << 127:
        g -= 1 << 128
    return int(x), g


def decide_many(nodes, off, col, w2, zeta, volC, vol, S, gamma=(1, 1)) -> np.ndarray:
    nodes = _i32(nodes)
    off, col, w2, zeta, volC, vol = _i64(off), _i32(col), _i64(w2), _i32(zeta), _i64(volC), _i64(vol)
    out = np.zeros(max(nodes.shape[0], 1), np.int32)
    lib().orc_decide_many(off.shape[0] - 1, nodes.shape[0], _p(nodes, ctypes.c_int32), _p(off, ctypes.c_int64),
                          _p(col, ctypes.c_int32), _p(w2, ctypes.c_int64), _p(zeta, ctypes.c_int32),
                          _p(volC, ctypes.c_int64), _p(vol, ctypes.c_int64), S, gamma[0], gamma[1],
                          _p(out, ctypes.c_int32))
    return out[: nodes.shape[0]]


def class_step(off, col, w2, vol, S, colours, c, zeta, volC, gamma=(1, 1)) -> int:
    """In place on zeta (int32) and volC (int64) numpy arrays."""
    off, col, w2, vol, colours = _i64(off), _i32(col), _i64(w2), _i64(vol), _i32(colours)
    assert zeta.dtype == np.int32 and volC.dtype == np.int64
    return int(lib().orc_class_step(off.shape[0] - 1, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                                    _p(w2, ctypes.c_int64), _p(vol, ctypes.c_int64), S, gamma[0], gamma[1],
                                    _p(colours, ctypes.c_int32), c, _p(zeta, ctypes.c_int32),
                                    _p(volC, ctypes.c_int64)))


def sweep(off, col, w2, vol, S, colours, ncol, zeta, volC, gamma=(1, 1)) -> int:
    """In place on zeta (int32) and volC (int64) numpy arrays."""
    off, col, w2, vol, colours = _i64(off), _i32(col), _i64(w2), _i64(vol), _i32(colours)
    assert zeta.dtype == np.int32 and volC.dtype == np.int64
    return int(lib().orc_sweep(off.shape[0] - 1, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                               _p(w2, ctypes.c_int64), _p(vol, ctypes.c_int64), S, gamma[0], gamma[1],
                               _p(colours, ctypes.c_int32),
                               ncol, _p(zeta, ctypes.c_int32), _p(volC, ctypes.c_int64)))


def sweep_mt(off, col, w2, vol, S, colours, ncol, zeta, volC, threads: int, gamma=(1, 1)) -> int:
    """sweep() with each class's decisions spread over `threads` threads (same result)."""
    off, col, w2, vol, colours = _i64(off), _i32(col), _i64(w2), _i64(vol), _i32(colours)
    assert zeta.dtype == np.int32 and volC.dtype == np.int64
    return int(lib().orc_sweep_mt(off.shape[0] - 1, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                                  _p(w2, ctypes.c_int64), _p(vol, ctypes.c_int64), S, gamma[0], gamma[1],
                                  _p(colours, ctypes.c_int32), ncol, _p(zeta, ctypes.c_int32),
                                  _p(volC, ctypes.c_int64), threads))


def relabel(zeta):
    zeta = _i32(zeta)
    n = zeta.shape[0]
    pi = np.zeros(max(n, 1), np.int32)
    k = lib().orc_relabel(n, _p(zeta, ctypes.c_int32), _p(pi, ctypes.c_int32))
    return pi[:n], int(k)


def contract(off, col, w2, pi, k):
    """Coarse CSR (off int64[k+1], col int32, w int64) with a doubled diagonal."""
    off, col, w2, pi = _i64(off), _i32(col), _i64(w2), _i32(pi)
    nnz = col.shape[0]
    coff = np.zeros(k + 1, np.int64)
    ccol = np.zeros(max(nnz, 1), np.int32)
    cw = np.zeros(max(nnz, 1), np.int64)
    m = lib().orc_contract(off.shape[0] - 1, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                           _p(w2, ctypes.c_int64), _p(pi, ctypes.c_int32), k, _p(coff, ctypes.c_int64),
                           _p(ccol, ctypes.c_int32), _p(cw, ctypes.c_int64))
    return coff, ccol[:m].copy(), cw[:m].copy()


def modularity_parts(off, col, w2, labels):
    """(N, D, Q): integer numerator S*I2 - sum vol(C)^2, denominator S^2, and Q."""
    off, col, w2, labels = _i64(off), _i32(col), _i64(w2), _i32(labels)
    nh, nl, dh, dl = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_uint64()
    q = lib().orc_modularity(off.shape[0] - 1, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32),
                             _p(w2, ctypes.c_int64), _p(labels, ctypes.c_int32), ctypes.byref(nh),
                             ctypes.byref(nl), ctypes.byref(dh), ctypes.byref(dl))
    N = _u128(nh.value, nl.value)
    if N >= 1 << 127:
        N -= 1 << 128
    return N, _u128(dh.value, dl.value), float(q)


def modularity(off, col, w, labels) -> float:
    """Q of labels on the input graph (w: input weights or None)."""
    return modularity_parts(off, col, double_diagonal(off, col, w), labels)[2]


def canonical(labels) -> np.ndarray:
    labels = _i32(labels)
    out = np.zeros(max(labels.shape[0], 1), np.int32)
    lib().orc_canonical(labels.shape[0], _p(labels, ctypes.c_int32), _p(out, ctypes.c_int32))
    return out[: labels.shape[0]]


@dataclass
class RunResult:
    labels: np.ndarray
    q: float
    levels: int
    n: list = field(default_factory=list)
    nnz: list = field(default_factory=list)
    colours: list = field(default_factory=list)
    sweeps: list = field(default_factory=list)
    communities: list = field(default_factory=list)
    moves: list = field(default_factory=list)
    S: int = 0
    ref_sweeps: list = field(default_factory=list)   # PLMR: sweeps of the move after prolongation, per level
    ref_moves: list = field(default_factory=list)


def run(off, col, w=None, max_sweeps: int = 32, max_levels: int = 0, seed: int = 0, schedule: int = 0,
        refine: bool = False, gamma=(1, 1)) -> RunResult:
    """Full multilevel PLM (Algorithm 3), or PLMR (Algorithm 4) with refine,
    with canonical output labels; gamma = (num, den) is the resolution."""
    off, col = _i64(off), _i32(col)
    n = off.shape[0] - 1
    wp = None
    if w is not None:
        w = _i64(w)
        wp = _p(w, ctypes.c_int64)
    opt = _Options(max_sweeps, max_levels, schedule, 1 if refine else 0, seed, gamma[0], gamma[1])
    tr = _Trace()
    labels = np.zeros(max(n, 1), np.int32)
    q = ctypes.c_double()
    rc = lib().orc_run(n, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), wp, ctypes.byref(opt),
                       _p(labels, ctypes.c_int32), ctypes.byref(q), ctypes.byref(tr))
    if rc != 0:
        raise ValueError("orc_run: bad options (sweeps, or gamma outside [0, 2^16) / [1, 2^16) or too large for S)")
    L = tr.levels
    return RunResult(labels[:n].copy(), float(q.value), L, [tr.n[i] for i in range(L)],
                     [tr.nnz[i] for i in range(L)], [tr.colours[i] for i in range(L)],
                     [tr.sweeps[i] for i in range(L)], [tr.communities[i] for i in range(L)],
                     [[tr.moves[i][s] for s in range(tr.sweeps[i])] for i in range(L)], int(tr.S),
                     [tr.ref_sweeps[i] for i in range(L)], [tr.ref_moves[i] for i in range(L)])


@dataclass
class PLPResult:
    labels: np.ndarray
    q: float
    iterations: int
    updates: list   # nodes updated in each iteration


def plp(off, col, w=None, seed: int = 0, max_iters: int = 64) -> PLPResult:
    """PLP (Algorithm 1) with the colour-class schedule, active sets and
    theta = n * 10^-5; canonical labels."""
    off, col = _i64(off), _i32(col)
    n = off.shape[0] - 1
    wp = None
    if w is not None:
        w = _i64(w)
        wp = _p(w, ctypes.c_int64)
    labels = np.zeros(max(n, 1), np.int32)
    q = ctypes.c_double()
    upd = np.zeros(MAX_SWEEPS, np.int64)
    it = ctypes.c_int32()
    rc = lib().orc_plp_run(n, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), wp, seed, max_iters,
                           _p(labels, ctypes.c_int32), ctypes.byref(q), _p(upd, ctypes.c_int64), ctypes.byref(it))
    if rc != 0:
        raise ValueError("orc_plp_run: max_iters must lie in [1, 64]")
    return PLPResult(labels[:n].copy(), float(q.value), int(it.value), [int(x) for x in upd[: it.value]])


@dataclass
class EPPResult:
    labels: np.ndarray
    q: float
    cores: int      # core groups (nodes of the coarse graph given to PLMR)
    core_groups: np.ndarray  # coarse node of each input node (ascending with the smallest member)
    levels: int     # levels of the final PLMR run
    run: RunResult  # trace of the final PLMR run (its level 0 is the core-group graph)


def epp(off, col, w=None, b: int = 4, seed: int = 0, plp_iters: int = 64, max_sweeps: int = 32,
        max_levels: int = 0, gamma=(1, 1), schedule: int = 0) -> EPPResult:
    """EPP(b, PLP, PLMR) (Algorithm 5) with exact core groups (Equation (3.2))."""
    off, col = _i64(off), _i32(col)
    n = off.shape[0] - 1
    wp = None
    if w is not None:
        w = _i64(w)
        wp = _p(w, ctypes.c_int64)
    opt = _Options(max_sweeps, max_levels, schedule, 1, seed, gamma[0], gamma[1])
    tr = _Trace()
    labels = np.zeros(max(n, 1), np.int32)
    q = ctypes.c_double()
    cores = ctypes.c_int64()
    cg = np.zeros(max(n, 1), np.int32)
    rc = lib().orc_epp(n, _p(off, ctypes.c_int64), _p(col, ctypes.c_int32), wp, b, plp_iters, ctypes.byref(opt),
                       _p(labels, ctypes.c_int32), ctypes.byref(q), ctypes.byref(cores), _p(cg, ctypes.c_int32),
                       ctypes.byref(tr))
    if rc != 0:
        raise ValueError("orc_epp: bad arguments")
    L = tr.levels
    run_tr = RunResult(labels[:n].copy(), float(q.value), L, [tr.n[i] for i in range(L)],
                       [tr.nnz[i] for i in range(L)], [tr.colours[i] for i in range(L)],
                       [tr.sweeps[i] for i in range(L)], [tr.communities[i] for i in range(L)],
                       [[tr.moves[i][s] for s in range(tr.sweeps[i])] for i in range(L)], 0,
                       [tr.ref_sweeps[i] for i in range(L)], [tr.ref_moves[i] for i in range(L)])
    return EPPResult(labels[:n].copy(), float(q.value), int(cores.value), cg[:n].copy(), L, run_tr)
