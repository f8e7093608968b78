"""paper_1304_4453_amd: PLM (Parallel Louvain Method) move sweep and coarsening
on AMD Instinct MI355X, behind the C ABI of ``include/plm.h``.

This module is argument marshalling only: every step of the method runs in the
HIP kernels of ``libplm.so``.  There is no CPU fallback; importing the binding
without a built library raises.

Low level: ``plm_create``, ``plm_move_sweep``, ``plm_move_class``,
``plm_coarsen``, ``plm_run``, ``plm_plp``, ``plm_epp``, ``plm_modularity``,
``plm_modularity_noalloc``, ``plm_reset``,
``plm_destroy``, ``plm_last_error``, ``plm_level_info``, ``plm_get_state``,
``plm_get_graph``, ``plm_get_stats``, ``plm_default_options`` (ctypes functions
with the C signatures).  ``Context`` wraps them for numpy (host) and torch
(device) arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime; loading it before libplm.so makes the library
# bind to that same runtime, so one process never holds two HIP runtimes.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplm.so")

PLM_OK, PLM_E_ARG, PLM_E_GRAPH, PLM_E_NOMEM, PLM_E_DEVICE, PLM_E_BUDGET, PLM_E_STATE = 0, -1, -2, -3, -4, -5, -6
PLM_MEM_HOST, PLM_MEM_DEVICE = 0, 1
PLM_SCHEDULE_COLOUR, PLM_SCHEDULE_SEQUENTIAL = 0, 1
PLM_INT_AUTO, PLM_INT_64, PLM_INT_128 = 0, 1, 2
PLM_MAX_LEVELS = 64

_STATUS_NAMES = {0: "PLM_OK", -1: "PLM_E_ARG", -2: "PLM_E_GRAPH", -3: "PLM_E_NOMEM", -4: "PLM_E_DEVICE",
                 -5: "PLM_E_BUDGET", -6: "PLM_E_STATE"}


class plm_options(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("colour_seed", ctypes.c_uint64), ("int_mode", ctypes.c_int32),
                ("bin_lane", ctypes.c_int32), ("bin_wave", ctypes.c_int32), ("bin_block", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("timing_kernel", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("gamma_num", ctypes.c_int32), ("gamma_den", ctypes.c_int32), ("graph_sweeps", ctypes.c_int32),
                ("hub_stream", ctypes.c_int32), ("colour_tail", ctypes.c_int32), ("hub_row_max", ctypes.c_int32),
                ("agg_max_keys", ctypes.c_int32), ("agg_tile", ctypes.c_int32), ("settle", ctypes.c_int32),
                ("join", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("pack_bits", ctypes.c_int32)]


class plm_level_info_t(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("colours", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("S", ctypes.c_int64), ("sweeps", ctypes.c_int32),
                ("weight_kind", ctypes.c_int32), ("communities", ctypes.c_int64), ("max_vol", ctypes.c_int64)]


_L = PLM_MAX_LEVELS


class plm_stats_t(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n", ctypes.c_int64 * _L), ("nnz", ctypes.c_int64 * _L), ("colours", ctypes.c_int64 * _L),
                ("sweeps", ctypes.c_int64 * _L), ("communities", ctypes.c_int64 * _L),
                ("moves", ctypes.c_int64 * _L), ("schedule_ms", ctypes.c_double * _L),
                ("sweep_ms", ctypes.c_double * _L), ("coarsen_ms", ctypes.c_double * _L),
                ("decide_ms", ctypes.c_double * _L), ("decide_launches", ctypes.c_int64 * _L),
                ("decide_bytes", ctypes.c_double * _L), ("schedule_rounds", ctypes.c_int64 * _L),
                ("colour_ms", ctypes.c_double * _L), ("bin_ms", (ctypes.c_double * 4) * _L),
                ("bin_bytes", (ctypes.c_double * 4) * _L), ("bin_nodes", (ctypes.c_int64 * 4) * _L),
                ("bin_entries", (ctypes.c_int64 * 4) * _L), ("loops", ctypes.c_int64 * _L),
                ("hub_single_ms", ctypes.c_double * _L), ("hub_single_bytes", ctypes.c_double * _L),
                ("hub_single_nodes", ctypes.c_int64 * _L), ("hub_single_entries", ctypes.c_int64 * _L),
                ("kernel_launches", (ctypes.c_int64 * 5) * _L), ("ref_sweeps", ctypes.c_int64 * _L),
                ("ref_moves", ctypes.c_int64 * _L), ("ref_ms", ctypes.c_double * _L),
                ("lp_runs", ctypes.c_int64), ("lp_iterations", ctypes.c_int64), ("lp_updates", ctypes.c_int64),
                ("lp_ms", ctypes.c_double), ("lp_decide_ms", ctypes.c_double), ("lp_first_ms", ctypes.c_double),
                ("lp_first_bytes", ctypes.c_double), ("ens_ms", ctypes.c_double), ("ens_cores", ctypes.c_int64),
                ("cycle_sweeps", ctypes.c_int64 * _L), ("ref_cycle_sweeps", ctypes.c_int64 * _L),
                ("settle_sweeps", ctypes.c_int64 * _L), ("decided_nodes", ctypes.c_int64 * _L),
                ("decided_entries", ctypes.c_int64 * _L), ("settled_nodes", ctypes.c_int64 * _L)]


class plm_server_info_t(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("held_results", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("inflight", ctypes.c_int64),
                ("running", ctypes.c_int64), ("resident_bytes", ctypes.c_int64), ("joined", ctypes.c_int64)]


class PLMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libplm.so not built ({LIB_PATH}); run paper_1304_4453_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.plm_default_options.argtypes = [P(plm_options)]
    lib.plm_default_options.restype = None
    lib.plm_create.argtypes = [P(vp), i64, i64, vp, vp, vp, i32, vp, P(plm_options)]
    lib.plm_move_sweep.argtypes = [vp, P(i64)]
    lib.plm_move_class.argtypes = [vp, i32, P(i64)]
    lib.plm_coarsen.argtypes = [vp, P(i64)]
    lib.plm_run.argtypes = [vp, vp, P(dbl), P(i32)]
    lib.plm_plp.argtypes = [vp, i32, vp, P(dbl), P(i32), P(i64)]
    lib.plm_epp.argtypes = [vp, i32, i32, vp, P(dbl), P(i32), P(i64)]
    lib.plm_modularity.argtypes = [vp, vp, i32, P(dbl)]
    lib.plm_modularity_noalloc.argtypes = [vp, vp, P(dbl)]
    lib.plm_reset.argtypes = [vp]
    lib.plm_get_options.argtypes = [vp, P(plm_options)]
    lib.plm_get_options.restype = i32
    lib.plm_resolve_options.argtypes = [P(plm_options), i32, i64]
    lib.plm_resolve_options.restype = i32
    lib.plm_tuned_table.argtypes = []
    lib.plm_tuned_table.restype = ctypes.c_char_p
    lib.plm_destroy.argtypes = [vp]
    lib.plm_destroy.restype = None
    lib.plm_last_error.argtypes = [vp]
    lib.plm_last_error.restype = ctypes.c_char_p
    lib.plm_level_info.argtypes = [vp, P(plm_level_info_t)]
    lib.plm_get_state.argtypes = [vp, vp, vp, vp, i32]
    lib.plm_get_graph.argtypes = [vp, vp, vp, vp, i32]
    lib.plm_get_stats.argtypes = [vp, P(plm_stats_t)]
    lib.plm_batch_create.argtypes = [P(vp), i64, vp, i64, vp, vp, vp, i32, vp, P(plm_options)]
    lib.plm_batch_run.argtypes = [vp, vp, vp, vp]
    lib.plm_server_create.argtypes = [P(vp), i64, i64, i32, vp, P(plm_options)]
    lib.plm_server_wait.argtypes = [vp, P(i32)]
    lib.plm_server_submit.argtypes = [vp, i64, i64, vp, vp, vp, i32, P(i64)]
    lib.plm_server_step.argtypes = [vp, P(i32)]
    lib.plm_server_result.argtypes = [vp, i64, vp, i32, P(dbl), P(i32), P(i32)]
    lib.plm_server_info.argtypes = [vp, P(plm_server_info_t)]
    lib.plm_server_destroy.argtypes = [vp]
    lib.plm_server_destroy.restype = None
    lib.plm_server_last_error.argtypes = [vp]
    lib.plm_server_last_error.restype = ctypes.c_char_p
    for f in ("plm_create", "plm_batch_create", "plm_batch_run", "plm_server_create", "plm_server_submit",
              "plm_server_step", "plm_server_wait", "plm_server_result", "plm_server_info", "plm_move_sweep", "plm_move_class", "plm_coarsen", "plm_run", "plm_plp", "plm_epp", "plm_modularity",
              "plm_modularity_noalloc",
              "plm_reset", "plm_level_info", "plm_get_state", "plm_get_graph", "plm_get_stats"):
        getattr(lib, f).restype = i32
    return lib


_lib = _load()

plm_default_options = _lib.plm_default_options
plm_create = _lib.plm_create
plm_move_sweep = _lib.plm_move_sweep
plm_move_class = _lib.plm_move_class
plm_coarsen = _lib.plm_coarsen
plm_run = _lib.plm_run
plm_plp = _lib.plm_plp
plm_epp = _lib.plm_epp
plm_modularity = _lib.plm_modularity
plm_modularity_noalloc = _lib.plm_modularity_noalloc
PLM_NOALLOC_MAX_NODES = 1 << 23
plm_reset = _lib.plm_reset
plm_get_options = _lib.plm_get_options
plm_tuned_table = _lib.plm_tuned_table
plm_resolve_options = _lib.plm_resolve_options


def resolve_options(batched: bool, nnz: int, **kw) -> plm_options:
    """The options a context (batched or not, of nnz entries) takes for kw:
    degree bins left at 0 filled from the tuned table or the compiled defaults."""
    o = default_options(**kw)
    rc = plm_resolve_options(ctypes.byref(o), int(batched), int(nnz))
    if rc != 0:
        raise PLMError(rc, "invalid options")
    return o
plm_destroy = _lib.plm_destroy
plm_last_error = _lib.plm_last_error
plm_level_info = _lib.plm_level_info
plm_get_state = _lib.plm_get_state
plm_get_graph = _lib.plm_get_graph
plm_get_stats = _lib.plm_get_stats
plm_batch_create = _lib.plm_batch_create
plm_batch_run = _lib.plm_batch_run
plm_server_create = _lib.plm_server_create
plm_server_submit = _lib.plm_server_submit
plm_server_step = _lib.plm_server_step
plm_server_wait = _lib.plm_server_wait
plm_server_result = _lib.plm_server_result
plm_server_info = _lib.plm_server_info
plm_server_destroy = _lib.plm_server_destroy
plm_server_last_error = _lib.plm_server_last_error


def default_options(**kw) -> plm_options:
    o = plm_options()
    plm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a) -> int:
    """Address of a numpy array, a torch tensor, an int address or None."""
    if a is None:
        return 0
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


class Context:
    """Owns one plm_ctx.  Host inputs: numpy arrays (mem_kind host).  Device
    inputs: torch tensors on the current HIP device or raw device addresses
    (mem_kind device).  stream: torch stream object, raw hipStream_t int, or None."""

    def __init__(self, off, col, w=None, mem_kind: int | None = None, stream=None, n: int | None = None,
                 nnz: int | None = None, **options):
        self._c = ctypes.c_void_p()
        if mem_kind is None:
            mem_kind = PLM_MEM_HOST if isinstance(off, np.ndarray) else PLM_MEM_DEVICE
        if mem_kind == PLM_MEM_HOST:
            off = np.ascontiguousarray(off, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            if w is not None:
                w = np.ascontiguousarray(w, dtype=np.int32)
        if n is None:
            n = int(off.shape[0]) - 1
        if nnz is None:
            nnz = int(col.shape[0])
        self._keep = (off, col, w)
        self.n, self.nnz, self.mem_kind = n, nnz, mem_kind
        sp = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
        self.opt = default_options(**options)
        rc = plm_create(ctypes.byref(self._c), n, nnz, _ptr(off), _ptr(col), _ptr(w), mem_kind, sp or 0,
                        ctypes.byref(self.opt))
        self._keep = None
        if rc != 0:
            raise PLMError(rc, plm_last_error(None).decode())

    def _check(self, rc):
        if rc != 0:
            raise PLMError(rc, plm_last_error(self._c).decode())

    def close(self):
        if self._c:
            plm_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- method
    def move_sweep(self) -> int:
        mv = ctypes.c_int64()
        self._check(plm_move_sweep(self._c, ctypes.byref(mv)))
        return mv.value

    def move_class(self, c: int) -> int:
        mv = ctypes.c_int64()
        self._check(plm_move_class(self._c, c, ctypes.byref(mv)))
        return mv.value

    def coarsen(self) -> int:
        k = ctypes.c_int64()
        self._check(plm_coarsen(self._c, ctypes.byref(k)))
        return k.value

    def run(self, labels=None):
        """Full run.  labels: output buffer (numpy int32 for host contexts,
        torch int32 tensor / address for device contexts) or None for a new
        numpy array (host contexts).  Returns (labels, q, levels)."""
        if labels is None and self.mem_kind == PLM_MEM_HOST:
            labels = np.zeros(self.n, np.int32)
        q, lv = ctypes.c_double(), ctypes.c_int32()
        self._check(plm_run(self._c, _ptr(labels), ctypes.byref(q), ctypes.byref(lv)))
        return labels, q.value, lv.value

    def plp(self, max_iters: int = 64, labels=None):
        """Label propagation (Algorithm 1) on the input graph.  Returns
        (labels, q, iterations, updates per iteration)."""
        if labels is None and self.mem_kind == PLM_MEM_HOST:
            labels = np.zeros(self.n, np.int32)
        q, it = ctypes.c_double(), ctypes.c_int32()
        upd = (ctypes.c_int64 * 64)()
        self._check(plm_plp(self._c, max_iters, _ptr(labels), ctypes.byref(q), ctypes.byref(it), upd))
        return labels, q.value, it.value, [int(upd[i]) for i in range(it.value)]

    def epp(self, ensemble_size: int = 4, plp_iters: int = 64, labels=None):
        """EPP(b, PLP, PLMR) (Algorithm 5).  Returns (labels, q, levels, cores)."""
        if labels is None and self.mem_kind == PLM_MEM_HOST:
            labels = np.zeros(self.n, np.int32)
        q, lv, k = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int64()
        self._check(plm_epp(self._c, ensemble_size, plp_iters, _ptr(labels), ctypes.byref(q), ctypes.byref(lv),
                            ctypes.byref(k)))
        return labels, q.value, lv.value, k.value

    def modularity(self, labels, mem_kind: int | None = None) -> float:
        if mem_kind is None:
            mem_kind = PLM_MEM_HOST if isinstance(labels, np.ndarray) else PLM_MEM_DEVICE
        if isinstance(labels, np.ndarray):
            labels = np.ascontiguousarray(labels, dtype=np.int32)
        q = ctypes.c_double()
        self._check(plm_modularity(self._c, _ptr(labels), mem_kind, ctypes.byref(q)))
        return q.value

    def modularity_noalloc(self, labels) -> float:
        """plm_modularity_noalloc: labels in device memory (torch int32 tensor
        or address); no device allocation inside the call."""
        q = ctypes.c_double()
        self._check(plm_modularity_noalloc(self._c, _ptr(labels), ctypes.byref(q)))
        return q.value

    def reset(self):
        self._check(plm_reset(self._c))

    def options(self) -> plm_options:
        """The options the context runs with (degree bins resolved)."""
        o = plm_options()
        self._check(plm_get_options(self._c, ctypes.byref(o)))
        return o

    # ---- inspection
    def level_info(self) -> plm_level_info_t:
        li = plm_level_info_t()
        self._check(plm_level_info(self._c, ctypes.byref(li)))
        return li

    def state(self):
        """(zeta, volC, colour) of the current level as numpy arrays."""
        n = self.level_info().n
        z = np.zeros(max(n, 1), np.int32); v = np.zeros(max(n, 1), np.int64); c = np.zeros(max(n, 1), np.int32)
        self._check(plm_get_state(self._c, z.ctypes.data, v.ctypes.data, c.ctypes.data, PLM_MEM_HOST))
        return z[:n], v[:n], c[:n]

    def graph(self):
        """(off, col, w with doubled diagonal) of the current level as numpy arrays."""
        li = self.level_info()
        off = np.zeros(li.n + 1, np.int64)
        col = np.zeros(max(li.nnz, 1), np.int32)
        w = np.zeros(max(li.nnz, 1), np.int64)
        self._check(plm_get_graph(self._c, off.ctypes.data, col.ctypes.data, w.ctypes.data, PLM_MEM_HOST))
        return off, col[: li.nnz], w[: li.nnz]

    def stats(self) -> dict:
        s = plm_stats_t()
        self._check(plm_get_stats(self._c, ctypes.byref(s)))
        L = s.levels
        out = {"levels": L}
        for f, _ in plm_stats_t._fields_[2:]:
            v = getattr(s, f)
            if isinstance(v, (int, float)):
                out[f] = v
                continue
            out[f] = [list(x) if not isinstance(x, (int, float)) else x for x in list(v)[:L]]
        return out


def pack_batch(graphs):
    """Disjoint union of host CSR graphs (objects with off, col, w or tuples
    (off, col, w)): returns (node_base, off, col, w) with global node ids; w is
    None when no graph carries weights (unit weights), else every graph's
    weights (unit weights filled in for unweighted members)."""
    parts = [(g.off, g.col, g.w) if hasattr(g, "off") else tuple(g) for g in graphs]
    ns = np.array([len(o) - 1 for o, _, _ in parts], np.int64)
    node_base = np.zeros(len(parts) + 1, np.int64)
    node_base[1:] = np.cumsum(ns)
    ms = np.array([len(c) for _, c, _ in parts], np.int64)
    ebase = np.zeros(len(parts) + 1, np.int64)
    ebase[1:] = np.cumsum(ms)
    off = np.zeros(int(node_base[-1]) + 1, np.int64)
    col = np.zeros(int(ebase[-1]), np.int32)
    weighted = any(w is not None for _, _, w in parts)
    w = np.ones(int(ebase[-1]), np.int32) if weighted else None
    for i, (o, c, ww) in enumerate(parts):
        a, b = int(node_base[i]), int(node_base[i + 1])
        off[a:b] = np.asarray(o[:-1], np.int64) + ebase[i]
        col[ebase[i]:ebase[i + 1]] = np.asarray(c, np.int64) + a
        if weighted and ww is not None:
            w[ebase[i]:ebase[i + 1]] = ww
    off[-1] = ebase[-1]
    return node_base, off, col, w


class BatchContext(Context):
    """Owns one batched plm_ctx (plm_batch_create): graph g holds the nodes
    node_base[g] .. node_base[g+1]-1 of the union CSR (off, col, w)."""

    def __init__(self, node_base, off, col, w=None, mem_kind: int | None = None, stream=None,
                 nnz: int | None = None, **options):
        self._c = ctypes.c_void_p()
        node_base = np.ascontiguousarray(node_base, dtype=np.int64)
        if mem_kind is None:
            mem_kind = PLM_MEM_HOST if isinstance(off, np.ndarray) else PLM_MEM_DEVICE
        if mem_kind == PLM_MEM_HOST:
            off = np.ascontiguousarray(off, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            if w is not None:
                w = np.ascontiguousarray(w, dtype=np.int32)
        if nnz is None:
            nnz = int(col.shape[0])
        self.G = int(node_base.shape[0]) - 1
        self.node_base = node_base
        self.n, self.nnz, self.mem_kind = int(node_base[-1]), nnz, mem_kind
        sp = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
        self.opt = default_options(**options)
        rc = plm_batch_create(ctypes.byref(self._c), self.G, node_base.ctypes.data, nnz, _ptr(off), _ptr(col),
                              _ptr(w), mem_kind, sp or 0, ctypes.byref(self.opt))
        if rc != 0:
            raise PLMError(rc, plm_last_error(None).decode())

    def run_batch(self, labels=None):
        """Runs every graph.  Returns (labels, q[G], levels[G]); labels are
        numbered from 0 within each graph."""
        if labels is None and self.mem_kind == PLM_MEM_HOST:
            labels = np.zeros(self.n, np.int32)
        q = np.zeros(max(self.G, 1), np.float64)
        lv = np.zeros(max(self.G, 1), np.int32)
        self._check(plm_batch_run(self._c, _ptr(labels), q.ctypes.data, lv.ctypes.data))
        return labels, q[: self.G], lv[: self.G]


class Server:
    """Owns one plm_server.  submit() queues a graph without copying it: the
    arrays (numpy for host, torch tensors or addresses for device memory) are
    kept alive here until its result is fetched.  max_inflight >= 2 runs up to
    that many batches at once on worker threads of the server; step() then
    returns after handing a batch over, and wait() blocks until none runs."""

    def __init__(self, hbm_budget_bytes: int, max_batch_entries: int = 1 << 40, stream=None, max_inflight: int = 1,
                 **options):
        self._s = ctypes.c_void_p()
        sp = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
        self.opt = default_options(**options)
        rc = plm_server_create(ctypes.byref(self._s), hbm_budget_bytes, max_batch_entries, max_inflight, sp or 0,
                               ctypes.byref(self.opt))
        if rc != 0:
            raise PLMError(rc, "plm_server_create failed")
        self._held = {}

    def _check(self, rc):
        if rc != 0:
            raise PLMError(rc, plm_server_last_error(self._s).decode())

    def submit(self, off, col, w=None, mem_kind: int | None = None, n: int | None = None,
               nnz: int | None = None) -> int:
        if mem_kind is None:
            mem_kind = PLM_MEM_HOST if isinstance(off, np.ndarray) else PLM_MEM_DEVICE
        if mem_kind == PLM_MEM_HOST:
            off = np.ascontiguousarray(off, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            if w is not None:
                w = np.ascontiguousarray(w, dtype=np.int32)
        if n is None:
            n = int(off.shape[0]) - 1
        if nnz is None:
            nnz = int(col.shape[0])
        rid = ctypes.c_int64()
        self._check(plm_server_submit(self._s, n, nnz, _ptr(off), _ptr(col), _ptr(w), mem_kind, ctypes.byref(rid)))
        self._held[rid.value] = (off, col, w, n)
        return rid.value

    def step(self) -> int:
        c = ctypes.c_int32()
        self._check(plm_server_step(self._s, ctypes.byref(c)))
        return c.value

    def wait(self) -> int:
        c = ctypes.c_int32()
        self._check(plm_server_wait(self._s, ctypes.byref(c)))
        return c.value

    def result(self, rid: int, labels=None, mem_kind: int | None = None):
        """(ready, labels, q, levels); labels: output buffer or None for a new
        numpy array (when the request's inputs were host arrays) or discarded."""
        held = self._held.get(rid)
        n = held[3] if held else 0
        if labels is None and held and isinstance(held[0], np.ndarray):
            labels = np.zeros(max(n, 1), np.int32)
        if mem_kind is None:
            mem_kind = PLM_MEM_HOST if labels is None or isinstance(labels, np.ndarray) else PLM_MEM_DEVICE
        q, lv, ready = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32()
        try:
            self._check(plm_server_result(self._s, rid, _ptr(labels), mem_kind, ctypes.byref(q), ctypes.byref(lv),
                                          ctypes.byref(ready)))
        except PLMError:
            self._held.pop(rid, None)
            raise
        if not ready.value:
            return False, None, None, None
        self._held.pop(rid, None)
        if isinstance(labels, np.ndarray):
            labels = labels[:n]
        return True, labels, q.value, lv.value

    def info(self) -> plm_server_info_t:
        i = plm_server_info_t()
        self._check(plm_server_info(self._s, ctypes.byref(i)))
        return i

    def close(self):
        if self._s:
            plm_server_destroy(self._s)
            self._s = ctypes.c_void_p()
        self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
