"""The C ABI: libplm.so loads, exports every entry point include/plm.h declares,
and the Python binding's struct layouts match the header.  CPU only: no call
here reaches the GPU (argument errors return before any HIP call)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plm.h")
LIB = os.path.join(ROOT, "paper_1304_4453_amd", "libplm.so")


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        subprocess.run(["python", os.path.join(ROOT, "paper_1304_4453_amd", "build.py")], check=True)
    assert os.path.exists(LIB), "libplm.so missing: run __graft_entry__.build()"
    return LIB


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(plm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["plm_create", "plm_move_sweep", "plm_coarsen", "plm_run", "plm_modularity", "plm_destroy",
                 "plm_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (plm_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(built)
    for f in declared_functions():
        assert hasattr(lib, f)


def test_struct_layouts_match_header(tmp_path, built):
    import paper_1304_4453_amd as P
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "plm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(plm_options), sizeof(plm_level_info_t),"
        " sizeof(plm_stats_t), offsetof(plm_options, colour_seed), offsetof(plm_stats_t, decide_bytes),"
        " offsetof(plm_level_info_t, max_vol)); return 0;}\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(P.plm_options), ctypes.sizeof(P.plm_level_info_t), ctypes.sizeof(P.plm_stats_t),
                    P.plm_options.colour_seed.offset, P.plm_stats_t.decide_bytes.offset,
                    P.plm_level_info_t.max_vol.offset]


def test_default_options(built):
    import paper_1304_4453_amd as P
    o = P.default_options()
    assert (o.max_sweeps, o.max_levels, o.schedule, o.validate, o.int_mode) == (32, 0, 0, 1, 0)
    assert (o.bin_lane, o.bin_wave, o.bin_block, o.timing) == (0, 0, 0, 0)   # 0: tuned table
    assert (o.graph_sweeps, o.hub_stream, o.colour_tail) == (1, 2, 1)
    assert (o.hub_row_max, o.agg_max_keys, o.agg_tile, o.settle) == (0, 0, 0, 0)
    assert (o.join, o.layout, o.pack_bits) == (0, 0, 0)


def test_argument_errors_need_no_gpu(built):
    import numpy as np
    import paper_1304_4453_amd as P
    c = ctypes.c_void_p()
    off = np.zeros(2, np.int64)
    col = np.zeros(0, np.int32)
    assert P.plm_create(None, 1, 0, off.ctypes.data, col.ctypes.data, None, 0, None, None) == P.PLM_E_ARG
    assert P.plm_create(ctypes.byref(c), -1, 0, off.ctypes.data, col.ctypes.data, None, 0, None, None) == P.PLM_E_ARG
    assert b"n must" in P.plm_last_error(None)
    assert P.plm_create(ctypes.byref(c), 1, 0, None, col.ctypes.data, None, 0, None, None) == P.PLM_E_ARG
    assert P.plm_create(ctypes.byref(c), 1, 0, off.ctypes.data, col.ctypes.data, None, 7, None, None) == P.PLM_E_ARG
    bad = P.default_options(bin_wave=9999)
    assert P.plm_create(ctypes.byref(c), 1, 0, off.ctypes.data, col.ctypes.data, None, 0, None,
                        ctypes.byref(bad)) == P.PLM_E_ARG
    for kw in (dict(max_sweeps=0), dict(graph_sweeps=2), dict(hub_stream=-1), dict(hub_stream=3), dict(colour_tail=2),
               dict(hub_row_max=-1), dict(hub_row_max=12289), dict(agg_max_keys=31), dict(agg_max_keys=1537),
               dict(agg_tile=-1), dict(agg_tile=513), dict(layout=2), dict(pack_bits=1), dict(pack_bits=63),
               dict(pack_bits=-2)):
        bad = P.default_options(**kw)
        assert P.plm_create(ctypes.byref(c), 1, 0, off.ctypes.data, col.ctypes.data, None, 0, None,
                            ctypes.byref(bad)) == P.PLM_E_ARG, kw
    off_bad = np.array([0, 3], np.int64)   # offsets[n] != nnz
    assert P.plm_create(ctypes.byref(c), 1, 0, off_bad.ctypes.data, col.ctypes.data, None, 0, None,
                        None) == P.PLM_E_GRAPH
    assert not c.value
    # every ctx entry point rejects a NULL context
    assert P.plm_move_sweep(None, None) == P.PLM_E_ARG
    assert P.plm_coarsen(None, None) == P.PLM_E_ARG
    assert P.plm_run(None, None, None, None) == P.PLM_E_ARG
    assert P.plm_modularity(None, None, 0, None) == P.PLM_E_ARG
    assert P.plm_batch_run(None, None, None, None) == P.PLM_E_ARG
    P.plm_destroy(None)
    # batched contexts: graph ranges and options are checked before any HIP call
    nb = np.array([0, 1], np.int64)
    assert P.plm_batch_create(ctypes.byref(c), 0, nb.ctypes.data, 0, off.ctypes.data, col.ctypes.data, None, 0,
                              None, None) == P.PLM_E_ARG
    assert P.plm_batch_create(ctypes.byref(c), 1, None, 0, off.ctypes.data, col.ctypes.data, None, 0, None,
                              None) == P.PLM_E_ARG
    nb_bad = np.array([1, 1], np.int64)
    assert P.plm_batch_create(ctypes.byref(c), 1, nb_bad.ctypes.data, 0, off.ctypes.data, col.ctypes.data, None,
                              0, None, None) == P.PLM_E_ARG
    seq = P.default_options(schedule=P.PLM_SCHEDULE_SEQUENTIAL)
    assert P.plm_batch_create(ctypes.byref(c), 1, nb.ctypes.data, 0, off.ctypes.data, col.ctypes.data, None, 0,
                              None, ctypes.byref(seq)) == P.PLM_E_ARG
    i64 = P.default_options(int_mode=P.PLM_INT_64)
    assert P.plm_batch_create(ctypes.byref(c), 1, nb.ctypes.data, 0, off.ctypes.data, col.ctypes.data, None, 0,
                              None, ctypes.byref(i64)) == P.PLM_E_ARG
    assert not c.value


def test_server_queue_needs_no_gpu(built):
    """Creation, submission, queue accounting and argument errors of the
    request server run on the host only."""
    import numpy as np
    import graphgen
    import paper_1304_4453_amd as P
    s = ctypes.c_void_p()
    assert P.plm_server_create(None, 1 << 30, 1 << 20, 1, None, None) == P.PLM_E_ARG
    assert P.plm_server_create(ctypes.byref(s), 0, 1 << 20, 1, None, None) == P.PLM_E_ARG
    for k in (0, 17):   # max_inflight outside [1, 16]
        assert P.plm_server_create(ctypes.byref(s), 1 << 30, 1 << 20, k, None, None) == P.PLM_E_ARG
    seq = P.default_options(schedule=P.PLM_SCHEDULE_SEQUENTIAL)
    assert P.plm_server_create(ctypes.byref(s), 1 << 30, 1 << 20, 1, None, ctypes.byref(seq)) == P.PLM_E_ARG
    g = graphgen.disjoint_cliques(2, 4)
    srv = P.Server(1 << 30)
    a = srv.submit(g.off, g.col, g.w)
    b = srv.submit(g.off, g.col, g.w)
    assert (a, b) == (0, 1) and srv.info().queued == 2 and srv.info().budget_bytes == 1 << 30
    ready, _, _, _ = srv.result(a)
    assert not ready
    with pytest.raises(P.PLMError) as e:
        srv.submit(np.array([0, 3], np.int64), np.zeros(2, np.int32))   # offsets[n] != nnz
    assert e.value.status == P.PLM_E_GRAPH
    tiny = P.Server(64)
    with pytest.raises(P.PLMError) as e:
        tiny.submit(g.off, g.col, g.w)
    assert e.value.status == P.PLM_E_BUDGET
    with pytest.raises(P.PLMError) as e:
        srv.result(99)
    assert e.value.status == P.PLM_E_ARG
    assert P.plm_server_step(None, None) == P.PLM_E_ARG
    assert P.plm_server_wait(None, None) == P.PLM_E_ARG
    i = srv.info()
    assert i.inflight == 0 and i.running == 0 and i.resident_bytes == 0


def test_pack_batch_is_the_disjoint_union(built):
    import numpy as np
    import graphgen
    import paper_1304_4453_amd as P
    gs = [graphgen.disjoint_cliques(2, 3), graphgen.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), None),
          graphgen.random_graph(10, 0.3, seed=1), graphgen.from_edges(3, [])]
    nb, off, col, w = P.pack_batch(gs)
    assert nb.tolist() == [0, 6, 6, 16, 19] and off[0] == 0 and off[-1] == sum(g.nnz for g in gs)
    for i, g in enumerate(gs):
        a, b = int(nb[i]), int(nb[i + 1])
        assert np.array_equal(off[a:b + 1] - off[a], g.off)
        assert np.array_equal(col[off[a]:off[b]] - a, g.col)
        assert np.array_equal(w[off[a]:off[b]], np.ones(g.nnz) if g.w is None else g.w)
    nb, off, col, w = P.pack_batch([graphgen.disjoint_cliques(1, 3)] * 2)
    assert w is None and col.tolist() == [1, 2, 0, 2, 0, 1, 4, 5, 3, 5, 3, 4]


def test_product_has_no_oracle_dependency():
    """The library sources and the binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1304_4453_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
