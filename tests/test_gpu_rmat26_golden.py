"""R-MAT scale 26 (weights 1..100, seed 3) end to end against the oracle.

tests/golden/rmat26_oracle.json holds the oracle's own run on this graph
(written by tests/golden/make_rmat26_golden.py, which calls only the oracle
and the input generators): per level n, nnz, S, the SHA-256 of the level's
CSR and node volumes, the colour count and the SHA-256 of the colouring, and
for every sweep its move count and the SHA-256 of the community ids and
community volumes after it; the community count; then the SHA-256 of the
canonical labels, Q and the level count.

Two tests, both on the graph the device generator builds (checked here
against the SHA-256 of the host generator's arrays the oracle ran on):

* stepwise: level by level through plm_move_sweep / plm_coarsen, every
  sweep's move count, community ids and community volumes, the colouring and
  every coarse level's CSR compared with the oracle's (section III-B,
  Algorithms 2 and 3);
* full run in the launch configuration the benchmark times (default
  options: captured sweeps, concurrent kernel branches, the period-2 cycle
  fast-forward): canonical labels, Q bit for bit, the level count and the
  per-level trace.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat26_oracle.json")


def _gold():
    if not os.path.exists(GOLDEN):
        pytest.skip("no stored oracle run of R-MAT 26 (tests/golden/make_rmat26_golden.py writes it)")
    g = json.load(open(GOLDEN))
    if "graph" not in g:
        pytest.skip("the stored oracle run has no level yet")
    return g


def _levels(gold):
    """Recorded levels; while the writer runs, the level in progress (its
    finished sweeps, without a community count) comes last."""
    return gold.get("levels_partial", gold["levels"])


def _sha(a) -> str:
    h = hashlib.sha256()
    mv = memoryview(np.ascontiguousarray(a)).cast("B")
    step = 1 << 28
    for i in range(0, len(mv), step):
        h.update(mv[i:i + step])
    return h.hexdigest()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


@pytest.fixture(scope="module")
def rmat26():
    gold = _gold()
    _say("rmat26 generate")
    dg = graphgen.rmat_gpu(26, 16, seed=3, weighted=True)
    try:
        gr = gold["graph"]
        assert (dg.n, dg.nnz) == (gr["n"], gr["nnz"])
        lib = graphgen._gpu_lib()
        off = np.empty(dg.n + 1, np.int64)
        lib.ggpu_copy_to_host(off.ctypes.data, ctypes.c_void_p(dg.off_ptr), off.nbytes)
        assert _sha(off) == gr["off_sha256"]
        del off
        for ptr, key in ((dg.col_ptr, "col_sha256"), (dg.w_ptr, "w_sha256")):
            a = np.empty(dg.nnz, np.int32)
            lib.ggpu_copy_to_host(a.ctypes.data, ctypes.c_void_p(ptr), a.nbytes)
            assert _sha(a) == gr[key], key
            del a
        yield gold, dg
    finally:
        dg.free()


@pytest.mark.timeout(900)
def test_rmat26_stepwise_equals_oracle(P, rmat26):
    gold, dg = rmat26
    ctx = P.Context(dg.off_ptr, dg.col_ptr, dg.w_ptr, mem_kind=P.PLM_MEM_DEVICE, n=dg.n, nnz=dg.nnz)
    try:
        for lv in _levels(gold):
            li = ctx.level_info()
            assert (li.level, li.n, li.nnz, li.S) == (lv["level"], lv["n"], lv["nnz"], lv["S"])
            if lv["level"] > 0:
                off, col, w = ctx.graph()
                assert _sha(off) == lv["off_sha256"] and _sha(col) == lv["col_sha256"]
                assert _sha(w) == lv["w_sha256"]
                del off, col, w
            z, volc, colour = ctx.state()            # builds the level's colouring
            assert ctx.level_info().colours == lv["colours"]
            assert _sha(colour) == lv["colour_sha256"], f"level {lv['level']} colouring"
            assert _sha(volc) == lv["vol_sha256"] and np.array_equal(z, np.arange(li.n))
            _say(f"level {lv['level']}: n={li.n} nnz={li.nnz} colours={lv['colours']} equal")
            for s, sw in enumerate(lv["sweeps"]):
                mv = ctx.move_sweep()
                z, volc, _ = ctx.state()
                assert mv == sw["moves"], f"level {lv['level']} sweep {s + 1}: moves {mv} != {sw['moves']}"
                assert _sha(z) == sw["zeta_sha256"], f"level {lv['level']} sweep {s + 1}: community ids"
                assert _sha(volc) == sw["volc_sha256"], f"level {lv['level']} sweep {s + 1}: community volumes"
                _say(f"level {lv['level']} sweep {s + 1}: {mv} moves, state equal")
            if "communities" not in lv:
                break                                # the level the writer is still on
            assert ctx.level_info().communities == lv["communities"]
            if lv["communities"] < lv["n"]:
                assert ctx.coarsen() == lv["communities"]
    finally:
        ctx.close()


@pytest.mark.timeout(600)
def test_rmat26_full_run_equals_oracle(P, rmat26):
    import torch
    gold, dg = rmat26
    if not gold.get("complete"):
        pytest.skip("the stored oracle run is not complete yet")
    ctx = P.Context(dg.off_ptr, dg.col_ptr, dg.w_ptr, mem_kind=P.PLM_MEM_DEVICE, n=dg.n, nnz=dg.nnz)
    try:
        lab = torch.empty(dg.n, dtype=torch.int32, device="cuda:0")
        _, q, levels = ctx.run(lab)
        st = ctx.stats()
        labels = lab.cpu().numpy()
        assert _sha(labels) == gold["labels_sha256"]
        assert q == float.fromhex(gold["q_hex"]) and levels == gold["levels_count"]
        for i, lv in enumerate(gold["levels"]):
            assert st["n"][i] == lv["n"] and st["nnz"][i] == lv["nnz"] and st["colours"][i] == lv["colours"]
            assert st["sweeps"][i] == len(lv["sweeps"]) and st["communities"][i] == lv["communities"]
            assert st["moves"][i] == sum(s["moves"] for s in lv["sweeps"]), f"level {i} moves"
        _say(f"rmat26 full run equal: Q={q!r} levels={levels} cycle sweeps skipped {st['cycle_sweeps']}")
    finally:
        ctx.close()
