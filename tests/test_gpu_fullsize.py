"""Parity at the benchmark's full sizes.

* The 1,000-node planted partition and R-MAT scale 20 (unit weights, seed 2),
  PLM and PLMR: the whole run is compared with the oracle's stored result
  (tests/golden/oracle_runs.json, written by tests/golden/make_golden.py from
  the oracle alone): SHA-256 of the canonical labels, Q bit for bit, and the
  per-level trace.
* R-MAT scale 26 (weights 1..100, seed 3), in the launch configuration the
  benchmark times (default options): sampled outputs the oracle computes one by
  one -- the decisions of sampled nodes of several colour classes after real
  sweeps -- and properties that hold at any size: volumes sum to S and match
  the communities, the colouring is proper on the sampled rows, the run's Q
  equals plm_modularity of its labels, labels are canonical.
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
import oracle

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_golden(P, name, g, refine=False):
    gold = json.load(open(GOLDEN))[name + ("_plmr" if refine else "")]
    with P.Context(g.off, g.col, g.w, refine=int(refine)) as ctx:
        labels, q, lv = ctx.run()
        st = ctx.stats()
    assert hashlib.sha256(labels.astype(np.int32).tobytes()).hexdigest() == gold["labels_sha256"]
    assert q == float.fromhex(gold["q_hex"]) and lv == gold["levels"]
    keys = ("n", "nnz", "colours", "sweeps", "communities", "moves") + (("ref_sweeps", "ref_moves") if refine else ())
    for k in keys:
        assert st[k] == gold["trace"][k], k


def test_planted_partition_golden(P):
    _check_golden(P, "planted_partition_1000_seed1", graphgen.planted_partition_1000(seed=1))


@pytest.mark.timeout(300)
def test_rmat20_golden(P):
    _say("rmat20 golden")
    _check_golden(P, "rmat20_seed2_unit", graphgen.rmat20(seed=2))


def test_planted_partition_golden_plmr(P):
    _check_golden(P, "planted_partition_1000_seed1", graphgen.planted_partition_1000(seed=1), refine=True)


@pytest.mark.timeout(300)
def test_rmat20_golden_plmr(P):
    _say("rmat20 golden plmr")
    _check_golden(P, "rmat20_seed2_unit", graphgen.rmat20(seed=2), refine=True)


def test_device_generator_matches_host(P):
    for s, w in [(12, True), (16, False)]:
        g = graphgen.rmat(s, 16, seed=7, weighted=w)
        dg = graphgen.rmat_gpu(s, 16, seed=7, weighted=w)
        try:
            h = dg.to_host()
        finally:
            dg.free()
        assert np.array_equal(h.off, g.off) and np.array_equal(h.col, g.col)
        assert (h.w is None) == (g.w is None) and (g.w is None or np.array_equal(h.w, g.w))


def _rows(dg, off, nodes):
    """CSR of the given rows (node ids kept), other rows empty."""
    lib = graphgen._gpu_lib()
    n = dg.n
    deg = np.diff(off)
    soff = np.zeros(n + 1, np.int64)
    soff[nodes.astype(np.int64) + 1] = deg[nodes]
    soff = np.cumsum(soff)
    col = np.zeros(int(soff[-1]), np.int32)
    w = np.zeros(int(soff[-1]), np.int32)
    for u in nodes:
        a, b = int(off[u]), int(off[u + 1])
        o = int(soff[u])
        if b > a:
            lib.ggpu_copy_to_host(col[o:].ctypes.data, ctypes.c_void_p(dg.col_ptr + 4 * a), 4 * (b - a))
            lib.ggpu_copy_to_host(w[o:].ctypes.data, ctypes.c_void_p(dg.w_ptr + 4 * a), 4 * (b - a))
    return soff, col, w


@pytest.mark.timeout(600)
def test_rmat26_sampled_parity_and_invariants(P):
    import torch
    _say("rmat26 generate")
    dg = graphgen.rmat_gpu(26, 16, seed=3, weighted=True)
    try:
        n = dg.n
        off = np.zeros(n + 1, np.int64)
        graphgen._gpu_lib().ggpu_copy_to_host(off.ctypes.data, ctypes.c_void_p(dg.off_ptr), off.nbytes)
        ctx = P.Context(dg.off_ptr, dg.col_ptr, dg.w_ptr, mem_kind=P.PLM_MEM_DEVICE, n=n, nnz=dg.nnz)
        li = ctx.level_info()
        S = li.S
        z, vol, colour = ctx.state()
        assert np.array_equal(z, np.arange(n)) and int(vol.sum()) == S
        rng = np.random.default_rng(26)
        # colouring proper on the rows of 2000 random non-isolated nodes
        deg = np.diff(off)
        probe = np.sort(rng.choice(np.nonzero(deg > 0)[0], 2000, replace=False)).astype(np.int32)
        soff, scol, sw = _rows(dg, off, probe)
        for u in probe:
            nb = scol[soff[u]:soff[u + 1]]
            nb = nb[nb != u]
            assert not np.any(colour[nb] == colour[u])
        _say("rmat26 sweeps")
        for _ in range(2):
            ctx.move_sweep()
        z, volC, colour = ctx.state()
        C = int(colour.max()) + 1
        assert int(volC.sum()) == S
        vc = np.zeros(n, np.int64)
        np.add.at(vc, z, vol)
        assert np.array_equal(vc, volC)
        for c in (0, C // 2, C - 1):
            members = np.nonzero(colour == c)[0]
            sample = members if len(members) <= 1500 else rng.choice(members, 1500, replace=False)
            sample = np.sort(sample).astype(np.int32)
            soff, scol, sw = _rows(dg, off, sample)
            w2 = oracle.double_diagonal(soff, scol, sw)
            want = oracle.decide_many(sample, soff, scol, w2, z, volC, vol, S)
            _say(f"rmat26 class {c}: {len(members)} members, {len(sample)} sampled, {int(soff[-1])} entries")
            ctx.move_class(c)
            z2, volC2, _ = ctx.state()
            expect = np.where(want >= 0, want, z[sample])
            assert np.array_equal(z2[sample], expect), f"class {c}"
            z, volC = z2, volC2
        _say("rmat26 full run")
        lab = torch.empty(n, dtype=torch.int32, device="cuda:0")
        _, q, lv = ctx.run(lab)
        labels = lab.cpu().numpy()
        assert ctx.modularity(lab) == q
        uniq, idx = np.unique(labels, return_index=True)
        assert np.array_equal(uniq, np.arange(len(uniq)))            # dense ids
        assert np.all(np.diff(idx) > 0)                              # numbered by first occurrence
        st = ctx.stats()
        assert st["levels"] == lv and st["communities"][-1] == len(uniq)
        ctx.close()
    finally:
        dg.free()
