"""Parity of the partitioned hub path's rarely reached branches with the oracle.

A row longer than the one-workgroup hub limit is aggregated by chunk
workgroups that hash their merged (community, weight) pairs into buckets, and
by one bucket workgroup per bucket that flattens the bucket's segments of all
chunks, a tile of chunks at a time, into an LDS table.  Two branches exist only
to keep every input exact and are not reached by ordinary graphs:

* a bucket holding more distinct communities than one pass takes is redone in
  2, 4, ... sub-partition passes;
* a hub of more chunks than one tile loops over several tiles.

Both are reached here at the compiled limits (a star whose leaf ids all hash
into bucket 0; a star of more than 512 chunks) and, through the test knobs of
plm_options (hub_row_max, agg_max_keys, agg_tile), on small graphs in every
mode that uses the path: PLM, PLMR, gamma, forced 128-bit gains and label
propagation.  Results are compared with the oracle element by element.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

from .test_gpu_parity import full_run, stepwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _csr(n, rows, cols, ws):
    """Symmetric CSR from undirected (row < col) pairs with weights."""
    r = np.concatenate([rows, cols]).astype(np.int64)
    c = np.concatenate([cols, rows]).astype(np.int64)
    w = np.concatenate([ws, ws]).astype(np.int32)
    order = np.lexsort((c, r))
    r, c, w = r[order], c[order], w[order]
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, r + 1, 1)
    return graphgen.Graph(np.cumsum(off), c.astype(np.int32), w)


def _bucket(x, pbits):
    """Bucket of community x among 2^pbits (the multiplicative hash of the
    chunk workgroups, top pbits bits of x * 2654435769 mod 2^32)."""
    return ((np.asarray(x, np.uint64) * np.uint64(2654435769)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - pbits)


def _paired_star(leaves):
    """Hub 0 joined (weight 1) to the given leaf ids, consecutive leaves paired
    by weight-100 edges: whenever the hub decides, its candidates are the
    leaves' singleton or pair communities, all named by leaf ids."""
    leaves = np.sort(np.asarray(leaves, np.int64))
    n = int(leaves[-1]) + 1
    hub_r = np.zeros(len(leaves), np.int64)
    pa, pb = leaves[0:len(leaves) - 1:2], leaves[1:len(leaves):2]
    rows = np.concatenate([hub_r, pa])
    cols = np.concatenate([leaves, pb])
    ws = np.concatenate([np.ones(len(leaves), np.int64), np.full(len(pa), 100, np.int64)])
    return _csr(n, rows, cols, ws)


def test_agg_subpartition_passes_at_compiled_limits(P):
    """13,000 leaves (16 buckets of ~1024 expected) whose ids all hash into
    bucket 0: that bucket holds far more than 1,536 communities, so its bucket
    workgroup takes the sub-partition passes."""
    d = 13000
    cand = np.arange(1, 16 * d + 64000, dtype=np.int64)
    leaves = cand[_bucket(cand, 4) == 0][:d]
    assert len(leaves) == d
    g = _paired_star(leaves)
    _say("agg sub-partition star", g.n, g.nnz)
    full_run(P, g)
    stepwise(P, g, per_class=True, max_levels=2)


def test_agg_multi_tile_at_compiled_limits(P):
    """A hub of 600,000 entries: 586 chunks of 1024, more than the 512 a
    bucket workgroup flattens at once."""
    leaves = np.arange(1, 600001, dtype=np.int64)
    g = _paired_star(leaves)
    _say("agg multi-tile star", g.n, g.nnz)
    full_run(P, g)
    full_run(P, g, refine=True)


# every hub-bin row (longer than 3 entries) partitioned once longer than 4,
# buckets split after 32 communities, tiles of 1-3 chunks
KNOBS = [dict(bin_lane=1, bin_wave=2, bin_block=3, hub_row_max=4, agg_max_keys=32, agg_tile=1),
         dict(bin_lane=4, bin_wave=16, bin_block=64, hub_row_max=64, agg_max_keys=32, agg_tile=3)]
KNOB_IDS = ["tiny", "small"]


@pytest.mark.parametrize("knobs", KNOBS, ids=KNOB_IDS)
def test_knobs_stepwise_rmat(P, knobs):
    _say("hub knobs stepwise", knobs)
    stepwise(P, graphgen.rmat(12, 16, seed=31, weighted=True), seed=2, per_class=False, **knobs)


@pytest.mark.parametrize("knobs", KNOBS, ids=KNOB_IDS)
def test_knobs_stepwise_per_class_random(P, knobs):
    _say("hub knobs per class", knobs)
    g = graphgen.random_graph(150, 0.15, seed=8, weighted=True, loops=0.1)
    stepwise(P, g, seed=1, **knobs)


@pytest.mark.parametrize("knobs", KNOBS, ids=KNOB_IDS)
def test_knobs_full_runs(P, knobs):
    _say("hub knobs full runs", knobs)
    g = graphgen.rmat(13, 16, seed=32, weighted=True)
    full_run(P, g, **knobs)
    full_run(P, g, refine=True, **knobs)
    full_run(P, g, gamma=(3, 2), **knobs)
    full_run(P, g, int_mode=P.PLM_INT_128, **knobs)
    full_run(P, graphgen.rmat(12, 16, seed=33, weighted=False), seed=5, **knobs)


@pytest.mark.parametrize("knobs", KNOBS, ids=KNOB_IDS)
def test_knobs_label_propagation(P, knobs):
    _say("hub knobs plp", knobs)
    g = graphgen.rmat(13, 16, seed=34, weighted=True)
    want = oracle.plp(g.off, g.col, g.w, seed=3)
    with P.Context(g.off, g.col, g.w, colour_seed=3, **knobs) as ctx:
        labels, q, it, upd = ctx.plp()
    assert np.array_equal(labels, want.labels) and q == want.q
    assert it == want.iterations and upd == want.updates


def test_knobs_star_subpartitions(P):
    """The 20,000-leaf star with a ring among the leaves, split into
    sub-partition passes and single-chunk tiles."""
    n = 20001
    rows = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n - 1)])
    cols = np.concatenate([np.arange(1, n), np.arange(2, n)])
    rng = np.random.default_rng(1)
    g = _csr(n, rows, cols, rng.integers(1, 50, len(rows)))
    _say("hub knobs star")
    full_run(P, g, agg_max_keys=32, agg_tile=1)
    full_run(P, g, agg_max_keys=64, agg_tile=7, refine=True)
