"""Parity with the oracle of packed contraction items (plm_options.pack_bits).

At a level with 32-bit or unit weights whose largest entry (twice that for a
self-loop) fits the bits that the two coarse ids leave free in 64, the
contraction sorts each (coarse row, coarse column) key together with its weight
as one 64-bit word; a merged weight too large for those bits is split over
several words of the same key and summed again after the sort.  On small graphs
the ids leave tens of bits free and nothing splits, so pack_bits = k caps the
weight field at k bits: unit weights with k = 2 (field maximum 3: a self-loop's
2 fits, a merge of two entries or more splits), weights up to 100 with k = 8
(maximum 255).  Weights too large for the field fall back to key-weight pairs
(k = 2 on weighted graphs), as does k = -1.  Every coarse CSR must be the
oracle's element by element (stepwise), and so must full runs, PLMR and
batches.  R-MAT 26 (the golden test) packs with the default field of 12 bits
at level 0 and splits there too.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen

from .test_gpu_batch import _mix, batch_vs_oracle
from .test_gpu_parity import MID_BINS, SMALL_BINS, full_run, stepwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("k", [2, 3, 0, -1])
def test_stepwise_unit_weights(P, k):
    _say("pack stepwise planted partition", k)
    stepwise(P, graphgen.planted_partition_1000(), seed=1, per_class=False, pack_bits=k)


@pytest.mark.parametrize("k", [2, 8, 9, 0, -1])
def test_stepwise_weighted_rmat(P, k):
    _say("pack stepwise rmat 12 weighted", k)
    stepwise(P, graphgen.rmat(12, 16, seed=9, weighted=True), seed=2, per_class=False, pack_bits=k)


@pytest.mark.parametrize("seed", range(3))
def test_stepwise_loops_per_class(P, seed):
    _say("pack stepwise random with loops", seed)
    g = graphgen.random_graph(300, 0.05, seed=70 + seed, weighted=bool(seed % 2), loops=0.3)
    stepwise(P, g, seed=seed, pack_bits=8 if seed % 2 else 2, **(SMALL_BINS if seed == 2 else {}))


@pytest.mark.parametrize("bins", [{}, MID_BINS], ids=["default", "mid"])
def test_full_run_rmat14(P, bins):
    _say("pack full rmat 14", bins)
    full_run(P, graphgen.rmat(14, 16, seed=14, weighted=True), seed=14, pack_bits=8, **bins)
    full_run(P, graphgen.rmat(14, 16, seed=15, weighted=False), seed=15, pack_bits=2, **bins)


def test_plmr_and_gamma(P):
    _say("pack plmr, gamma")
    g = graphgen.rmat(12, 16, seed=5, weighted=False)
    full_run(P, g, seed=3, refine=True, pack_bits=2)
    full_run(P, g, seed=3, gamma=(2, 1), pack_bits=2)


@pytest.mark.parametrize("k", [2, 8])
def test_batch(P, k):
    _say("pack batch", k)
    batch_vs_oracle(P, _mix(), seed=2, pack_bits=k)


def test_same_labels_packed_or_pairs(P):
    g = graphgen.rmat(13, 16, seed=21, weighted=True)
    out = []
    for k in (0, 8, -1):
        with P.Context(g.off, g.col, g.w, pack_bits=k) as ctx:
            labels, q, lv = ctx.run()
            out.append((labels.copy(), q, lv))
    for labels, q, lv in out[1:]:
        assert np.array_equal(labels, out[0][0]) and q == out[0][1] and lv == out[0][2]


@pytest.mark.parametrize("k", [1, 63, -2])
def test_pack_bits_out_of_range(P, k):
    g = graphgen.planted_partition_1000()
    with pytest.raises(P.PLMError):
        P.Context(g.off, g.col, pack_bits=k)
