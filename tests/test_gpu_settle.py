"""Parity with the oracle of the settled-node skip (plm_options.settle).

A node none of whose neighbours moved since it last stayed, and whose margin
(the slack of its best candidate) exceeds vol(u) times the community volume
moved since then, keeps its community without a new scan of its row.  The
skip is exact, so every class step, sweep, level and full run must equal the
oracle's (which decides every node every time) element by element: here with
the skip armed from the first sweep of every move phase (settle = 1), in every
degree bin, with forced 128-bit gains, gamma != 1, PLMR refinement, the
partitioned hub path (small hub_row_max) and the label-propagation runs that
share the kernels; and with the skip off (settle = -1).  A timed run checks
that nodes were actually skipped.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

from .test_gpu_parity import MID_BINS, SMALL_BINS, full_run, stepwise

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BINS = [{}, SMALL_BINS, MID_BINS]
BIN_IDS = ["default", "small", "mid"]


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_stepwise_classes_settle(P, seed, bins):
    _say("settle stepwise classes", seed, bins)
    g = graphgen.random_graph(150, 0.08, seed=40 + seed, weighted=True, loops=0.1)
    stepwise(P, g, seed=seed, settle=1, **bins)


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_stepwise_sweeps_rmat_settle(P, bins):
    _say("settle stepwise rmat 12", bins)
    g = graphgen.rmat(12, 16, seed=9, weighted=True)
    stepwise(P, g, seed=2, per_class=False, settle=1, **bins)


def test_stepwise_sweeps_planted_partition_settle(P):
    stepwise(P, graphgen.planted_partition_1000(), per_class=False, settle=1)


def test_stepwise_default_arming(P):
    """settle = 0 arms after a sweep that moved at most n/16 nodes (n/1024 on coarse levels)."""
    g = graphgen.rmat(13, 16, seed=4, weighted=True)
    stepwise(P, g, seed=1, per_class=False, settle=0, bin_lane=4, bin_wave=32, bin_block=256)


def test_stepwise_partitioned_hubs_settle(P):
    """Rows above 64 entries take the partitioned hub path (chunks, buckets,
    reduce in the apply launch), whose settled hubs skip all three."""
    g = graphgen.rmat(12, 16, seed=11, weighted=True)
    stepwise(P, g, seed=5, per_class=False, settle=1, bin_lane=4, bin_wave=8, bin_block=16, hub_row_max=64)
    stepwise(P, g, seed=6, per_class=True, max_sweeps=4, max_levels=2, settle=1, bin_lane=4, bin_wave=8,
             bin_block=16, hub_row_max=64)


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_stepwise_int128_settle(P, bins):
    g = graphgen.random_graph(140, 0.1, seed=77, weighted=True, loops=0.2)
    stepwise(P, g, seed=3, settle=1, int_mode=P.PLM_INT_128, **bins)


@pytest.mark.parametrize("gamma", [(1, 2), (3, 2), (0, 1), (7, 3)], ids=["1_2", "3_2", "0_1", "7_3"])
def test_full_run_gamma_settle(P, gamma):
    g = graphgen.rmat(12, 16, seed=13, weighted=True)
    for bins in BINS:
        full_run(P, g, seed=1, gamma=gamma, settle=1, **bins)


@pytest.mark.parametrize("settle", [1, -1, 0])
@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_full_run_rmat14_settle(P, settle, bins):
    _say("settle full rmat 14", settle, bins)
    g = graphgen.rmat(14, 16, seed=3, weighted=True)
    full_run(P, g, seed=0, settle=settle, **bins)


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_plmr_settle(P, bins):
    g = graphgen.rmat(13, 16, seed=21, weighted=True)
    full_run(P, g, seed=2, refine=True, settle=1, **bins)
    full_run(P, graphgen.planted_partition_1000(), refine=True, settle=1, **bins)


def test_plmr_hub_path_int128_settle(P):
    g = graphgen.rmat(12, 16, seed=23, weighted=True)
    full_run(P, g, seed=4, refine=True, settle=1, int_mode=P.PLM_INT_128, bin_lane=4, bin_wave=8, bin_block=16,
             hub_row_max=64)


def test_plp_epp_unchanged_by_settle(P):
    """Label propagation shares the decide kernels but never skips."""
    g = graphgen.rmat(12, 16, seed=5, weighted=True)
    ref = oracle.plp(g.off, g.col, g.w)
    with P.Context(g.off, g.col, g.w, settle=1) as ctx:
        lab, q, it, upd = ctx.plp(64)
        assert np.array_equal(lab, ref.labels) and upd == ref.updates
        lab2, q2, lv = ctx.run()                       # a PLM run after PLP on the same context
    r = oracle.run(g.off, g.col, g.w)
    assert np.array_equal(lab2, r.labels) and q2 == r.q


def test_settle_skips_and_counts(P):
    """A timed run reports skipped decisions, and the result is the oracle's."""
    g = graphgen.rmat(14, 16, seed=8, weighted=True)
    r = oracle.run(g.off, g.col, g.w)
    with P.Context(g.off, g.col, g.w, settle=1, timing=1) as ctx:
        labels, q, lv = ctx.run()
        st = ctx.stats()
    assert np.array_equal(labels, r.labels) and q == r.q and lv == r.levels
    assert sum(st["settle_sweeps"]) > 0
    assert sum(st["settled_nodes"]) > 0
    # every bin node is either decided or settled in every executed sweep
    _say("settled", st["settled_nodes"], "decided", st["decided_nodes"])


def test_settle_option_errors(P):
    g = graphgen.rmat(8, 8, seed=1, weighted=False)
    for bad in (-2, 2):
        with pytest.raises(P.PLMError):
            P.Context(g.off, g.col, None, settle=bad)
