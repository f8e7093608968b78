"""Parity with the oracle of the sweep layout (plm_options.layout).

With the layout, the move sweeps read neighbour communities and community
volumes through copies ordered by descending degree, and rank, tie-break and
report candidates by their original ids; results must be the oracle's element
by element.  By default only graphs of more than 2^27 entries take it (the
R-MAT 26 tests cover that size); here layout = 1 forces it on small graphs:
per class step and per sweep in every bin setting, on the partitioned hub path,
with forced 128-bit gains, gamma != 1, PLMR, the settled-node skip, label
propagation and the ensemble; layout = -1 keeps the graph's own ids.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

from .test_gpu_parity import MID_BINS, SMALL_BINS, full_run, stepwise
from .test_gpu_plp import epp_run, plp_run

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
HUBS = dict(bin_lane=4, bin_wave=8, bin_block=16, hub_row_max=64)


@pytest.mark.parametrize("seed", range(2))
@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_stepwise_classes_layout(P, seed, bins):
    _say("layout stepwise classes", seed, bins)
    g = graphgen.random_graph(150, 0.08, seed=60 + seed, weighted=True, loops=0.1)
    stepwise(P, g, seed=seed, layout=1, **bins)


@pytest.mark.parametrize("bins", BINS + [HUBS], ids=BIN_IDS + ["hubs"])
def test_stepwise_sweeps_rmat_layout(P, bins):
    _say("layout stepwise rmat 12", bins)
    stepwise(P, graphgen.rmat(12, 16, seed=9, weighted=True), seed=2, per_class=False, layout=1, **bins)


def test_stepwise_partitioned_hubs_per_class_layout(P):
    g = graphgen.rmat(12, 16, seed=11, weighted=True)
    stepwise(P, g, seed=6, per_class=True, max_sweeps=4, max_levels=2, layout=1, **HUBS)


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
def test_stepwise_int128_layout(P, bins):
    g = graphgen.random_graph(140, 0.1, seed=78, weighted=True, loops=0.2)
    stepwise(P, g, seed=3, layout=1, int_mode=P.PLM_INT_128, **bins)


@pytest.mark.parametrize("layout", [1, -1, 0])
@pytest.mark.parametrize("bins", BINS + [HUBS], ids=BIN_IDS + ["hubs"])
def test_full_run_rmat14_layout(P, layout, bins):
    _say("layout full rmat 14", layout, bins)
    full_run(P, graphgen.rmat(14, 16, seed=3, weighted=True), seed=0, layout=layout, **bins)


@pytest.mark.parametrize("gamma", [(1, 2), (3, 2), (0, 1)], ids=["1_2", "3_2", "0_1"])
def test_full_run_gamma_layout(P, gamma):
    g = graphgen.rmat(12, 16, seed=13, weighted=True)
    for bins in BINS:
        full_run(P, g, seed=1, gamma=gamma, layout=1, **bins)


@pytest.mark.parametrize("settle", [1, 0])
def test_full_run_settle_layout(P, settle):
    g = graphgen.rmat(13, 16, seed=17, weighted=True)
    for bins in BINS + [HUBS]:
        full_run(P, g, seed=2, settle=settle, layout=1, **bins)


@pytest.mark.parametrize("bins", BINS + [HUBS], ids=BIN_IDS + ["hubs"])
def test_plmr_layout(P, bins):
    full_run(P, graphgen.rmat(13, 16, seed=21, weighted=True), seed=2, refine=True, layout=1, **bins)
    full_run(P, graphgen.planted_partition_1000(), refine=True, layout=1, **bins)


def test_plmr_hub_path_int128_layout(P):
    full_run(P, graphgen.rmat(12, 16, seed=23, weighted=True), seed=4, refine=True, layout=1,
             int_mode=P.PLM_INT_128, **HUBS)


@pytest.mark.parametrize("bins", BINS + [HUBS], ids=BIN_IDS + ["hubs"])
def test_plp_layout(P, bins):
    g = graphgen.rmat(12, 16, seed=5, weighted=True)
    plp_run(P, g, seed=1, layout=1, **bins)
    with P.Context(g.off, g.col, g.w, layout=1, **bins) as ctx:
        ctx.plp(64)
        lab, q, lv = ctx.run()                         # a PLM run after PLP on the same context
    r = oracle.run(g.off, g.col, g.w)
    assert np.array_equal(lab, r.labels) and q == r.q and lv == r.levels


@pytest.mark.parametrize("bins", [{}, HUBS], ids=["default", "hubs"])
def test_epp_layout(P, bins):
    epp_run(P, graphgen.rmat(12, 16, seed=7, weighted=True), b=3, seed=2, layout=1, **bins)
    epp_run(P, graphgen.planted_partition_1000(seed=3), b=4, layout=1, **bins)


def test_layout_option_errors(P):
    g = graphgen.rmat(8, 8, seed=1, weighted=False)
    for bad in (-2, 2):
        with pytest.raises(P.PLMError):
            P.Context(g.off, g.col, None, layout=bad)
