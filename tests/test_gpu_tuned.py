"""The tuned degree bins (paper_1304_4453_amd/tuned_bins.txt, written by
paper_1304_4453_amd/tune.py on the GPU) against the oracle: contexts that leave
the bins at 0 take the table's row for their kind and size (checked through
plm_get_options), and every row's setting gives the oracle's partitions: the
batch row on 64 SBM graphs of the batched workload's recipe, the single-graph
rows on R-MAT and random weighted graphs, each setting also forced explicitly
on a small graph so that rows for large graphs are exercised too.  (R-MAT 26
itself runs with the large-graph row in the stored-oracle test.)"""
from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle

from .test_gpu_parity import full_run

pytestmark = pytest.mark.gpu
TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1304_4453_amd",
                     "tuned_bins.txt")


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _rows():
    rows = []
    for line in open(TABLE):
        if line.strip() and not line.startswith("#"):
            kind, mx, a, b, c, h = line.split()
            rows.append((kind, int(mx), dict(bin_lane=int(a), bin_wave=int(b), bin_block=int(c), hub_row_max=int(h))))
    return rows


def _bins(o):
    return dict(bin_lane=o.bin_lane, bin_wave=o.bin_wave, bin_block=o.bin_block, hub_row_max=o.hub_row_max)


def test_table_is_the_one_in_use(P):
    assert os.path.exists(TABLE)
    assert os.path.realpath(P.plm_tuned_table().decode()) == os.path.realpath(TABLE)
    assert len(_rows()) >= 2


def test_single_graph_row_applies_and_matches_oracle(P):
    g = graphgen.rmat(14, 16, seed=3, weighted=True)
    want = next(r for k, mx, r in _rows() if k == "single" and (mx == 0 or g.nnz <= mx))
    with P.Context(g.off, g.col, g.w) as ctx:
        assert _bins(ctx.options()) == want
    full_run(P, g)                                    # options left at 0: the tuned row
    full_run(P, g, refine=True)


@pytest.mark.parametrize("row", range(3))
def test_every_row_setting_matches_oracle(P, row):
    rows = _rows()
    if row >= len(rows):
        pytest.skip("table has fewer rows")
    _, _, bins = rows[row]
    for seed in range(2):
        full_run(P, graphgen.rmat(13, 16, seed=30 + seed, weighted=True), seed=seed, **bins)
        full_run(P, graphgen.random_graph(300, 0.05, seed=50 + seed, weighted=True, loops=0.1), seed=seed, **bins)


def test_batch_row_applies_and_matches_oracle(P):
    graphs = graphgen.sbm_batch(4, 64)
    nb, off, col, w = P.pack_batch(graphs)
    want = next(r for k, mx, r in _rows() if k == "batch" and (mx == 0 or len(col) <= mx))
    with P.BatchContext(nb, off, col, w) as ctx:
        assert _bins(ctx.options()) == want
        labels, q, lv = ctx.run_batch()
    for i, g in enumerate(graphs):
        r = oracle.run(g.off, g.col, g.w)
        a, b = int(nb[i]), int(nb[i + 1])
        assert np.array_equal(labels[a:b], r.labels) and q[i] == r.q and lv[i] == r.levels, i
