"""Batched runs (plm_batch_create / plm_batch_run): each graph of a batch must
get exactly the result of a separate run on it -- the oracle's canonical
labels, modularity (bit for bit) and number of levels -- whatever the other
graphs are, including empty graphs, edgeless graphs, graphs that stop after
one level, and graphs reaching the hub bins."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _empty():
    return graphgen.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), None)


def _mix():
    return [
        graphgen.planted_partition_1000(seed=3),
        _empty(),
        graphgen.disjoint_cliques(2, 5),
        graphgen.from_edges(5, []),                      # edgeless
        graphgen.ring_of_cliques(6, 4),
        graphgen.random_graph(120, 0.06, seed=3, weighted=True, loops=0.2),
        graphgen.from_edges(1, []),                      # single node
        graphgen.disjoint_edges(4),
        graphgen.sbm(300, 3, 0.2, 0.01, seed=5),
        graphgen.rmat(10, 16, seed=4, weighted=True),
        _empty(),
    ]


def batch_vs_oracle(P, graphs, seed=0, max_sweeps=32, max_levels=0, **opts):
    nb, off, col, w = P.pack_batch(graphs)
    with P.BatchContext(nb, off, col, w, colour_seed=seed, max_sweeps=max_sweeps, max_levels=max_levels,
                        **opts) as ctx:
        labels, q, lv = ctx.run_batch()
    for i, g in enumerate(graphs):
        r = oracle.run(g.off, g.col, g.w, max_sweeps=max_sweeps, max_levels=max_levels, seed=seed)
        a, b = int(nb[i]), int(nb[i + 1])
        assert np.array_equal(labels[a:b], r.labels[: b - a]), f"graph {i} labels"
        assert q[i] == r.q, f"graph {i}: q {q[i]!r} vs {r.q!r}"
        assert lv[i] == r.levels, f"graph {i}: levels {lv[i]} vs {r.levels}"
    return labels, q, lv


SMALL_BINS = dict(bin_lane=1, bin_wave=2, bin_block=3)
MID_BINS = dict(bin_lane=4, bin_wave=16, bin_block=64)


@pytest.mark.parametrize("bins", [{}, SMALL_BINS, MID_BINS], ids=["default", "small", "mid"])
def test_batch_mix_matches_oracle(P, bins):
    _say("batch mix", bins)
    batch_vs_oracle(P, _mix(), seed=2, **bins)


@pytest.mark.parametrize("max_levels", [1, 2])
def test_batch_level_cap(P, max_levels):
    _say("batch level cap", max_levels)
    batch_vs_oracle(P, _mix(), max_levels=max_levels)


def test_batch_sweep_cap(P):
    _say("batch sweep cap")
    batch_vs_oracle(P, _mix(), max_sweeps=1, seed=5)


def test_batch_forced_int128(P):
    _say("batch int128")
    batch_vs_oracle(P, _mix(), int_mode=P.PLM_INT_128)


def test_batch_sbm_workload(P):
    """64 uneven SBM graphs of 100..3000 nodes, the batched workload's recipe."""
    _say("batch sbm 64")
    graphs = graphgen.sbm_batch(seed=4, count=64, n_lo=100, n_hi=3000)
    batch_vs_oracle(P, graphs)


def test_batch_equals_separate_runs_and_repeats(P):
    _say("batch vs separate runs")
    graphs = _mix()
    nb, off, col, w = P.pack_batch(graphs)
    with P.BatchContext(nb, off, col, w) as ctx:
        l1, q1, v1 = ctx.run_batch()
        l2, q2, v2 = ctx.run_batch()
        st = ctx.stats()
    assert np.array_equal(l1, l2) and np.array_equal(q1, q2) and np.array_equal(v1, v2)
    assert st["levels"] == int(v1.max())
    for i, g in enumerate(graphs):
        if g.n == 0:
            continue
        with P.Context(g.off, g.col, g.w) as c:
            lab, q, lv = c.run()
        a, b = int(nb[i]), int(nb[i + 1])
        assert np.array_equal(l1[a:b], lab) and q1[i] == q and v1[i] == lv, i


def test_batch_single_graph_equals_plain(P):
    _say("batch of one")
    g = graphgen.rmat(12, 16, seed=7, weighted=True)
    with P.BatchContext(np.array([0, g.n]), g.off, g.col, g.w, bin_lane=8, bin_wave=32, bin_block=128) as ctx:
        lb, qb, vb = ctx.run_batch()
    with P.Context(g.off, g.col, g.w, bin_lane=8, bin_wave=32, bin_block=128) as ctx:
        l, q, v = ctx.run()
    assert np.array_equal(lb, l) and qb[0] == q and vb[0] == v


def test_batch_device_inputs(P):
    import torch
    _say("batch device inputs")
    graphs = _mix()
    nb, off, col, w = P.pack_batch(graphs)
    d = torch.device("cuda:0")
    toff, tcol, tw = (torch.from_numpy(x).to(d) for x in (off, col, w))
    lab = torch.full((int(nb[-1]),), -1, dtype=torch.int32, device=d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with P.BatchContext(nb, toff, tcol, tw, stream=s) as ctx:
            _, q, lv = ctx.run_batch(lab)
    s.synchronize()
    with P.BatchContext(nb, off, col, w) as ctx:
        lh, qh, lvh = ctx.run_batch()
    assert np.array_equal(lab.cpu().numpy(), lh) and np.array_equal(q, qh) and np.array_equal(lv, lvh)


def test_batch_errors(P):
    _say("batch errors")
    g = graphgen.disjoint_cliques(2, 3)
    # the two triangles as two graphs is valid; split inside a triangle is not
    with P.BatchContext(np.array([0, 3, 6]), g.off, g.col, g.w) as ctx:
        _, q, _ = ctx.run_batch()
        assert np.all(q == 0.0)          # a lone triangle: one community, Q = 0
        with pytest.raises(P.PLMError) as e:
            ctx.run()
        assert e.value.status == P.PLM_E_STATE
        with pytest.raises(P.PLMError) as e:
            ctx.coarsen()
        assert e.value.status == P.PLM_E_STATE
    with pytest.raises(P.PLMError) as e:
        P.BatchContext(np.array([0, 2, 6]), g.off, g.col, g.w)
    assert e.value.status == P.PLM_E_GRAPH
    with pytest.raises(P.PLMError) as e:
        P.BatchContext(np.array([0, 4, 3, 6]), g.off, g.col, g.w)
    assert e.value.status == P.PLM_E_ARG
    with pytest.raises(P.PLMError) as e:
        P.BatchContext(np.array([0, 3, 6]), g.off, g.col, g.w, schedule=P.PLM_SCHEDULE_SEQUENTIAL)
    assert e.value.status == P.PLM_E_ARG
    with pytest.raises(P.PLMError) as e:
        P.BatchContext(np.array([0, 3, 6]), g.off, g.col, g.w, int_mode=P.PLM_INT_64)
    assert e.value.status == P.PLM_E_ARG
    with P.Context(g.off, g.col, g.w) as ctx:
        assert P.plm_batch_run(ctx._c, None, None, None) == P.PLM_E_STATE
