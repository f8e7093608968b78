"""Parity of label propagation (plm_plp, Algorithm 1) and of the ensemble
EPP(b, PLP, PLMR) (plm_epp, Algorithm 5) on the HIP path with the oracle:
labels, iterations and label changes per iteration, core groups and PLMR
levels bit for bit, modularity exactly (both sides divide the same two
integers)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

SMALL_BINS = dict(bin_lane=1, bin_wave=2, bin_block=3)   # every decide path on small graphs
MID_BINS = dict(bin_lane=4, bin_wave=16, bin_block=64)
BINS = [{}, SMALL_BINS, MID_BINS]
BIN_IDS = ["default", "small", "mid"]


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P  # fails loudly without the built library
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def plp_run(P, g, seed=0, max_iters=64, **opts):
    r = oracle.plp(g.off, g.col, g.w, seed=seed, max_iters=max_iters)
    with P.Context(g.off, g.col, g.w, colour_seed=seed, **opts) as ctx:
        labels, q, it, upd = ctx.plp(max_iters)
        st = ctx.stats()
    assert it == r.iterations and upd == r.updates
    assert np.array_equal(labels, r.labels)
    assert q == r.q
    assert st["lp_runs"] == 1 and st["lp_iterations"] == it and st["lp_updates"] == sum(upd)
    return r


def epp_run(P, g, b=4, seed=0, plp_iters=64, max_sweeps=32, max_levels=0, gamma=(1, 1), **opts):
    r = oracle.epp(g.off, g.col, g.w, b=b, seed=seed, plp_iters=plp_iters, max_sweeps=max_sweeps,
                   max_levels=max_levels, gamma=gamma)
    with P.Context(g.off, g.col, g.w, colour_seed=seed, max_sweeps=max_sweeps, max_levels=max_levels,
                   gamma_num=gamma[0], gamma_den=gamma[1], **opts) as ctx:
        labels, q, lv, cores = ctx.epp(b, plp_iters)
        st = ctx.stats()
    assert cores == r.cores and lv == r.levels
    assert np.array_equal(labels, r.labels)
    assert q == r.q
    # level 0 is the input; the PLMR trace of the oracle starts at level 1
    assert st["communities"][0] == r.cores and st["lp_runs"] == b
    assert st["n"][1:] == r.run.n and st["communities"][1:] == r.run.communities
    assert st["sweeps"][1:] == r.run.sweeps and st["ref_sweeps"][1:] == r.run.ref_sweeps
    return r


# ------------------------------------------------------------------ PLP
def test_plp_planted_partition(P):
    _say("plp planted partition")
    r = plp_run(P, graphgen.planted_partition_1000(seed=1))
    assert r.q > 0.5


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
@pytest.mark.parametrize("scale,weighted", [(10, False), (12, True), (14, False)])
def test_plp_rmat(P, scale, weighted, bins):
    _say(f"plp rmat {scale} weighted={weighted} bins={bins}")
    plp_run(P, graphgen.rmat(scale, 16, seed=40 + scale, weighted=weighted), seed=scale, **bins)


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
@pytest.mark.parametrize("seed", range(4))
def test_plp_random_with_loops(P, seed, bins):
    _say(f"plp random seed={seed} bins={bins}")
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(50, 600))
    g = graphgen.random_graph(n, float(rng.uniform(0.005, 0.05)), seed=310 + seed, weighted=seed % 2 == 0,
                              loops=0.2)
    plp_run(P, g, seed=seed, **bins)


def test_plp_sbm(P):
    _say("plp sbm")
    plp_run(P, graphgen.sbm(20000, 40, 0.01, 0.0002, seed=9), seed=3)


@pytest.mark.parametrize("iters", [1, 2, 5])
def test_plp_iteration_cap(P, iters):
    _say(f"plp cap {iters}")
    plp_run(P, graphgen.rmat(12, 16, seed=7, weighted=False), max_iters=iters)


def test_plp_forced_int128(P):
    _say("plp int128")
    g = graphgen.rmat(12, 16, seed=8, weighted=True)
    plp_run(P, g, int_mode=P.PLM_INT_128)
    plp_run(P, g, int_mode=P.PLM_INT_128, **SMALL_BINS)


def test_plp_heavy_weights_take_wide_scores(P):
    """vol(u) >= 2^31: (w << 32) no longer fits 64 bits, the node is scored in
    128 bits (lane path) or goes to the partitioned hub path."""
    _say("plp heavy weights")
    big = 2**31 - 1
    rng = np.random.default_rng(5)
    n = 400
    edges = sorted({tuple(sorted(map(int, rng.choice(n, 2, replace=False)))) for _ in range(1600)})
    w = rng.integers(1, 20, len(edges))
    w[rng.random(len(edges)) < 0.2] = big
    g = graphgen.from_edges(n, edges, w, loops={3: big, 7: 5})
    plp_run(P, g)
    plp_run(P, g, **SMALL_BINS)


def test_plp_hub_multi_workgroup(P):
    """A star of 20000 weighted leaves plus a path through the leaves: the
    centre's row takes the partitioned hub path."""
    _say("plp hub star")
    n = 20001
    edges = [(0, i) for i in range(1, n)] + [(i, i + 1) for i in range(1, n - 1)]
    rng = np.random.default_rng(2)
    g = graphgen.from_edges(n, edges, rng.integers(1, 50, len(edges)))
    plp_run(P, g)
    plp_run(P, g, seed=4, bin_wave=32, bin_block=64)


def test_plp_structures_and_degenerate(P):
    _say("plp structures")
    r = plp_run(P, graphgen.ring_of_cliques(12, 6))
    assert len(set(r.labels.tolist())) == 12
    plp_run(P, graphgen.disjoint_cliques(10, 8))
    plp_run(P, graphgen.disjoint_edges(7))
    plp_run(P, graphgen.from_edges(5, [(1, 2)], loops={0: 3}))
    plp_run(P, graphgen.from_edges(4, []))
    e = graphgen.from_edges(0, [])
    with P.Context(e.off, e.col, e.w) as ctx:
        labels, q, it, upd = ctx.plp()
        assert labels.shape == (0,) and it == 0 and q == 0.0


def test_plp_then_run_is_unchanged(P):
    """plm_plp leaves the context at level 0: a following plm_run gives the
    oracle's PLM result."""
    _say("plp then run")
    g = graphgen.rmat(11, 16, seed=12, weighted=True)
    r = oracle.run(g.off, g.col, g.w)
    with P.Context(g.off, g.col, g.w) as ctx:
        ctx.plp()
        labels, q, lv = ctx.run()
        ctx.plp(3)
        labels2, q2, _ = ctx.run()
    assert np.array_equal(labels, r.labels) and q == r.q and lv == r.levels
    assert np.array_equal(labels2, r.labels) and q2 == r.q


def test_plp_device_inputs(P):
    import torch
    _say("plp device inputs")
    g = graphgen.rmat(11, 16, seed=13, weighted=False)
    r = oracle.plp(g.off, g.col, g.w, seed=2)
    d = torch.device("cuda:0")
    off, col = torch.from_numpy(g.off).to(d), torch.from_numpy(g.col).to(d)
    lab = torch.empty(g.n, dtype=torch.int32, device=d)
    with P.Context(off, col, None, n=g.n, nnz=g.nnz, colour_seed=2) as ctx:
        _, q, it, upd = ctx.plp(64, lab)
    assert np.array_equal(lab.cpu().numpy(), r.labels) and q == r.q and upd == r.updates


def test_plp_epp_argument_errors(P):
    g = graphgen.disjoint_cliques(2, 3)
    with P.Context(g.off, g.col, g.w) as ctx:
        for it in (0, 65):
            with pytest.raises(P.PLMError) as ei:
                ctx.plp(it)
            assert ei.value.status == P.PLM_E_ARG
        for b, it in ((0, 8), (1025, 8), (2, 0), (2, 65)):
            with pytest.raises(P.PLMError) as ei:
                ctx.epp(b, it)
            assert ei.value.status == P.PLM_E_ARG
    node_base, off, col, w = P.pack_batch([g, g])
    with P.BatchContext(node_base, off, col, w) as bc:
        for call in (lambda: P.plm_plp(bc._c, 8, None, None, None, None),
                     lambda: P.plm_epp(bc._c, 2, 8, None, None, None, None)):
            assert call() == P.PLM_E_STATE


# ------------------------------------------------------------------ EPP
@pytest.mark.parametrize("b", [1, 2, 4, 8])
def test_epp_planted_partition(P, b):
    _say(f"epp planted partition b={b}")
    r = epp_run(P, graphgen.planted_partition_1000(seed=2), b=b, seed=5)
    assert r.q > 0.55


@pytest.mark.parametrize("bins", BINS, ids=BIN_IDS)
@pytest.mark.parametrize("scale,weighted", [(10, True), (13, False)])
def test_epp_rmat(P, scale, weighted, bins):
    _say(f"epp rmat {scale} bins={bins}")
    epp_run(P, graphgen.rmat(scale, 16, seed=60 + scale, weighted=weighted), b=4, seed=scale, **bins)


@pytest.mark.parametrize("seed", range(3))
def test_epp_random_caps_gamma(P, seed):
    _say(f"epp random seed={seed}")
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(100, 900))
    g = graphgen.random_graph(n, float(rng.uniform(0.004, 0.03)), seed=510 + seed, weighted=True, loops=0.1)
    epp_run(P, g, b=3, seed=seed)
    epp_run(P, g, b=2, seed=seed, plp_iters=2, max_sweeps=3, max_levels=2)
    epp_run(P, g, b=3, seed=seed, gamma=[(1, 2), (3, 2), (7, 3)][seed])


def test_epp_sbm_and_structures(P):
    _say("epp sbm")
    epp_run(P, graphgen.sbm(20000, 40, 0.01, 0.0002, seed=10), b=4, seed=1)
    epp_run(P, graphgen.ring_of_cliques(10, 5), b=4)
    epp_run(P, graphgen.disjoint_cliques(4, 6), b=2)
    epp_run(P, graphgen.from_edges(4, []), b=2)
    e = graphgen.from_edges(0, [])
    with P.Context(e.off, e.col, e.w) as ctx:
        labels, q, lv, cores = ctx.epp(3)
        assert labels.shape == (0,) and cores == 0 and lv == 1


def test_epp_forced_int128_and_hub(P):
    _say("epp int128 + hub")
    epp_run(P, graphgen.rmat(12, 16, seed=14, weighted=True), b=3, int_mode=P.PLM_INT_128)
    n = 20001
    edges = [(0, i) for i in range(1, n)] + [(i, i + 1) for i in range(1, n - 1)]
    g = graphgen.from_edges(n, edges, np.random.default_rng(3).integers(1, 50, len(edges)))
    epp_run(P, g, b=2)


def test_epp_then_run_is_unchanged(P):
    _say("epp then run")
    g = graphgen.rmat(11, 16, seed=15, weighted=True)
    r = oracle.run(g.off, g.col, g.w, refine=True)
    with P.Context(g.off, g.col, g.w, refine=1) as ctx:
        ctx.epp(3)
        labels, q, lv = ctx.run()
    assert np.array_equal(labels, r.labels) and q == r.q and lv == r.levels
