"""Pins of the oracle against facts fixed outside it: closed forms, networkx,
brute force, the published SplitMix64 outputs, an exact-fraction sequential
Louvain written from the paper's Delta-mod, and invariants of each step.

CPU only.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from tests import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)
    graphgen.build(force=False)


def _state_after_random_moves(g, rng, moves=0.6):
    """A random partition (via random labels) with consistent volC."""
    n = g.n
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    k = max(1, n // 3)
    zeta = rng.integers(0, k, n).astype(np.int32)
    keep = rng.random(n) > moves
    zeta[keep] = np.arange(n, dtype=np.int32)[keep]
    volC = np.zeros(n, np.int64)
    np.add.at(volC, zeta, vol)
    return w2, vol, S, zeta, volC


def _N(g, w2, labels):
    return oracle.modularity_parts(g.off, g.col, w2, labels)[0]


# ------------------------------------------------------------------ hashing
def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.startswith("0x")]
    gamma = 0x9E3779B97F4A7C15
    for i, v in enumerate(vals):
        assert oracle.splitmix64((i * gamma) & refs.MASK64) == v
        assert refs.splitmix64((i * gamma) & refs.MASK64) == v


def test_priority_order_matches_reference():
    for seed, level in [(0, 0), (7, 3), (2**63 + 5, 1)]:
        assert list(oracle.priority_order(300, seed, level)) == refs.priority_order(300, seed, level)


# ------------------------------------------------------------------ modularity (Equation 3.1)
@pytest.mark.parametrize("k", [3, 5, 8])
def test_two_cliques_half(k):
    g = graphgen.disjoint_cliques(2, k)
    labels = np.repeat(np.arange(2), k).astype(np.int32)
    assert oracle.modularity(g.off, g.col, None, labels) == 0.5


@pytest.mark.parametrize("c,k", [(10, 5), (6, 4), (3, 3), (30, 5)])
def test_ring_of_cliques_closed_form(c, k):
    g = graphgen.ring_of_cliques(c, k)
    labels = np.repeat(np.arange(c), k).astype(np.int32)
    a = k * (k - 1)
    want = float(Fraction(a, a + 2) - Fraction(1, c))
    assert oracle.modularity(g.off, g.col, None, labels) == want
    if (c, k) == (10, 5):
        assert want == 89 / 110


@pytest.mark.parametrize("c", [1, 2, 7, 50])
def test_disjoint_edges(c):
    g = graphgen.disjoint_edges(c)
    labels = np.repeat(np.arange(c), 2).astype(np.int32)
    assert oracle.modularity(g.off, g.col, None, labels) == float(Fraction(c - 1, c))


def test_one_community_and_singletons():
    g = graphgen.random_graph(30, 0.2, seed=3, weighted=True, loops=0.2)
    assert oracle.modularity(g.off, g.col, g.w, np.zeros(30, np.int32)) == 0.0
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    # singletons: only self-loops are intra
    rows = np.repeat(np.arange(30), np.diff(g.off))
    I2 = int(w2[rows == g.col].sum())
    want = Fraction(S * I2 - int((vol.astype(object) ** 2).sum()), S * S)
    assert oracle.modularity(g.off, g.col, g.w, np.arange(30, dtype=np.int32)) == float(want)


@pytest.mark.parametrize("seed", range(12))
def test_modularity_matches_networkx(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 60))
    g = graphgen.random_graph(n, float(rng.uniform(0.05, 0.5)), seed=seed, weighted=True, loops=0.3)
    for _ in range(3):
        labels = rng.integers(0, max(1, n // 4), n).astype(np.int32)
        q = oracle.modularity(g.off, g.col, g.w, labels)
        assert abs(q - refs.nx_modularity(g.off, g.col, g.w, labels)) < 1e-12
        ex = refs.modularity_fraction(n, refs.edges_of(g.off, g.col, g.w), labels)
        assert abs(q - float(ex)) <= 1e-15


# ------------------------------------------------------------------ gain (Delta-mod)
@pytest.mark.parametrize("seed", range(20))
def test_gain_is_half_the_numerator_change_and_best(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 40))
    g = graphgen.random_graph(n, float(rng.uniform(0.1, 0.6)), seed=1000 + seed, weighted=True, loops=0.25)
    w2, vol, S, zeta, volC = _state_after_random_moves(g, rng)
    N0 = _N(g, w2, zeta)
    for u in range(n):
        x, gain = oracle.decide(u, g.off, g.col, w2, zeta, volC, vol, S)
        # brute force every neighbouring community by full recomputation
        cands = sorted({int(zeta[v]) for v in g.col[g.off[u]:g.off[u + 1]] if v != u} - {int(zeta[u])})
        best, bestX = 0, -1
        for X in cands:
            z2 = zeta.copy(); z2[u] = X
            d = _N(g, w2, z2) - N0
            if d > best:
                best, bestX = d, X
        assert x == bestX
        assert 2 * gain == best


def test_gain_ties_go_to_lowest_id():
    # star centre 0 joined to leaves 1..4 with equal weights; leaf 1 sees only 0.
    g = graphgen.from_edges(5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    w2 = oracle.double_diagonal(g.off, g.col, None)
    vol, S = oracle.volumes(g.off, w2)
    zeta = np.arange(5, dtype=np.int32)
    x, gain = oracle.decide(0, g.off, g.col, w2, zeta, vol.copy(), vol, S)
    assert gain > 0 and x == 1


def test_no_move_without_positive_gain():
    g = graphgen.from_edges(2, [(0, 1)], loops={0: 5, 1: 5})
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    zeta = np.arange(2, dtype=np.int32)
    x, gain = oracle.decide(0, g.off, g.col, w2, zeta, vol.copy(), vol, S)
    assert x == -1 and gain == 0
    # isolated and loop-only nodes never move
    g = graphgen.from_edges(3, [(0, 1)], loops={2: 3})
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    assert oracle.decide(2, g.off, g.col, w2, np.arange(3, dtype=np.int32), vol.copy(), vol, S)[0] == -1


# ------------------------------------------------------------------ colouring
@pytest.mark.parametrize("seed", range(6))
def test_colouring_is_greedy_in_priority_order(seed):
    g = graphgen.random_graph(80, 0.08 + 0.04 * seed, seed=seed, weighted=False, loops=0.1)
    for level in (0, 2):
        col, C = oracle.colour(g.off, g.col, seed=seed, level=level)
        order = refs.priority_order(g.n, seed, level)
        assert np.array_equal(col, refs.nx_greedy_colouring(g.off, g.col, order))
        rows = np.repeat(np.arange(g.n), np.diff(g.off))
        nl = rows != g.col
        assert not np.any(col[rows[nl]] == col[g.col[nl]])      # proper colouring
        assert C == col.max() + 1


def test_sequential_schedule_classes_are_priority_ranks():
    g = graphgen.random_graph(40, 0.2, seed=1, weighted=False)
    col, C = oracle.colour(g.off, g.col, seed=9, level=1, schedule=1)
    order = refs.priority_order(40, 9, 1)
    assert C == 40 and [int(col[u]) for u in order] == list(range(40))


def test_jones_plassmann_rounds_equal_greedy():
    """Jones-Plassmann (colour a node once all higher-priority neighbours are
    coloured, with the smallest free colour) computed round by round here gives
    the oracle's greedy colouring."""
    g = graphgen.rmat(10, 8, seed=4)
    col, _ = oracle.colour(g.off, g.col, seed=3, level=0)
    n = g.n
    pr = {u: (refs.splitmix64(3 ^ u), u) for u in range(n)}
    jp = [-1] * n
    left = set(range(n))
    while left:
        ready = [u for u in left if all(jp[v] >= 0 for v in g.col[g.off[u]:g.off[u + 1]]
                                         if v != u and pr[int(v)] > pr[u])]
        for u in ready:
            used = {jp[v] for v in g.col[g.off[u]:g.off[u + 1]] if v != u and pr[int(v)] > pr[u]}
            c = 0
            while c in used:
                c += 1
            jp[u] = c
        left -= set(ready)
    assert list(col) == jp


# ------------------------------------------------------------------ class step / sweep
@pytest.mark.parametrize("seed", range(6))
def test_class_step_invariants_and_bruteforce(seed):
    rng = np.random.default_rng(seed)
    g = graphgen.random_graph(50, 0.15, seed=50 + seed, weighted=True, loops=0.2)
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    colours, C = oracle.colour(g.off, g.col, seed=seed)
    zeta = np.arange(g.n, dtype=np.int32)
    volC = vol.copy()
    for c in range(C):
        members = np.nonzero(colours == c)[0]
        # each member's decision against the class-start state, by brute force
        want = oracle.decide_many(members, g.off, g.col, w2, zeta, volC, vol, S)
        z0 = zeta.copy()
        mv = oracle.class_step(g.off, g.col, w2, vol, S, colours, c, zeta, volC)
        assert mv == int(np.count_nonzero(want >= 0))
        exp = z0.copy()
        exp[members[want >= 0]] = want[want >= 0]
        assert np.array_equal(zeta, exp)
        assert int(volC.sum()) == S
        vc = np.zeros(g.n, np.int64); np.add.at(vc, zeta, vol)
        assert np.array_equal(vc, volC)


@pytest.mark.parametrize("seed", range(4))
def test_converged_sweep_is_locally_optimal(seed):
    g = graphgen.random_graph(60, 0.1, seed=70 + seed, weighted=True, loops=0.1)
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    colours, C = oracle.colour(g.off, g.col, seed=seed)
    zeta = np.arange(g.n, dtype=np.int32); volC = vol.copy()
    for _ in range(200):
        if oracle.sweep(g.off, g.col, w2, vol, S, colours, C, zeta, volC) == 0:
            break
    else:
        pytest.skip("did not converge in 200 sweeps")
    N0 = _N(g, w2, zeta)
    for u in range(g.n):
        for X in {int(zeta[v]) for v in g.col[g.off[u]:g.off[u + 1]] if v != u}:
            z2 = zeta.copy(); z2[u] = X
            assert _N(g, w2, z2) - N0 <= 0


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_threaded_sweep_equals_plain_sweep(threads):
    """orc_sweep_mt (class decisions spread over threads, for writing stored
    values of very large graphs) leaves the same communities, volumes and move
    counts as orc_sweep, sweep after sweep, on graphs with classes large enough
    to be split."""
    for g, seed in ((graphgen.rmat(13, 16, seed=41, weighted=True), 1),
                    (graphgen.random_graph(400, 0.05, seed=42, weighted=True, loops=0.1), 2),
                    (graphgen.planted_partition_1000(seed=3), 3)):
        w2 = oracle.double_diagonal(g.off, g.col, g.w)
        vol, S = oracle.volumes(g.off, w2)
        colours, C = oracle.colour(g.off, g.col, seed=seed)
        z1 = np.arange(g.n, dtype=np.int32); v1 = vol.copy()
        z2 = z1.copy(); v2 = vol.copy()
        for _ in range(6):
            m1 = oracle.sweep(g.off, g.col, w2, vol, S, colours, C, z1, v1)
            m2 = oracle.sweep_mt(g.off, g.col, w2, vol, S, colours, C, z2, v2, threads)
            assert m1 == m2 and np.array_equal(z1, z2) and np.array_equal(v1, v2)
            if m1 == 0:
                break


# ------------------------------------------------------------------ coarsening
@pytest.mark.parametrize("seed", range(8))
def test_contraction_invariants(seed):
    rng = np.random.default_rng(seed)
    g = graphgen.random_graph(70, 0.1, seed=90 + seed, weighted=True, loops=0.2)
    w2, vol, S, zeta, volC = _state_after_random_moves(g, rng)
    pi, k = oracle.relabel(zeta)
    assert sorted(set(pi.tolist())) == list(range(k))
    # ids ascend with the old community ids
    firsts = {int(zeta[u]): int(pi[u]) for u in range(g.n)}
    ks = sorted(firsts)
    assert [firsts[x] for x in ks] == list(range(k))
    coff, ccol, cw = oracle.contract(g.off, g.col, w2, pi, k)
    assert int(cw.sum()) == S and np.all(cw > 0)
    # rows ascending, symmetric
    ent = {}
    for c in range(k):
        row = ccol[coff[c]:coff[c + 1]]
        assert np.all(np.diff(row) > 0)
        for e in range(coff[c], coff[c + 1]):
            ent[(c, int(ccol[e]))] = int(cw[e])
    assert all(ent.get((b, a)) == wt for (a, b), wt in ent.items())
    # coarse volumes are the community volumes
    cvol, S2 = oracle.volumes(coff, cw)
    assert S2 == S
    assert np.array_equal(cvol, np.array([volC[x] for x in ks]))
    # modularity of the projected partition is preserved exactly
    assert _N(g, w2, zeta) == oracle.modularity_parts(coff, ccol, cw, np.arange(k, dtype=np.int32))[0]
    for _ in range(3):
        zc = rng.integers(0, max(1, k // 2), k).astype(np.int32)
        assert _N(g, w2, zc[pi]) == oracle.modularity_parts(coff, ccol, cw, zc)[0]


# ------------------------------------------------------------------ full run (Algorithm 3)
def _q_opt(g):
    best = None
    for p in refs.set_partitions(g.n):
        q = refs.modularity_fraction(g.n, refs.edges_of(g.off, g.col, g.w), p)
        best = q if best is None or q > best else best
    return best


@pytest.mark.parametrize("seed", range(10))
def test_run_never_beats_bruteforce_optimum(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 9))
    g = graphgen.random_graph(n, float(rng.uniform(0.2, 0.7)), seed=200 + seed, weighted=True, loops=0.2)
    r = oracle.run(g.off, g.col, g.w, seed=seed)
    assert r.q <= float(_q_opt(g)) + 1e-12


@pytest.mark.parametrize("g,opt", [
    (graphgen.disjoint_cliques(2, 4), Fraction(1, 2)),
    (graphgen.disjoint_edges(5), Fraction(4, 5)),
    (graphgen.ring_of_cliques(3, 3), Fraction(6, 8) - Fraction(1, 3)),
])
def test_run_reaches_optimum_on_small_structured(g, opt):
    assert _q_opt(g) == opt
    assert oracle.run(g.off, g.col, g.w).q == float(opt)


@pytest.mark.parametrize("c,k", [(10, 5), (6, 4), (20, 6)])
def test_ring_of_cliques_found(c, k):
    g = graphgen.ring_of_cliques(c, k)
    r = oracle.run(g.off, g.col, None)
    a = k * (k - 1)
    assert c < a + 2
    assert np.array_equal(r.labels, np.repeat(np.arange(c), k).astype(np.int32))
    assert r.q == float(Fraction(a, a + 2) - Fraction(1, c))


@pytest.mark.parametrize("seed", range(8))
def test_sequential_schedule_equals_fraction_louvain(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 70))
    g = graphgen.random_graph(n, float(rng.uniform(0.05, 0.3)), seed=300 + seed, weighted=True, loops=0.15)
    r = oracle.run(g.off, g.col, g.w, seed=seed, schedule=1)
    ref = refs.seq_louvain(n, refs.edges_of(g.off, g.col, g.w), seed=seed)
    assert np.array_equal(r.labels, ref)


def test_sequential_schedule_on_planted_partition_matches_reference():
    g = graphgen.sbm(200, 4, 0.2, 0.01, seed=11)
    r = oracle.run(g.off, g.col, None, seed=5, schedule=1)
    assert np.array_equal(r.labels, refs.seq_louvain(g.n, refs.edges_of(g.off, g.col, None), seed=5))


def test_canonical_labels_and_trace_consistency():
    g = graphgen.planted_partition_1000()
    r = oracle.run(g.off, g.col, None)
    # canonical: first occurrence order
    seen = []
    for x in r.labels:
        if x not in seen:
            assert x == len(seen)
            seen.append(x)
    assert r.n[0] == 1000 and r.communities[-1] == r.n[-1]
    assert all(r.communities[i] == r.n[i + 1] for i in range(r.levels - 1))
    assert abs(r.q - refs.nx_modularity(g.off, g.col, None, r.labels)) < 1e-12


def test_planted_partition_statistics():
    """Statistical expectation only: the 10 planted blocks are (nearly) recovered."""
    g = graphgen.planted_partition_1000()
    r = oracle.run(g.off, g.col, None)
    blocks = np.arange(1000) // 100
    assert len(set(r.labels.tolist())) == 10
    for b in range(10):
        assert np.bincount(r.labels[blocks == b]).max() >= 90
    assert 0.55 < r.q < 0.65


def test_max_levels_and_sweeps_respected():
    g = graphgen.planted_partition_1000()
    r = oracle.run(g.off, g.col, None, max_levels=1, max_sweeps=2)
    assert r.levels == 1 and r.sweeps == [2]


def test_empty_and_edgeless():
    r = oracle.run(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert r.levels == 1 and r.q == 0.0
    g = graphgen.from_edges(5, [])
    r = oracle.run(g.off, g.col, None)
    assert np.array_equal(r.labels, np.arange(5)) and r.q == 0.0


# ------------------------------------------------------------------ PLMR (Algorithm 4)
@pytest.mark.parametrize("seed", range(8))
def test_plmr_sequential_equals_fraction_reference(seed):
    """With the sequential schedule, the oracle's PLMR equals an independent
    recursive implementation of Algorithm 4 in exact fractions."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 80))
    g = graphgen.random_graph(n, float(rng.uniform(0.04, 0.25)), seed=500 + seed, weighted=True, loops=0.15)
    r = oracle.run(g.off, g.col, g.w, seed=seed, schedule=1, refine=True)
    ref = refs.seq_plmr(n, refs.edges_of(g.off, g.col, g.w), seed=seed)
    assert np.array_equal(r.labels, ref)


def test_plmr_sequential_on_planted_partition_and_level_cap():
    g = graphgen.sbm(300, 6, 0.15, 0.01, seed=12)
    e = refs.edges_of(g.off, g.col, None)
    for ml in (0, 2):
        r = oracle.run(g.off, g.col, None, seed=3, schedule=1, refine=True, max_levels=ml)
        assert np.array_equal(r.labels, refs.seq_plmr(g.n, e, seed=3, max_levels=ml))


@pytest.mark.parametrize("seed", range(4))
def test_plmr_single_level_is_plm(seed):
    """With one level there is no prolongation, so PLMR is PLM."""
    g = graphgen.random_graph(120, 0.06, seed=600 + seed, weighted=True, loops=0.1)
    a = oracle.run(g.off, g.col, g.w, seed=seed, max_levels=1)
    b = oracle.run(g.off, g.col, g.w, seed=seed, max_levels=1, refine=True)
    assert np.array_equal(a.labels, b.labels) and a.q == b.q and b.ref_sweeps == [0]


@pytest.mark.parametrize("seed", range(4))
def test_plmr_final_partition_is_locally_optimal(seed):
    """When the refinement at level 0 ends on a sweep without moves, no single
    node move to a neighbouring community raises N (on the input graph)."""
    g = graphgen.random_graph(70, 0.09, seed=700 + seed, weighted=True, loops=0.1)
    r = oracle.run(g.off, g.col, g.w, seed=seed, refine=True, max_sweeps=64)
    if r.levels < 2 or r.ref_sweeps[0] >= 64:
        pytest.skip("no refinement at level 0, or it did not converge")
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    zeta = r.labels.astype(np.int32)
    N0 = _N(g, w2, zeta)
    for u in range(g.n):
        for X in {int(zeta[v]) for v in g.col[g.off[u]:g.off[u + 1]] if v != u}:
            z2 = zeta.copy(); z2[u] = X
            assert _N(g, w2, z2) - N0 <= 0


def test_plmr_keeps_the_optimum_of_clear_structures():
    for g, q in [(graphgen.disjoint_cliques(2, 5), Fraction(1, 2)),
                 (graphgen.ring_of_cliques(6, 4), Fraction(12, 14) - Fraction(1, 6))]:
        r = oracle.run(g.off, g.col, g.w, refine=True)
        assert r.q == float(q)


# ------------------------------------------------------------------ resolution gamma
def _Ng(g, w2, zeta, gamma):
    """q S I2 - p sum vol(C)^2 for gamma = p / q (q S^2 times the gamma-modularity)."""
    p, q = gamma
    vol, S = oracle.volumes(g.off, w2)
    I2 = 0
    for u in range(g.n):
        for e in range(g.off[u], g.off[u + 1]):
            if zeta[g.col[e]] == zeta[u]:
                I2 += int(w2[e])
    vc = {}
    for u in range(g.n):
        vc[int(zeta[u])] = vc.get(int(zeta[u]), 0) + int(vol[u])
    return q * S * I2 - p * sum(x * x for x in vc.values())


@pytest.mark.parametrize("gamma", [(1, 2), (3, 2), (7, 3), (0, 1), (5, 1)])
def test_gamma_gain_is_half_the_change_of_Ngamma(gamma):
    """For every node of a random partition: the chosen move's gain is half the
    exact change of q S I2 - p sum vol(C)^2, no candidate changes it more (ties
    to the lowest id), and staying means no candidate raises it."""
    g = graphgen.random_graph(40, 0.15, seed=900 + gamma[0], weighted=True, loops=0.2)
    w2 = oracle.double_diagonal(g.off, g.col, g.w)
    vol, S = oracle.volumes(g.off, w2)
    rng = np.random.default_rng(gamma[0] * 10 + gamma[1])
    zeta = rng.integers(0, 8, g.n).astype(np.int32)
    volC = np.zeros(g.n, np.int64)
    np.add.at(volC, zeta, vol)
    N0 = _Ng(g, w2, zeta, gamma)
    for u in range(g.n):
        x, gain = oracle.decide(u, g.off, g.col, w2, zeta, volC, vol, S, gamma=gamma)
        best, bestX = 0, -1
        for X in sorted({int(zeta[v]) for v in g.col[g.off[u]:g.off[u + 1]] if v != u} - {int(zeta[u])}):
            z2 = zeta.copy(); z2[u] = X
            d = _Ng(g, w2, z2, gamma) - N0
            if d > best:
                best, bestX = d, X
        assert x == bestX and (x < 0 or 2 * gain == best)


@pytest.mark.parametrize("seed", range(6))
def test_gamma_sequential_equals_fraction_louvain(seed):
    gammas = [(1, 2), (3, 2), (7, 3), (2, 5), (4, 1), (1, 1)]
    gm = gammas[seed]
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(8, 70))
    g = graphgen.random_graph(n, float(rng.uniform(0.05, 0.25)), seed=1100 + seed, weighted=True, loops=0.15)
    r = oracle.run(g.off, g.col, g.w, seed=seed, schedule=1, gamma=gm)
    ref = refs.seq_louvain(n, refs.edges_of(g.off, g.col, g.w), seed=seed, gamma=Fraction(*gm))
    assert np.array_equal(r.labels, ref)


def test_gamma_threshold_on_two_cliques():
    """Two K5 (S = 40, vol = 4): a first move gains 40 q - 16 p, so every gamma
    below 5/2 finds the cliques and gamma >= 5/2 keeps singletons."""
    g = graphgen.disjoint_cliques(2, 5)
    assert oracle.run(g.off, g.col, g.w, gamma=(249, 100)).q == 0.5
    r = oracle.run(g.off, g.col, g.w, gamma=(5, 2))
    assert r.q == -0.1 and len(set(r.labels.tolist())) == 10


def test_gamma_one_in_any_form_is_plm():
    g = graphgen.rmat(11, 16, seed=4, weighted=True)
    a = oracle.run(g.off, g.col, g.w)
    for gm in [(1, 1), (2, 2), (0, 0), (37, 37)]:
        b = oracle.run(g.off, g.col, g.w, gamma=gm)
        assert np.array_equal(a.labels, b.labels) and a.q == b.q


def test_gamma_bounds():
    g = graphgen.disjoint_cliques(2, 3)
    for gm in [(-1, 1), (1, 0), (1 << 16, 1), (1, 1 << 16)]:
        with pytest.raises(ValueError):
            oracle.run(g.off, g.col, g.w, gamma=gm)


# ------------------------------------------------------------------ PLP (Algorithm 1)
def _canon(lab):
    m, out = {}, []
    for x in lab:
        m.setdefault(int(x), len(m))
        out.append(m[int(x)])
    return np.array(out, np.int32)


def _seq_plp(g, seed=0, max_iters=64, active_sets=True):
    colours = refs.nx_greedy_colouring(g.off, g.col, refs.priority_order(g.n, seed, 0))
    return refs.seq_plp(g.off, g.col, g.w, colours, seed=seed, max_iters=max_iters, active_sets=active_sets)


@pytest.mark.parametrize("seed", range(8))
def test_plp_equals_python_label_propagation(seed):
    """Same colour classes (networkx greedy colouring in priority order), same
    tie key: labels, iterations and updates per iteration agree."""
    rng = np.random.default_rng(1200 + seed)
    n = int(rng.integers(20, 160))
    g = graphgen.random_graph(n, float(rng.uniform(0.03, 0.2)), seed=1300 + seed, weighted=seed % 2 == 1,
                              loops=0.2 if seed % 3 == 0 else 0.0)
    r = oracle.plp(g.off, g.col, g.w, seed=seed)
    lab, upd = _seq_plp(g, seed)
    assert np.array_equal(r.labels, _canon(lab))
    assert r.updates == upd and r.iterations == len(upd)
    assert r.q == pytest.approx(refs.nx_modularity(g.off, g.col, g.w, r.labels), abs=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_plp_active_sets_change_nothing(seed):
    """A node turns inactive only after keeping its label; its neighbourhood's
    labels are unchanged until a neighbour moves, so evaluating it anyway would
    keep the label again: the active set is an optimisation only."""
    g = graphgen.sbm(400, 8, 0.12, 0.01, seed=1400 + seed)
    r = oracle.plp(g.off, g.col, g.w, seed=seed)
    lab, upd = _seq_plp(g, seed, active_sets=False)
    assert np.array_equal(r.labels, _canon(lab)) and r.updates == upd


@pytest.mark.parametrize("seed", range(5))
def test_plp_fixed_point_is_dominant(seed):
    """When the last iteration updated nothing, every node carries a dominant
    label of its neighbourhood (by brute force over its neighbours)."""
    g = graphgen.rmat(9, 8, seed=1500 + seed, weighted=seed % 2 == 0)
    r = oracle.plp(g.off, g.col, g.w, seed=seed)
    assert r.updates[-1] == 0
    wts = np.ones(g.nnz, np.int64) if g.w is None else g.w
    for v in range(g.n):
        acc = {}
        for e in range(g.off[v], g.off[v + 1]):
            u = int(g.col[e])
            if u != v:
                acc[int(r.labels[u])] = acc.get(int(r.labels[u]), 0) + int(wts[e])
        if acc:
            assert acc.get(int(r.labels[v]), 0) == max(acc.values())


@pytest.mark.parametrize("c,k", [(2, 3), (3, 5), (6, 4), (10, 8)])
def test_plp_disjoint_cliques_one_label_each(c, k):
    """In K_k the first node to move takes a neighbour's label, which then
    carries weight 2 against 1 for every other label: one label per clique,
    Q = 1 - 1/c."""
    g = graphgen.disjoint_cliques(c, k)
    r = oracle.plp(g.off, g.col, g.w)
    assert np.array_equal(r.labels, np.repeat(np.arange(c), k).astype(np.int32))
    assert r.q == pytest.approx(1 - 1 / c, abs=1e-15)


def test_plp_isolated_loops_and_empty():
    """Nodes without non-loop neighbours keep their own label and are never
    visited; the empty graph takes no iteration work."""
    g = graphgen.from_edges(5, [(1, 2)], loops={0: 3})
    r = oracle.plp(g.off, g.col, g.w)
    assert r.labels[0] != r.labels[1] and r.labels[1] == r.labels[2]
    assert len(set(r.labels.tolist())) == 4
    e = graphgen.from_edges(0, [])
    assert oracle.plp(e.off, e.col, e.w).labels.shape == (0,)


def test_plp_iteration_cap_and_threshold():
    g = graphgen.rmat(12, 16, seed=7, weighted=False)
    r1 = oracle.plp(g.off, g.col, g.w, max_iters=1)
    assert r1.iterations == 1 and r1.updates[0] > 0
    r = oracle.plp(g.off, g.col, g.w)
    # theta = n 10^-5 < 1 here: the loop ends on an iteration without updates or at the cap
    assert r.updates[-1] == 0 or r.iterations == 64
    assert all(u > 0 for u in r.updates[:-1])
    for bad in (0, 65):
        with pytest.raises(ValueError):
            oracle.plp(g.off, g.col, g.w, max_iters=bad)


def test_plp_ring_of_cliques():
    g = graphgen.ring_of_cliques(12, 6)
    r = oracle.plp(g.off, g.col, g.w)
    assert np.array_equal(r.labels, np.repeat(np.arange(12), 6).astype(np.int32))


# ------------------------------------------------------------------ EPP (Algorithm 5)
def _coarse_edges(g, pi):
    out = {}
    for (u, v), wt in refs.edges_of(g.off, g.col, g.w).items():
        a, b = sorted((int(pi[u]), int(pi[v])))
        out[(a, b)] = out.get((a, b), 0) + wt
    return out


@pytest.mark.parametrize("b", [1, 2, 4])
def test_epp_core_groups_are_equation_3_2(b):
    """Two nodes share a core group iff every base PLP solution (seeds
    seed .. seed+b-1) gives them the same label; coarse ids ascend with the
    smallest member."""
    g = graphgen.planted_partition_1000(seed=3)
    r = oracle.epp(g.off, g.col, g.w, b=b, seed=11)
    base = [oracle.plp(g.off, g.col, g.w, seed=11 + i).labels for i in range(b)]
    tuples = {}
    for v in range(g.n):
        tuples.setdefault(tuple(int(x[v]) for x in base), len(tuples))
    expect = np.array([tuples[tuple(int(x[v]) for x in base)] for v in range(g.n)], np.int32)
    assert np.array_equal(r.core_groups, expect)   # first-occurrence order = ascending smallest member
    assert r.cores == len(tuples) == r.run.n[0]
    if b == 1:
        assert np.array_equal(r.core_groups, base[0])


@pytest.mark.parametrize("seed", range(4))
def test_epp_equals_fraction_plmr_on_core_graph(seed):
    """Sequential schedule: EPP's result is the exact-fraction PLMR on the
    core-group graph (as level 1), prolonged to the input nodes."""
    rng = np.random.default_rng(1600 + seed)
    n = int(rng.integers(30, 120))
    g = graphgen.random_graph(n, float(rng.uniform(0.04, 0.15)), seed=1700 + seed, weighted=seed % 2 == 0,
                              loops=0.1)
    r = oracle.epp(g.off, g.col, g.w, b=3, seed=seed, schedule=1)
    zc = refs.seq_plmr(r.cores, _coarse_edges(g, r.core_groups), seed=seed, first_level=1)
    assert np.array_equal(r.labels, _canon(zc[r.core_groups]))
    assert r.q == pytest.approx(refs.nx_modularity(g.off, g.col, g.w, r.labels), abs=1e-12)


def test_epp_clear_structures_and_bounds():
    for g, q in [(graphgen.disjoint_cliques(4, 6), 0.75), (graphgen.ring_of_cliques(8, 5), None)]:
        r = oracle.epp(g.off, g.col, g.w, b=4)
        if q is not None:
            assert r.q == q
        else:
            ref = oracle.run(g.off, g.col, g.w, refine=True)
            assert r.q >= ref.q - 1e-12
    g = graphgen.disjoint_cliques(2, 3)
    for kw in [dict(b=0), dict(plp_iters=0), dict(plp_iters=65), dict(max_sweeps=0)]:
        with pytest.raises(ValueError):
            oracle.epp(g.off, g.col, g.w, **kw)
    e = graphgen.from_edges(0, [])
    assert oracle.epp(e.off, e.col, e.w).labels.shape == (0,)


def test_epp_planted_partition_quality():
    """On the planted partition the ensemble's cores feed PLMR a small graph:
    no worse than PLP alone."""
    g = graphgen.planted_partition_1000(seed=1)
    p = oracle.plp(g.off, g.col, g.w)
    r = oracle.epp(g.off, g.col, g.w, b=4)
    assert r.q >= p.q and r.cores < g.n
