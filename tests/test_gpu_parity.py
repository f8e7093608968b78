"""Parity of the HIP path (through the C ABI) with the oracle, element by
element: colouring, every class step, every sweep, every coarse CSR, full-run
labels, modularity.  Integer results must match bit for bit; modularity is
compared for exact equality (both sides divide the same two correctly rounded
128-bit integers), which is inside the 1e-12 tolerance the method allows.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P  # fails loudly without the built library
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def stepwise(P, g, seed=0, schedule=0, per_class=True, max_sweeps=32, max_levels=8, **opts):
    """Walks the GPU context and the oracle level by level in lock step."""
    ctx = P.Context(g.off, g.col, g.w, colour_seed=seed, schedule=schedule, **opts)
    off, col = g.off.astype(np.int64), g.col.astype(np.int32)
    w2 = oracle.double_diagonal(off, col, g.w)
    level = 0
    try:
        while True:
            goff, gcol, gw = ctx.graph()
            assert np.array_equal(goff, off) and np.array_equal(gcol, col) and np.array_equal(gw, w2), level
            vol, S = oracle.volumes(off, w2)
            colours, C = oracle.colour(off, col, seed, level, schedule)
            z, v, c = ctx.state()
            assert np.array_equal(c, colours), f"colouring differs at level {level}"
            assert np.array_equal(z, np.arange(len(z))) and np.array_equal(v, vol)
            li = ctx.level_info()
            assert li.colours == C and li.S == S and li.level == level
            zeta = np.arange(len(vol), dtype=np.int32)
            volC = vol.copy()
            for s in range(max_sweeps):
                if per_class:
                    mv = 0
                    for cls in range(C):
                        mo = oracle.class_step(off, col, w2, vol, S, colours, cls, zeta, volC)
                        mg = ctx.move_class(cls)
                        assert mg == mo, (level, s, cls)
                        mv += mo
                else:
                    mv = oracle.sweep(off, col, w2, vol, S, colours, C, zeta, volC)
                    assert ctx.move_sweep() == mv, (level, s)
                z, v, _ = ctx.state()
                assert np.array_equal(z, zeta) and np.array_equal(v, volC), (level, s)
                if mv == 0:
                    break
            pi, k = oracle.relabel(zeta)
            if k == len(vol) or level + 1 >= max_levels:
                return level + 1
            coff, ccol, cw = oracle.contract(off, col, w2, pi, k)
            assert ctx.coarsen() == k
            off, col, w2 = coff, ccol, cw
            level += 1
    finally:
        ctx.close()


def full_run(P, g, seed=0, schedule=0, max_sweeps=32, max_levels=0, refine=False, gamma=(1, 1), **opts):
    r = oracle.run(g.off, g.col, g.w, max_sweeps=max_sweeps, max_levels=max_levels, seed=seed, schedule=schedule,
                   refine=refine, gamma=gamma)
    with P.Context(g.off, g.col, g.w, colour_seed=seed, schedule=schedule, max_sweeps=max_sweeps,
                   max_levels=max_levels, refine=int(refine), gamma_num=gamma[0], gamma_den=gamma[1],
                   **opts) as ctx:
        labels, q, lv = ctx.run()
        st = ctx.stats()
    assert lv == r.levels
    assert np.array_equal(labels, r.labels)
    assert q == r.q
    assert st["n"] == r.n and st["nnz"] == r.nnz and st["colours"] == r.colours
    assert st["sweeps"] == r.sweeps and st["communities"] == r.communities
    assert st["moves"] == [sum(m) for m in r.moves]
    if refine:
        assert st["ref_sweeps"] == r.ref_sweeps and st["ref_moves"] == r.ref_moves
    return r


SMALL_BINS = dict(bin_lane=1, bin_wave=2, bin_block=3)   # every path on small graphs
MID_BINS = dict(bin_lane=4, bin_wave=16, bin_block=64)


# ------------------------------------------------------------------ class / sweep / level parity
@pytest.mark.parametrize("seed", range(3))
def test_stepwise_random_weighted_with_loops(P, seed):
    _say("stepwise random", seed)
    g = graphgen.random_graph(120, 0.06, seed=10 + seed, weighted=True, loops=0.2)
    stepwise(P, g, seed=seed)


@pytest.mark.parametrize("bins", [SMALL_BINS, MID_BINS], ids=["small", "mid"])
def test_stepwise_all_bins(P, bins):
    _say("stepwise bins", bins)
    g = graphgen.random_graph(150, 0.12, seed=5, weighted=True, loops=0.1)
    stepwise(P, g, seed=3, **bins)


def test_stepwise_planted_partition(P):
    _say("stepwise planted partition 1000")
    stepwise(P, graphgen.planted_partition_1000(), per_class=False)


def test_stepwise_rmat_small_hubs(P):
    _say("stepwise rmat 12")
    g = graphgen.rmat(12, 16, seed=7, weighted=True)
    stepwise(P, g, seed=1, per_class=False, bin_lane=8, bin_wave=32, bin_block=128)


def test_stepwise_sequential_schedule(P):
    _say("stepwise sequential")
    g = graphgen.random_graph(60, 0.1, seed=2, weighted=True, loops=0.2)
    stepwise(P, g, seed=4, schedule=1)


# ------------------------------------------------------------------ full runs
def test_full_run_planted_partition(P):
    _say("full planted partition 1000")
    r = full_run(P, graphgen.planted_partition_1000())
    assert len(set(r.labels.tolist())) == 10


@pytest.mark.parametrize("bins", [{}, SMALL_BINS, MID_BINS], ids=["default", "small", "mid"])
@pytest.mark.parametrize("scale", [10, 14])
def test_full_run_rmat(P, scale, bins):
    _say("full rmat", scale, bins)
    g = graphgen.rmat(scale, 16, seed=scale, weighted=(scale == 14))
    full_run(P, g, seed=scale, **bins)


@pytest.mark.parametrize("seed", range(4))
def test_full_run_random(P, seed):
    _say("full random", seed)
    g = graphgen.random_graph(300, 0.02, seed=40 + seed, weighted=bool(seed % 2), loops=0.1 * seed)
    full_run(P, g, seed=seed, max_sweeps=1 + 10 * seed)


def test_full_run_forced_int128_same(P):
    _say("full int128")
    g = graphgen.rmat(12, 16, seed=3, weighted=True)
    full_run(P, g, int_mode=P.PLM_INT_128)
    full_run(P, g, int_mode=P.PLM_INT_128, **SMALL_BINS)


# ------------------------------------------------------------------ PLMR (Algorithm 4)
def test_plmr_planted_partition(P):
    _say("plmr planted partition")
    full_run(P, graphgen.planted_partition_1000(seed=2), refine=True)


@pytest.mark.parametrize("bins", [{}, SMALL_BINS, MID_BINS], ids=["default", "small", "mid"])
def test_plmr_rmat(P, bins):
    _say("plmr rmat", bins)
    full_run(P, graphgen.rmat(13, 16, seed=31, weighted=True), seed=5, refine=True, **bins)


@pytest.mark.parametrize("seed", range(3))
def test_plmr_random_caps_and_schedules(P, seed):
    _say("plmr random", seed)
    g = graphgen.random_graph(250, 0.03, seed=80 + seed, weighted=True, loops=0.1)
    full_run(P, g, seed=seed, refine=True, max_sweeps=3 + 10 * seed, max_levels=[0, 2, 3][seed])
    full_run(P, g, seed=seed, refine=True, schedule=1)


def test_plmr_forced_int128(P):
    _say("plmr int128")
    full_run(P, graphgen.rmat(12, 16, seed=9, weighted=True), refine=True, int_mode=P.PLM_INT_128)


def test_plmr_rejected_for_batches(P):
    g = graphgen.disjoint_cliques(2, 3)
    with pytest.raises(P.PLMError) as e:
        P.BatchContext(np.array([0, 3, 6]), g.off, g.col, g.w, refine=1)
    assert e.value.status == P.PLM_E_ARG


# ------------------------------------------------------------------ resolution gamma
GAMMAS = [(1, 2), (3, 2), (7, 3), (0, 1), (5, 1)]


@pytest.mark.parametrize("gamma", GAMMAS, ids=[f"{a}_{b}" for a, b in GAMMAS])
@pytest.mark.parametrize("bins", [{}, SMALL_BINS, MID_BINS], ids=["default", "small", "mid"])
def test_gamma_random_all_bins(P, gamma, bins):
    _say("gamma random", gamma, bins)
    g = graphgen.random_graph(200, 0.05, seed=90 + gamma[0], weighted=True, loops=0.1)
    full_run(P, g, seed=gamma[1], gamma=gamma, **bins)


@pytest.mark.parametrize("gamma", [(1, 2), (7, 3)], ids=["1_2", "7_3"])
def test_gamma_rmat_plmr_int128(P, gamma):
    _say("gamma rmat plmr int128", gamma)
    g = graphgen.rmat(12, 16, seed=14, weighted=True)
    full_run(P, g, gamma=gamma)
    full_run(P, g, gamma=gamma, refine=True)
    full_run(P, g, gamma=gamma, int_mode=P.PLM_INT_128, **SMALL_BINS)


def test_gamma_batch_matches_oracle(P):
    _say("gamma batch")
    graphs = [graphgen.planted_partition_1000(seed=4), graphgen.ring_of_cliques(6, 4),
              graphgen.random_graph(150, 0.05, seed=3, weighted=True, loops=0.2), graphgen.rmat(11, 16, seed=2)]
    nb, off, col, w = P.pack_batch(graphs)
    with P.BatchContext(nb, off, col, w, gamma_num=3, gamma_den=2) as ctx:
        labels, q, lv = ctx.run_batch()
    for i, g in enumerate(graphs):
        r = oracle.run(g.off, g.col, g.w, gamma=(3, 2))
        a, b = int(nb[i]), int(nb[i + 1])
        assert np.array_equal(labels[a:b], r.labels) and q[i] == r.q and lv[i] == r.levels


def test_gamma_argument_errors(P):
    g = graphgen.disjoint_cliques(2, 3)
    for gm in [(-1, 1), (1, 0), (1 << 16, 1)]:
        with pytest.raises(P.PLMError) as e:
            P.Context(g.off, g.col, g.w, gamma_num=gm[0], gamma_den=gm[1])
        assert e.value.status == P.PLM_E_ARG
    with P.Context(g.off, g.col, g.w, gamma_num=0, gamma_den=0) as ctx:   # 0/0 means 1
        assert ctx.run()[1] == oracle.run(g.off, g.col, g.w).q


def test_int64_mode_rejects_overflow(P):
    # S * vol(u) >= 2^62: one heavy edge
    big = 2**31 - 1
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], [big, big], loops={0: big})
    with pytest.raises(P.PLMError) as ei:
        P.Context(g.off, g.col, g.w, int_mode=P.PLM_INT_64)
    assert ei.value.status == P.PLM_E_STATE
    full_run(P, g)   # auto mode takes the 128-bit path


def test_hub_multi_workgroup(P):
    """A star with 20000 weighted leaves plus a ring among the leaves: one hub
    whose table spans many eval workgroups."""
    _say("hub star")
    n = 20001
    edges = [(0, i) for i in range(1, n)] + [(i, i + 1) for i in range(1, n - 1)]
    rng = np.random.default_rng(1)
    g = graphgen.from_edges(n, edges, rng.integers(1, 50, len(edges)))
    full_run(P, g)
    full_run(P, g, bin_wave=32, bin_block=64)


def test_sequential_schedule_full(P):
    _say("full sequential")
    g = graphgen.random_graph(200, 0.03, seed=9, weighted=True, loops=0.1)
    full_run(P, g, seed=2, schedule=1)


def test_ring_of_cliques_and_two_cliques(P):
    g = graphgen.ring_of_cliques(10, 5)
    with P.Context(g.off, g.col) as ctx:
        labels, q, _ = ctx.run()
    assert q == 89 / 110 and np.array_equal(labels, np.repeat(np.arange(10), 5))
    g = graphgen.disjoint_cliques(2, 8)
    with P.Context(g.off, g.col) as ctx:
        assert ctx.run()[1] == 0.5


# ------------------------------------------------------------------ modularity
@pytest.mark.parametrize("seed", range(3))
def test_modularity_api(P, seed):
    rng = np.random.default_rng(seed)
    g = graphgen.random_graph(200, 0.05, seed=seed, weighted=True, loops=0.2)
    with P.Context(g.off, g.col, g.w) as ctx:
        for _ in range(4):
            lab = rng.integers(0, 30, 200).astype(np.int32)
            assert ctx.modularity(lab) == oracle.modularity(g.off, g.col, g.w, lab)
        with pytest.raises(P.PLMError):
            ctx.modularity(np.full(200, 500, np.int32))


# ------------------------------------------------------------------ device inputs, streams, repeatability
def test_device_inputs_and_stream(P):
    import torch
    _say("device inputs")
    g = graphgen.rmat(13, 16, seed=11, weighted=True)
    r = oracle.run(g.off, g.col, g.w)
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    off = torch.from_numpy(g.off).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    torch.cuda.synchronize()
    with P.Context(off, col, w, stream=s) as ctx:
        lab = torch.empty(g.n, dtype=torch.int32, device=dev)
        _, q, lv = ctx.run(lab)
        assert q == r.q and lv == r.levels
        assert np.array_equal(lab.cpu().numpy(), r.labels)
        assert ctx.modularity(lab) == r.q
        # repeat: identical
        lab2 = torch.empty_like(lab)
        ctx.run(lab2)
        assert torch.equal(lab, lab2)


def test_repeat_runs_identical(P):
    g = graphgen.rmat(14, 16, seed=1)
    with P.Context(g.off, g.col) as ctx:
        a = ctx.run()[0].copy()
        for _ in range(3):
            assert np.array_equal(ctx.run()[0], a)


# ------------------------------------------------------------------ edge cases and validation
def test_empty_and_degenerate(P):
    with P.Context(np.zeros(1, np.int64), np.zeros(0, np.int32)) as ctx:
        labels, q, lv = ctx.run()
        assert labels.shape == (0,) and q == 0.0 and lv == 1
    g = graphgen.from_edges(5, [])
    with P.Context(g.off, g.col) as ctx:
        labels, q, _ = ctx.run()
        assert np.array_equal(labels, np.arange(5)) and q == 0.0
    g = graphgen.from_edges(3, [(0, 1)], [4], loops={2: 7})
    full_run(P, g)
    g = graphgen.from_edges(1, [], loops={0: 3})
    full_run(P, g)


@pytest.mark.parametrize("case", ["asym", "range", "unsorted", "zero_w", "dup"])
def test_validation_rejects(P, case):
    g = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)], [1, 2, 3])
    off, col, w = g.off.copy(), g.col.copy(), g.w.copy()
    if case == "asym":
        w[0] = 9
    elif case == "range":
        col[0] = 7
    elif case == "unsorted":
        col[[1, 2]] = col[[2, 1]]
        w[[1, 2]] = w[[2, 1]]
    elif case == "zero_w":
        w[:] = 0
    elif case == "dup":
        col[2] = col[1]
    with pytest.raises(P.PLMError) as ei:
        P.Context(off, col, w)
    assert ei.value.status == P.PLM_E_GRAPH


def test_coarsen_api_and_state_errors(P):
    g = graphgen.planted_partition_1000()
    with P.Context(g.off, g.col) as ctx:
        while ctx.move_sweep():
            pass
        z, _, _ = ctx.state()
        k = ctx.coarsen()
        assert k == len(set(z.tolist()))
        li = ctx.level_info()
        assert li.level == 1 and li.n == k and li.weight_kind == 2
        with pytest.raises(P.PLMError):
            ctx.move_class(10**6)
        ctx.reset()
        assert ctx.level_info().level == 0


# ------------------------------------------------------------------ period-2 sweep cycles
@pytest.mark.parametrize("max_sweeps", [31, 32, 33])
def test_sweep_cycles_fast_forward(P, max_sweeps):
    """Graphs whose sweeps settle into a period-2 cycle (a few nodes moving back
    and forth until the sweep cap).  The library stops sweeping once the state
    repeats and takes the state the last sweep would leave; labels, Q, sweeps
    and move counts must still equal the oracle's, for both parities of the
    remaining sweep count, with and without refinement."""
    _say(f"cycles max_sweeps={max_sweeps}")
    skipped = 0
    for g in (graphgen.rmat(11, 16, seed=5, weighted=False), graphgen.rmat(10, 16, seed=8, weighted=False)):
        for refine in (False, True):
            r = full_run(P, g, max_sweeps=max_sweeps, refine=refine)
            with P.Context(g.off, g.col, g.w, max_sweeps=max_sweeps, refine=int(refine)) as ctx:
                ctx.run()
                st = ctx.stats()
            skipped += sum(st["cycle_sweeps"]) + sum(st["ref_cycle_sweeps"])
            assert all(c < s for c, s in zip(st["cycle_sweeps"], st["sweeps"]))
            assert r.sweeps[0] == max_sweeps
    rng = np.random.default_rng(9)
    n = int(rng.integers(50, 800))
    g = graphgen.random_graph(n, float(rng.uniform(0.005, 0.05)), seed=9, weighted=True, loops=0.1)
    full_run(P, g, max_sweeps=max_sweeps, refine=True)
    assert skipped > 0


# ------------------------------------------------------------------ sweeps replayed from a HIP graph
def test_graph_sweeps_equal_eager(P):
    """graph_sweeps: every sweep of a move phase (and every label-propagation
    iteration) is replayed from a HIP graph captured once per plan;
    hub_stream: the partitioned-hub kernels (1) or a class's kernel groups in
    three branches (2) run as forked branches inside the captured graph.
    Replays are interleaved with eager work (counter clears, read-backs,
    re-planning); every combination must equal the plain one and the oracle."""
    _say("graph sweeps / hub stream vs eager")
    cases = [(graphgen.rmat(12, 16, seed=31, weighted=True), {}),
             (graphgen.rmat(11, 16, seed=5, weighted=False), SMALL_BINS),
             (graphgen.rmat(11, 16, seed=4, weighted=False), MID_BINS)]
    for g, bins in cases:
        res = []
        for gs, hs in ((0, 0), (1, 0), (0, 1), (1, 1), (1, 2)):
            with P.Context(g.off, g.col, g.w, graph_sweeps=gs, hub_stream=hs, refine=1, **bins) as ctx:
                labels, q, lv = ctx.run()
                st = ctx.stats()
                lp = ctx.plp()
                labels2, q2, lv2 = ctx.run()   # a second run re-captures every level
            res.append((labels, q, lv, st["sweeps"], st["moves"], st["ref_moves"], lp[0], lp[2], lp[3]))
            assert np.array_equal(labels, labels2) and q == q2 and lv == lv2
        a = res[0]
        for b in res[1:]:
            assert np.array_equal(a[0], b[0]) and a[1:6] == b[1:6]
            assert np.array_equal(a[6], b[6]) and a[7:] == b[7:]
        r = oracle.run(g.off, g.col, g.w, refine=True)
        assert np.array_equal(b[0], r.labels) and b[1] == r.q
        p = oracle.plp(g.off, g.col, g.w)
        assert np.array_equal(b[6], p.labels) and b[8] == p.updates


def test_graph_sweeps_batch_equal_eager(P):
    _say("graph sweeps batch")
    gs = [graphgen.rmat(11, 16, seed=s, weighted=s % 2 == 0) for s in range(3, 9)] + \
         [graphgen.planted_partition_1000(seed=4)]
    node_base, off, col, w = P.pack_batch(gs)
    out = []
    for gs, hs in ((0, 0), (1, 0), (0, 1), (1, 1), (1, 2)):
        with P.BatchContext(node_base, off, col, w, graph_sweeps=gs, hub_stream=hs, **SMALL_BINS) as bc:
            out.append(bc.run_batch())
    la, qa, lva = out[0]
    for lb, qb, lvb in out[1:]:
        assert np.array_equal(la, lb) and list(qa) == list(qb) and list(lva) == list(lvb)


# ------------------------------------------------------------------ colouring rounds inside one workgroup
def _tail_handoff_graph(seed, m=20000, chain=20):
    """A chain of `chain` nodes in descending priority ending at a star centre
    of m lower-priority leaves: the frontiers hold one node for chain + 1
    rounds (the one-workgroup tail takes over after the first grid rounds),
    then all m leaves at once (more than the tail keeps, so the grid takes the
    rounds back).  The centre's row is long enough for the multi-workgroup
    chunk path inside the tail."""
    n = chain + 1 + m
    order = sorted(range(n), key=lambda u: (oracle.priority(seed, 0, u), u), reverse=True)
    path, centre, leaves = order[:chain], order[chain], order[chain + 1:]
    edges = [tuple(sorted((path[i], path[i + 1]))) for i in range(chain - 1)]
    edges += [tuple(sorted((path[-1], centre)))] + [tuple(sorted((centre, x))) for x in leaves]
    return graphgen.from_edges(n, sorted(edges))


@pytest.mark.parametrize("tail", [0, 1])
def test_colour_tail_matches_oracle(P, tail):
    """colour_tail = 1 runs small frontiers as back-to-back rounds in one
    workgroup, 0 launches every round on the grid: both give the oracle's
    colouring (and hence its results), including a hand-over from the tail
    back to the grid and long rows coloured inside the tail."""
    _say(f"colour tail={tail}")
    cases = [(_tail_handoff_graph(3), 3), (graphgen.rmat(13, 16, seed=21, weighted=True), 1),
             (graphgen.rmat(14, 8, seed=22, weighted=False), 2), (graphgen.planted_partition_1000(seed=5), 0)]
    for g, seed in cases:
        colours, C = oracle.colour(g.off.astype(np.int64), g.col.astype(np.int32), seed, 0, 0)
        with P.Context(g.off, g.col, g.w, colour_seed=seed, colour_tail=tail) as ctx:
            assert np.array_equal(ctx.state()[2], colours) and ctx.level_info().colours == C
        full_run(P, g, seed=seed, colour_tail=tail)
    stepwise(P, graphgen.rmat(12, 16, seed=23, weighted=True), seed=4, per_class=False, colour_tail=tail)


# ------------------------------------------------------------------ runs of empty rows
def _islands(seed, gap=200000, block=1000, weighted=True):
    """Two random blocks of `block` nodes separated by `gap` isolated nodes:
    the entry tiles that cross the gap span far more rows than they can stage
    (the per-entry fallback of the tiled kernels), the others stage theirs."""
    rng = np.random.default_rng(seed)
    n = 2 * block + gap
    edges = set()
    for base in (0, block + gap):
        for _ in range(12 * block):
            a, b = (int(x) for x in rng.integers(0, block, 2))
            if a != b:
                edges.add((base + min(a, b), base + max(a, b)))
    edges = sorted(edges)
    w = rng.integers(1, 50, len(edges)) if weighted else None
    loops = {int(x): int(rng.integers(1, 9)) for x in rng.integers(0, block, 20)} if weighted else None
    return graphgen.from_edges(n, edges, w, loops=loops)


@pytest.mark.parametrize("seed", [0, 1])
def test_runs_of_isolated_nodes(P, seed):
    _say(f"islands seed={seed}")
    g = _islands(seed, weighted=seed == 0)
    full_run(P, g, seed=seed)
    full_run(P, g, seed=seed, refine=True)
    r = oracle.plp(g.off, g.col, g.w, seed=seed)
    with P.Context(g.off, g.col, g.w, colour_seed=seed) as ctx:
        labels, q, it, upd = ctx.plp()
        assert np.array_equal(labels, r.labels) and q == r.q and upd == r.updates
        assert ctx.modularity(r.labels) == r.q
    stepwise(P, g, seed=seed, per_class=False)
