"""Independent test-side references used to pin the oracle.

Nothing here imports the oracle or the GPU library.  Everything is written from
the paper's formulas in their own (rational) form, or delegated to networkx:

* ``nx_graph`` / ``nx_modularity``: networkx's modularity (an independent
  implementation of Equation (3.1)).
* ``nx_greedy_colouring``: networkx's greedy colouring in a given node order.
* ``seq_louvain``: sequential Louvain local moving + coarsening (Blondel et al.,
  as recalled in section III-B and Algorithm 3) using the paper's Delta-mod in
  exact fractions, visiting nodes in a given priority order.
* ``set_partitions``: brute-force enumeration for tiny graphs.
* ``splitmix64``: the published SplitMix64 step.
* ``seq_plp``: label propagation (Algorithm 1) over given colour classes, in
  plain Python dictionaries.
"""
from __future__ import annotations

from fractions import Fraction

import networkx as nx
import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def priority_order(n: int, seed: int, level: int):
    """Nodes by descending (H(seed ^ (level << 40) ^ u), u)."""
    keys = [(splitmix64(seed ^ (level << 40) ^ u), u) for u in range(n)]
    return [u for _, u in sorted(keys, reverse=True)]


def edges_of(off, col, w):
    """{(u, v): w} with u <= v from a symmetric CSR (self-loops once)."""
    out = {}
    n = len(off) - 1
    for u in range(n):
        for e in range(off[u], off[u + 1]):
            v = int(col[e])
            if u <= v:
                out[(u, v)] = 1 if w is None else int(w[e])
    return out


def nx_graph(off, col, w):
    G = nx.Graph()
    G.add_nodes_from(range(len(off) - 1))
    for (u, v), wt in edges_of(off, col, w).items():
        G.add_edge(u, v, weight=wt)
    return G


def nx_modularity(off, col, w, labels) -> float:
    G = nx_graph(off, col, w)
    comms = {}
    for v, l in enumerate(labels):
        comms.setdefault(int(l), set()).add(v)
    return float(nx.community.modularity(G, list(comms.values()), weight="weight"))


def nx_greedy_colouring(off, col, order):
    G = nx_graph(off, col, None)
    order = list(order)
    col_map = nx.coloring.greedy_color(G, strategy=lambda g, c: iter(order))
    return np.array([col_map[v] for v in range(len(off) - 1)], dtype=np.int64)


def modularity_fraction(n, edges, labels) -> Fraction:
    """Equation (3.1) in exact fractions from an edge dict {(u<=v): w}."""
    W = sum(edges.values())
    if W == 0:
        return Fraction(0)
    wC, volC = {}, {}
    for (u, v), wt in edges.items():
        if u == v:
            volC[labels[u]] = volC.get(labels[u], 0) + 2 * wt
            wC[labels[u]] = wC.get(labels[u], 0) + wt
        else:
            volC[labels[u]] = volC.get(labels[u], 0) + wt
            volC[labels[v]] = volC.get(labels[v], 0) + wt
            if labels[u] == labels[v]:
                wC[labels[u]] = wC.get(labels[u], 0) + wt
    q = Fraction(0)
    for c in set(labels[:n]):
        q += Fraction(wC.get(c, 0), W) - Fraction(volC.get(c, 0) ** 2, 4 * W * W)
    return q


def set_partitions(n):
    """All set partitions of range(n) as restricted growth strings."""
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for c in range(m + 1):
            a[i] = c
            yield from rec(i + 1, max(m, c + 1) if c == m else m)

    if n == 0:
        yield []
        return
    a[0] = 0
    yield from rec(1, 1)


def seq_louvain(n, edges, seed=0, max_sweeps=32, max_levels=0, gamma=Fraction(1)):
    """Sequential Louvain with the paper's Delta-mod in fractions.

    Per level: singletons; sweeps visit nodes in descending priority; node u in
    community C moves to the neighbouring community D maximising
      Delta-mod(u, C -> D) = (w(u,D\\u) - w(u,C\\u)) / w(E)
                             + (vol(C\\u) - vol(D\\u)) vol(u) / (2 w(E)^2)
    (lowest D among equal values) if that value is > 0; with a resolution gamma
    the volume term is multiplied by gamma.  A level stops after a
    sweep without moves or max_sweeps sweeps; the run descends iff communities
    merged; coarse ids ascend with the old community ids; intra-community
    weight becomes a self-loop.  Returns canonical labels of the input nodes.
    """
    lab = list(range(n))               # input node -> current level node
    level = 0
    cur_n, cur_edges = n, dict(edges)
    while True:
        W = Fraction(sum(cur_edges.values()))
        adj = [dict() for _ in range(cur_n)]
        vol = [0] * cur_n
        for (u, v), wt in cur_edges.items():
            if u == v:
                vol[u] += 2 * wt
            else:
                adj[u][v] = wt
                adj[v][u] = wt
                vol[u] += wt
                vol[v] += wt
        zeta = list(range(cur_n))
        volC = list(vol)
        order = priority_order(cur_n, seed, level)
        for _ in range(max_sweeps):
            moves = 0
            for u in order:
                C = zeta[u]
                wto = {}
                for v, wt in adj[u].items():
                    wto[zeta[v]] = wto.get(zeta[v], 0) + wt
                best, bestD = None, None
                for D in sorted(wto):
                    if D == C:
                        continue
                    delta = (Fraction(wto[D] - wto.get(C, 0)) / W
                             + gamma * Fraction((volC[C] - vol[u]) - volC[D]) * vol[u] / (2 * W * W))
                    if best is None or delta > best:
                        best, bestD = delta, D
                if best is not None and best > 0:
                    volC[C] -= vol[u]
                    volC[bestD] += vol[u]
                    zeta[u] = bestD
                    moves += 1
            if moves == 0:
                break
        ids = sorted(set(zeta))
        level += 1
        if len(ids) == cur_n or (max_levels and level >= max_levels):
            lab = [zeta[x] for x in lab]
            break
        newid = {c: i for i, c in enumerate(ids)}
        pi = [newid[zeta[u]] for u in range(cur_n)]
        coarse = {}
        for (u, v), wt in cur_edges.items():
            a, b = sorted((pi[u], pi[v]))
            coarse[(a, b)] = coarse.get((a, b), 0) + wt
        lab = [pi[x] for x in lab]
        cur_n, cur_edges = len(ids), coarse
    canon, out = {}, []
    for x in lab:
        canon.setdefault(x, len(canon))
        out.append(canon[x])
    return np.array(out, dtype=np.int32)


def seq_plmr(n, edges, seed=0, max_sweeps=32, max_levels=0, first_level=0):
    """PLMR (Algorithm 4) with the sequential schedule and the paper's
    Delta-mod in fractions, written recursively as the algorithm is stated:
    move from singletons; if communities merged, coarsen, recurse, prolong
    (u takes the community of its coarse node, named by that node's community
    id on the coarse level) and move again from the prolonged communities.
    Moves, ties and coarse ids follow seq_louvain.  The input graph is level
    first_level (priorities are drawn for that level; max_levels counts from
    it).  Returns canonical labels."""

    def graph(cur_n, cur_edges):
        adj = [dict() for _ in range(cur_n)]
        vol = [0] * cur_n
        for (u, v), wt in cur_edges.items():
            if u == v:
                vol[u] += 2 * wt
            else:
                adj[u][v] = wt
                adj[v][u] = wt
                vol[u] += wt
                vol[v] += wt
        return adj, vol, Fraction(sum(cur_edges.values()))

    def move(cur_n, adj, vol, W, zeta, level):
        volC = [0] * cur_n
        for u in range(cur_n):
            volC[zeta[u]] += vol[u]
        order = priority_order(cur_n, seed, level)
        for _ in range(max_sweeps):
            moves = 0
            for u in order:
                C = zeta[u]
                wto = {}
                for v, wt in adj[u].items():
                    wto[zeta[v]] = wto.get(zeta[v], 0) + wt
                best, bestD = None, None
                for D in sorted(wto):
                    if D == C:
                        continue
                    delta = (Fraction(wto[D] - wto.get(C, 0)) / W
                             + Fraction((volC[C] - vol[u]) - volC[D]) * vol[u] / (2 * W * W))
                    if best is None or delta > best:
                        best, bestD = delta, D
                if best is not None and best > 0:
                    volC[C] -= vol[u]
                    volC[bestD] += vol[u]
                    zeta[u] = bestD
                    moves += 1
            if moves == 0:
                break
        return zeta

    def rec(cur_n, cur_edges, level):
        adj, vol, W = graph(cur_n, cur_edges)
        zeta = move(cur_n, adj, vol, W, list(range(cur_n)), level)
        ids = sorted(set(zeta))
        if len(ids) == cur_n or (max_levels and level - first_level + 1 >= max_levels):
            return zeta
        newid = {c: i for i, c in enumerate(ids)}
        pi = [newid[zeta[u]] for u in range(cur_n)]
        coarse = {}
        for (u, v), wt in cur_edges.items():
            a, b = sorted((pi[u], pi[v]))
            coarse[(a, b)] = coarse.get((a, b), 0) + wt
        zc = rec(len(ids), coarse, level + 1)
        zeta = [zc[pi[u]] for u in range(cur_n)]
        return move(cur_n, adj, vol, W, zeta, level)

    z = rec(n, dict(edges), first_level)
    canon, out = {}, []
    for x in z:
        canon.setdefault(x, len(canon))
        out.append(canon[x])
    return np.array(out, dtype=np.int32)


def seq_plp(off, col, w, colours, seed=0, level=0, max_iters=64, active_sets=True):
    """Label propagation (Algorithm 1) over the given colour classes, in plain
    Python: classes in ascending colour, each deciding against the labels at
    its start; dominant label by weight over non-loop neighbours, own label
    kept when it attains the maximum, else the largest tie key
    t(v, l) = SplitMix64(H(seed, level, v) ^ l) >> 32, then the lowest label;
    active sets as in the algorithm (or every node every iteration); stop when
    updated <= n * 10^-5.  Returns (labels as node ids, updates per iteration)."""
    n = len(off) - 1
    wts = np.ones(len(col), np.int64) if w is None else np.asarray(w, np.int64)
    zeta = list(range(n))
    active = [any(int(c) != v for c in col[off[v]:off[v + 1]]) for v in range(n)]
    has_nb = list(active)
    classes = {}
    for v in range(n):
        classes.setdefault(int(colours[v]), []).append(v)
    updates, updated, it = [], n, 0
    while updated * 100000 > n and it < max_iters:
        updated = 0
        for c in sorted(classes):
            dec = {}
            for v in classes[c]:
                if not (active[v] if active_sets else has_nb[v]):
                    continue
                acc = {}
                for e in range(off[v], off[v + 1]):
                    u = int(col[e])
                    if u != v:
                        acc[zeta[u]] = acc.get(zeta[u], 0) + int(wts[e])
                own = zeta[v]
                hv = splitmix64(seed ^ (level << 40) ^ v)
                cands = [(acc[l], splitmix64(hv ^ l) >> 32, -l) for l in acc if l != own]
                best = max(cands) if cands else None
                dec[v] = -best[2] if best is not None and best[0] > acc.get(own, 0) else own
            for v, l in dec.items():
                if l != zeta[v]:
                    zeta[v] = l
                    updated += 1
                    for e in range(off[v], off[v + 1]):
                        if int(col[e]) != v:
                            active[int(col[e])] = True
                else:
                    active[v] = False
        updates.append(updated)
        it += 1
    return np.array(zeta, np.int32), updates
