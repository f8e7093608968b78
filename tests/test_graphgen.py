"""Structure of the seeded synthetic inputs (CPU)."""
import numpy as np
import pytest

import graphgen


def _check_csr(g, loops_allowed=False):
    n = g.n
    assert g.off[0] == 0 and g.off[-1] == g.nnz and np.all(np.diff(g.off) >= 0)
    rows = np.repeat(np.arange(n), np.diff(g.off))
    assert np.all((g.col >= 0) & (g.col < n))
    for u in range(min(n, 2000)):
        r = g.col[g.off[u]:g.off[u + 1]]
        assert np.all(np.diff(r) > 0)
    if not loops_allowed:
        assert not np.any(rows == g.col)
    key = rows.astype(np.int64) * n + g.col
    tkey = g.col.astype(np.int64) * n + rows
    order = np.argsort(tkey)
    assert np.array_equal(np.sort(key), tkey[order])
    if g.w is not None:
        assert np.array_equal(g.w[np.argsort(key)], g.w[order])


@pytest.mark.parametrize("scale,weighted", [(8, False), (10, True), (12, False)])
def test_rmat_structure_and_determinism(scale, weighted):
    g = graphgen.rmat(scale, 16, seed=5, weighted=weighted)
    _check_csr(g)
    g2 = graphgen.rmat(scale, 16, seed=5, weighted=weighted)
    assert np.array_equal(g.off, g2.off) and np.array_equal(g.col, g2.col)
    if weighted:
        assert g.w.min() >= 1 and g.w.max() <= 100
    deg = np.diff(g.off)
    assert deg.max() > 8 * deg[deg > 0].mean()          # skewed tail


def test_rmat_perm_is_bijection():
    s = 12
    img = {graphgen.rmat_perm(x, s, 9) for x in range(1 << s)}
    assert img == set(range(1 << s))


def test_planted_partition_shape():
    g = graphgen.planted_partition_1000()
    _check_csr(g)
    assert g.n == 1000 and g.w is None
    rows = np.repeat(np.arange(1000), np.diff(g.off))
    inside = (rows // 100) == (g.col // 100)
    m_in, m_out = inside.sum() // 2, (~inside).sum() // 2
    assert abs(m_in - 4950) < 5 * np.sqrt(4950) and abs(m_out - 2250) < 5 * np.sqrt(2250)


def test_batch_params():
    n, k, pin, pout, gs = graphgen.batch_params(4, 4096)
    assert n.min() >= 100 and n.max() < 100000
    assert np.all(k == np.maximum(2, n // 100))
    assert 9000 < n.mean() < 20000


def test_small_families():
    g = graphgen.ring_of_cliques(5, 4)
    _check_csr(g)
    assert g.undirected_edges() == 5 * 6 + 5
    g = graphgen.random_graph(30, 0.3, seed=1, loops=0.5)
    _check_csr(g, loops_allowed=True)


def test_serve_params_recipe():
    """Served workload: deterministic, exponential gaps of mean 1/rate, scales
    uniform over [12, 22], distinct request seeds."""
    a1, s1, d1 = graphgen.serve_params(5, 4000, 200.0)
    a2, s2, d2 = graphgen.serve_params(5, 4000, 200.0)
    assert np.array_equal(a1, a2) and np.array_equal(s1, s2) and np.array_equal(d1, d2)
    gaps = np.diff(np.concatenate([[0.0], a1]))
    assert np.all(gaps > 0) and abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    assert abs(np.median(gaps) - np.log(2) / 200.0) < 0.15 / 200.0      # exponential median
    assert s1.min() == 12 and s1.max() == 22
    counts = np.bincount(s1 - 12)
    assert counts.min() > 4000 / 11 * 0.8
    assert len(np.unique(d1)) == 4000
