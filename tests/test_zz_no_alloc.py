"""plm_modularity_noalloc (the allocation-free variant of plm_modularity,
whose workspace is a static device array) against plm_modularity on the same
labels: bit-equal Q on two calls in a row, the second on a smaller graph, and
a third back on the first graph (the workspace keeps the last call's contents,
which every call clears before use); the node limit and argument errors."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1304_4453_amd as P
    return P


def _labels_sets(n, rng):
    yield np.arange(n, dtype=np.int32)                       # singletons
    yield np.zeros(n, dtype=np.int32)                        # one community
    yield rng.integers(0, max(1, n // 50), n).astype(np.int32)
    yield rng.integers(0, n, n).astype(np.int32)


def _check(P, ctx, labels_np):
    import torch
    dev = torch.from_numpy(labels_np).to("cuda:0")
    torch.cuda.synchronize()
    q_ref = ctx.modularity(dev)
    q_na = ctx.modularity_noalloc(dev)
    assert q_na == q_ref, (q_na, q_ref)
    return q_na


def test_noalloc_modularity_matches(P):
    import torch
    rng = np.random.default_rng(11)
    big = graphgen.rmat(14, 16, seed=5, weighted=True)
    small = graphgen.planted_partition_1000(seed=1)
    with P.Context(big.off, big.col, big.w) as cb, P.Context(small.off, small.col, None) as cs:
        lab = torch.empty(big.n, dtype=torch.int32, device="cuda:0")
        _, q_run, _ = cb.run(lab)
        assert cb.modularity_noalloc(lab) == q_run
        for L in _labels_sets(big.n, rng):
            _check(P, cb, L)
        # the second call in a row on a smaller input
        for L in _labels_sets(small.n, rng):
            _check(P, cs, L)
        lab_s = torch.empty(small.n, dtype=torch.int32, device="cuda:0")
        _, q_s, _ = cs.run(lab_s)
        assert cs.modularity_noalloc(lab_s) == q_s
        # back on the larger graph after the smaller one
        for L in _labels_sets(big.n, rng):
            _check(P, cb, L)
        # labels out of range: an error, then the next call is correct again
        bad = torch.full((big.n,), big.n, dtype=torch.int32, device="cuda:0")
        with pytest.raises(P.PLMError):
            cb.modularity_noalloc(bad)
        assert cb.modularity_noalloc(lab) == q_run
        # host (pinned) memory is refused
        pinned = torch.zeros(big.n, dtype=torch.int32).pin_memory()
        with pytest.raises(P.PLMError):
            cb.modularity_noalloc(pinned)


def test_noalloc_node_limit(P):
    import torch
    n = P.PLM_NOALLOC_MAX_NODES + 1
    off = np.zeros(n + 1, np.int64)
    col = np.zeros(0, np.int32)
    with P.Context(off, col, None) as ctx:
        lab = torch.zeros(n, dtype=torch.int32, device="cuda:0")
        with pytest.raises(P.PLMError):
            ctx.modularity_noalloc(lab)
        assert ctx.modularity(lab) == 0.0
    # exactly at the limit: accepted (an edgeless graph has Q = 0)
    n = P.PLM_NOALLOC_MAX_NODES
    off = np.zeros(n + 1, np.int64)
    with P.Context(off, col, None) as ctx:
        lab = torch.arange(n, dtype=torch.int32, device="cuda:0")
        assert ctx.modularity_noalloc(lab) == ctx.modularity(lab) == 0.0
