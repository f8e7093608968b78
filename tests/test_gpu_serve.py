"""The request server (plm_server_*): every completed request carries exactly
the oracle's run on its graph (labels, Q bit for bit, levels), whatever it was
batched with and whatever ran beside it; admission keeps submission order under
the HBM budget and the per-batch entry cap; an invalid graph fails alone; with
several batches in flight, requests that arrive while a batch runs start beside
it, within the budget; with continuous batching (join = 1) requests that arrive
while a batch runs join it at its level boundaries, each with the result of its
own run alone."""
from __future__ import annotations

import sys
import time

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


def _graphs():
    return [
        graphgen.planted_partition_1000(seed=5),
        graphgen.rmat(11, 16, seed=21, weighted=False),
        graphgen.ring_of_cliques(6, 4),
        graphgen.from_edges(4, []),
        graphgen.random_graph(90, 0.08, seed=8, weighted=True, loops=0.2),
        graphgen.rmat(12, 16, seed=22, weighted=True),
        graphgen.disjoint_edges(5),
    ]


def _check(g, res):
    ready, labels, q, lv = res
    r = oracle.run(g.off, g.col, g.w)
    assert ready
    assert np.array_equal(labels, r.labels[: g.n]) and q == r.q and lv == r.levels


def _drain(srv, ids):
    out = {}
    steps = 0
    while len(out) < len(ids):
        srv.step()
        steps += 1
        for i in ids:
            if i not in out:
                res = srv.result(i)
                if res[0]:
                    out[i] = res
        assert steps <= 4 * len(ids)
    return out, steps


def test_server_results_match_oracle(P):
    _say("server: one batch")
    gs = _graphs()
    with P.Server(1 << 34) as srv:
        ids = [srv.submit(g.off, g.col, g.w) for g in gs]
        out, steps = _drain(srv, ids)
        assert steps == 1 and srv.info().completed == len(gs) and srv.info().batches == 1
    for g, i in zip(gs, ids):
        _check(g, out[i])


def test_server_budget_keeps_order(P):
    _say("server: tight budget")
    gs = _graphs()
    # the budget holds the largest request alone, so the requests take several steps
    fp = [8 * (g.n + 1) + 8 * g.nnz + 128 * g.n + 64 * g.nnz for g in gs]
    with P.Server(max(fp) + 1) as srv:
        ids = [srv.submit(g.off, g.col, g.w) for g in gs]
        out, steps = {}, 0
        while len(out) < len(ids):
            srv.step()
            steps += 1
            assert steps <= len(ids)
            # submission order: the completed requests are always a prefix
            first_waiting = None
            for k, i in enumerate(ids):
                if i in out:
                    continue
                res = srv.result(i)
                if res[0]:
                    assert first_waiting is None, f"request {k} completed before an earlier one"
                    out[i] = res
                elif first_waiting is None:
                    first_waiting = k
        assert steps > 1
    for g, i in zip(gs, ids):
        _check(g, out[i])


def test_server_entry_cap(P):
    _say("server: entry cap")
    gs = [graphgen.rmat(10, 16, seed=s, weighted=False) for s in range(4)]
    with P.Server(1 << 34, max_batch_entries=max(g.nnz for g in gs)) as srv:
        ids = [srv.submit(g.off, g.col, g.w) for g in gs]
        out, steps = _drain(srv, ids)
        assert steps == len(gs)
    for g, i in zip(gs, ids):
        _check(g, out[i])


def test_server_device_inputs_and_invalid_request(P):
    import torch
    _say("server: device inputs, invalid request")
    gs = _graphs()[:3]
    d = torch.device("cuda:0")
    bad = graphgen.disjoint_cliques(2, 3)
    bad_col = bad.col.copy()
    bad_col[0] = 2                      # row 0 becomes [2, 2]: not strictly ascending
    with P.Server(1 << 34) as srv:
        keep = []
        ids = []
        for k, g in enumerate(gs):
            if k == 1:
                ids.append(srv.submit(bad.off, bad_col, bad.w))
            t = [torch.from_numpy(x).to(d) for x in (g.off, g.col)] + \
                [None if g.w is None else torch.from_numpy(g.w).to(d)]
            keep.append(t)
            ids.append(srv.submit(t[0], t[1], t[2], n=g.n, nnz=g.nnz))
        for _ in range(8):
            srv.step()
            if srv.info().queued == 0:
                break
        assert srv.info().queued == 0
        bad_id = ids.pop(1)
        with pytest.raises(P.PLMError) as e:
            srv.result(bad_id)
        assert e.value.status == P.PLM_E_GRAPH
        for g, i in zip(gs, ids):
            lab = torch.empty(max(g.n, 1), dtype=torch.int32, device=d)
            ready, _, q, lv = srv.result(i, lab)
            _check(g, (ready, lab.cpu().numpy()[: g.n], q, lv))


def test_server_empty_step(P):
    with P.Server(1 << 30) as srv:
        assert srv.step() == 0 and srv.info().batches == 0


def _drain_async(srv, ids, budget):
    """Steps and polls until every request is ready; checks the budget and
    returns (results, most batches seen in flight at once)."""
    out, most = {}, 0
    for _ in range(100000):
        srv.step()
        info = srv.info()
        assert info.resident_bytes <= budget
        most = max(most, info.inflight)
        for i in ids:
            if i not in out:
                res = srv.result(i)
                if res[0]:
                    out[i] = res
        if len(out) == len(ids):
            break
        time.sleep(0.001)
    srv.wait()
    assert len(out) == len(ids) and srv.info().inflight == 0
    return out, most


def test_server_async_results_match_oracle(P):
    _say("server: three batches in flight")
    gs = _graphs() + [graphgen.rmat(13, 16, seed=23, weighted=False)]
    fp = [8 * (g.n + 1) + 8 * g.nnz + 128 * g.n + 64 * g.nnz for g in gs]
    budget = max(fp) + 1   # the largest request fits only alone: several batches, some waiting for memory
    assert sum(fp) > budget
    with P.Server(budget, max_inflight=3) as srv:
        ids = [srv.submit(g.off, g.col, g.w) for g in gs]
        out, _ = _drain_async(srv, ids, budget)
        assert srv.info().completed == len(gs) and srv.info().batches >= 2
    for g, i in zip(gs, ids):
        _check(g, out[i])


def test_server_async_admits_beside_a_running_batch(P):
    """A large request runs; small ones submitted meanwhile start in batches of
    their own beside it (a second batch is in flight before the first ends)."""
    _say("server: arrivals during a running batch")
    big = graphgen.rmat(18, 16, seed=24, weighted=False)
    small = [graphgen.planted_partition_1000(seed=s) for s in range(6, 9)] + [graphgen.rmat(10, 16, seed=25)]
    budget = 1 << 36
    with P.Server(budget, max_inflight=2) as srv:
        ids = [srv.submit(big.off, big.col, big.w)]
        srv.step()
        ids += [srv.submit(g.off, g.col, g.w) for g in small]
        srv.step()
        seen = srv.info().inflight
        out, most = _drain_async(srv, ids, budget)
        assert max(seen, most) == 2
    for g, i in zip([big] + small, ids):
        _check(g, out[i])


def test_server_async_invalid_request_and_device_inputs(P):
    import torch
    _say("server: async invalid request")
    gs = _graphs()[:4]
    d = torch.device("cuda:0")
    bad = graphgen.disjoint_cliques(2, 3)
    bad_col = bad.col.copy()
    bad_col[0] = 2
    with P.Server(1 << 34, max_inflight=4) as srv:
        ids, keep = [], []
        for k, g in enumerate(gs):
            if k == 2:
                bad_id = srv.submit(bad.off, bad_col, bad.w)
            t = [torch.from_numpy(x).to(d) for x in (g.off, g.col)] + \
                [None if g.w is None else torch.from_numpy(g.w).to(d)]
            keep.append(t)
            ids.append(srv.submit(t[0], t[1], t[2], n=g.n, nnz=g.nnz))
        for _ in range(100000):
            srv.step()
            if srv.info().queued == 0 and srv.info().inflight == 0:
                break
            time.sleep(0.001)
        srv.wait()
        with pytest.raises(P.PLMError) as e:
            srv.result(bad_id)
        assert e.value.status == P.PLM_E_GRAPH
        for g, i in zip(gs, ids):
            lab = torch.empty(max(g.n, 1), dtype=torch.int32, device=d)
            ready, _, q, lv = srv.result(i, lab)
            _check(g, (ready, lab.cpu().numpy()[: g.n], q, lv))


# ------------------------------------------------------------------ continuous batching (join = 1)
def _drain_join(srv, ids, budget=None):
    out = {}
    for _ in range(400000):
        srv.step()
        if budget is not None:
            assert srv.info().resident_bytes <= budget
        for i in ids:
            if i not in out:
                res = srv.result(i)
                if res[0]:
                    out[i] = res
        if len(out) == len(ids):
            break
        time.sleep(0.001)
    srv.wait()
    assert len(out) == len(ids)
    return out


def _check_opts(g, res, **kw):
    ready, labels, q, lv = res
    r = oracle.run(g.off, g.col, g.w, **kw)
    assert ready
    assert np.array_equal(labels, r.labels[: g.n]) and q == r.q and lv == r.levels


def test_server_join_results_match_oracle(P):
    """Requests submitted while a large one runs join its batch at a level
    boundary; each result is the oracle's run of its graph alone."""
    _say("server: continuous batching")
    big = graphgen.rmat(18, 16, seed=24, weighted=True)
    small = _graphs() + [graphgen.rmat(13, 16, seed=26, weighted=True), graphgen.rmat(12, 16, seed=27)]
    with P.Server(1 << 36, join=1) as srv:
        ids = [srv.submit(big.off, big.col, big.w)]
        srv.step()                                    # the batch starts on the server's worker
        ids += [srv.submit(g.off, g.col, g.w) for g in small]
        out = _drain_join(srv, ids)
        info = srv.info()
        _say(f"joined {info.joined} of {len(small)}, batches {info.batches}")
        assert info.joined >= 1 and info.completed == len(ids)
    for g, i in zip([big] + small, ids):
        _check(g, out[i])


def test_server_join_level_cap_and_device_inputs(P):
    """Joined graphs count their own levels (max_levels) and hash their own
    level into the priorities; device inputs join too."""
    import torch
    _say("server: joins with a level cap")
    d = torch.device("cuda:0")
    big = graphgen.rmat(17, 16, seed=31, weighted=False)
    small = [graphgen.rmat(12, 16, seed=32 + k, weighted=k % 2 == 0) for k in range(4)] + \
        [graphgen.planted_partition_1000(seed=9)]
    keep = []
    with P.Server(1 << 36, join=1, max_levels=2) as srv:
        ids = [srv.submit(big.off, big.col, big.w)]
        srv.step()
        for g in small:
            t = [torch.from_numpy(x).to(d) for x in (g.off, g.col)] + \
                [None if g.w is None else torch.from_numpy(g.w).to(d)]
            keep.append(t)
            ids.append(srv.submit(t[0], t[1], t[2], n=g.n, nnz=g.nnz))
        torch.cuda.synchronize()
        for _ in range(400000):
            srv.step()
            if srv.info().queued == 0 and srv.info().inflight == 0:
                break
            time.sleep(0.001)
        srv.wait()
        _say(f"joined {srv.info().joined}")
        _check_opts(big, srv.result(ids[0]), max_levels=2)
        for g, i in zip(small, ids[1:]):
            lab = torch.empty(max(g.n, 1), dtype=torch.int32, device=d)
            ready, _, q, lv = srv.result(i, lab)
            _check_opts(g, (ready, lab.cpu().numpy()[: g.n], q, lv), max_levels=2)


def test_server_join_budget_and_invalid_request(P):
    """Joins stay within the budget (a request that does not fit waits for a
    later batch) and an invalid joining graph fails alone."""
    _say("server: joins under a budget, invalid joiner")
    big = graphgen.rmat(17, 16, seed=41, weighted=True)
    mid = graphgen.rmat(15, 16, seed=42, weighted=True)
    small = [graphgen.planted_partition_1000(seed=s) for s in (11, 12)] + [graphgen.rmat(11, 16, seed=43)]
    bad = graphgen.disjoint_cliques(2, 3)
    bad_col = bad.col.copy()
    bad_col[0] = 2
    fp = lambda g: 8 * (g.n + 1) + 8 * g.nnz + 128 * g.n + 64 * g.nnz
    budget = fp(big) + sum(fp(g) for g in small) + fp(bad) + fp(mid) // 2   # mid fits only after big is done
    with P.Server(budget, join=1) as srv:
        ids = [srv.submit(big.off, big.col, big.w)]
        srv.step()
        ids.append(srv.submit(mid.off, mid.col, mid.w))
        bad_id = srv.submit(bad.off, bad_col, bad.w)
        ids += [srv.submit(g.off, g.col, g.w) for g in small]
        out = _drain_join(srv, ids, budget)
        with pytest.raises(P.PLMError) as e:
            srv.result(bad_id)
        assert e.value.status == P.PLM_E_GRAPH
        assert srv.info().resident_bytes == 0
    for g, i in zip([big, mid] + small, ids):
        _check(g, out[i])
