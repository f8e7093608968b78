"""Benchmark: PLM move-sweep edges/s on one MI355X, with the HBM roofline of the
dominant move-decide kernel and the oracle's CPU rate on a bounded sample.

One step = one full multilevel PLM run (plm_run: level set-up, colouring, class
bucketing, move sweeps, coarsening, prolongation, canonical labels) on a graph
already resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat26|rmat20|pp1000] [--no-batch]

The line also carries "plmr": one PLMR run (Algorithm 4) on the same graph;
"plp": label propagation (Algorithm 1) on the same graph, with the roofline of
its first iteration; "epp": EPP(4, PLP, PLMR) (Algorithm 5) on the same graph;
"gamma": R-MAT 20 runs at resolutions 1/2, 1 and 2;
"batched": the batched engine (plm_batch_run) on 4,096
uneven SBM graphs against a per-graph plm_run loop on the same GPU; and
"served": the request server (plm_server_*) under Poisson arrivals, with
p50/p99 latency and graphs/s.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNELS = ["k_decide_lane", "k_decide_wave", "k_decide_block", "k_hub_single", "k_hub_part+k_hub_agg"]

WORKLOADS = {
    "rmat26": dict(desc="R-MAT scale 26, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, loops and "
                        "duplicates removed, integer weights uniform in [1,100], seed 3",
                   scale=26, seed=3, weighted=True),
    "rmat20": dict(desc="R-MAT scale 20, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, loops and "
                        "duplicates removed, unit weights, seed 2", scale=20, seed=2, weighted=False),
    "pp1000": dict(desc="planted partition n=1000, 10 blocks of 100, p_in=0.1, p_out=0.005, unit weights, seed 1"),
}


def group_times(st, level):
    """Device ms and algorithmic bytes of the five move-decide kernel groups at a level."""
    bm, bb = st["bin_ms"][level], st["bin_bytes"][level]
    ms = [bm[0], bm[1], bm[2], st["hub_single_ms"][level], bm[3] - st["hub_single_ms"][level]]
    by = [bb[0], bb[1], bb[2], st["hub_single_bytes"][level], bb[3] - st["hub_single_bytes"][level]]
    return ms, by


def dominant(st):
    """(level, group) of the move-decide kernel group with the most device time over the run."""
    best = (0, 0, -1.0)
    for level in range(st["levels"]):
        ms, _ = group_times(st, level)
        for k in range(5):
            if ms[k] > best[2]:
                best = (level, k, ms[k])
    return best[0], best[1]


def roofline(st, level=0, k=None):
    """Roofline of a move-decide kernel group (by default the one with the most
    device time at the level): algorithmic bytes (per entry of a scanned row
    its column, weight and neighbour community; per distinct candidate its
    volume; per decided node 32 bytes; per settled node the 36 bytes of its
    check) over the group's event-timed duration, against the HBM peak."""
    ms, by = group_times(st, level)
    if k is None:
        k = max(range(5), key=lambda i: ms[i])
    launches = st["kernel_launches"][level][k]
    achieved = by[k] / (ms[k] * 1e6) if ms[k] > 0 else 0.0
    sweeps = max(st["sweeps"][level], 1)
    return {"bound": "hbm", "kernel": KERNELS[k], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "level": level, "launches": launches, "avg_launch_us": ms[k] * 1e3 / max(launches, 1),
            "algorithmic_bytes_per_launch": by[k] / max(launches, 1),
            "algorithmic_bytes_per_sweep": by[k] / sweeps, "kernel_ms_per_sweep": ms[k] / sweeps,
            "all_decide_GBs": st["decide_bytes"][level] / (st["decide_ms"][level] * 1e6)
            if st["decide_ms"][level] else 0.0,
            # every decide kernel of every level and executed sweep together
            "all_levels_decide_GBs": sum(st["decide_bytes"]) / (sum(st["decide_ms"]) * 1e6)
            if sum(st["decide_ms"]) else 0.0,
            "kernels": KERNELS, "kernel_ms": ms, "kernel_bytes": by,
            "decided_nodes": st["decided_nodes"][level], "settled_nodes": st["settled_nodes"][level],
            "decided_entries": st["decided_entries"][level]}


def level_summary(st):
    """Per level: the dominant decide group's roofline, all decide kernels
    together, the skipped (settled) decisions, and the colouring's rounds."""
    out = []
    for level in range(min(st["levels"], 4)):
        r = roofline(st, level)
        out.append({"level": level, "dominant_kernel": r["kernel"], "achieved_GBs": r["achieved"],
                    "frac": r["frac"], "avg_launch_us": r["avg_launch_us"],
                    "all_decide_GBs": r["all_decide_GBs"], "decide_ms": st["decide_ms"][level],
                    "decided_nodes": st["decided_nodes"][level], "settled_nodes": st["settled_nodes"][level],
                    "colour_rounds": st["schedule_rounds"][level], "colour_ms": st["colour_ms"][level],
                    "colour_us_per_round": st["colour_ms"][level] * 1e3 / max(st["schedule_rounds"][level], 1)})
    return out


def counter_traffic(kernel, level=0):
    """Per-launch HBM traffic of a move-decide kernel group from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or
    None when the kernels' source has changed since the counters were taken or
    the summary covers another level."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "decide_traffic_rmat26.md")
    src = os.path.join(ROOT, "paper_1304_4453_amd", "csrc", "move.hip")
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if blob["move_hip_sha256"] != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        if blob.get("level", 0) != level:
            return None
        for k in blob["kernels"]:
            if k["kernel"] == kernel:
                return {"bytes_per_launch": k["traffic_bytes_per_launch"],
                        "algorithmic_bytes_per_launch_same_sweep": k["algorithmic_bytes_per_launch"],
                        "fetch_scale": blob["fetch_scale"], "write_scale": blob["write_scale"],
                        "source": f"profiles/decide_traffic_rmat26.md (level-{level} sweep)"}
    except (OSError, KeyError, IndexError, ValueError):
        return None
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """CPU model, logical cores and RAM of the host the benchmark runs on."""
    model, mem_kb = platform.processor() or platform.machine(), None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem_kb = int(line.split()[1])
                break
    except OSError:
        pass
    return {"cpu": model, "logical_cores": os.cpu_count(), "ram_gib": None if mem_kb is None else round(mem_kb / 2**20, 1)}


def copy_peak(torch):
    """Device-to-device copy bandwidth (read + write bytes per second) of a
    4 GiB buffer, median of 5 copies timed with events on torch's stream."""
    x = torch.empty(1 << 30, dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = sorted(ts)[len(ts) // 2]
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * (4 << 30), "GBs": 2 * (4 << 30) / (ms * 1e6)}


def make_graph(name):
    """(device off, col, w pointers or tensors, n, nnz, m, keepalive, host_rows_fn)."""
    import torch
    import graphgen
    if name == "pp1000":
        g = graphgen.planted_partition_1000(seed=1)
        dev = torch.device("cuda:0")
        off = torch.from_numpy(g.off).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        torch.cuda.synchronize()
        return dict(off=off, col=col, w=None, n=g.n, nnz=g.nnz, m=g.undirected_edges(), host=g, dg=None)
    wl = WORKLOADS[name]
    dg = graphgen.rmat_gpu(wl["scale"], 16, seed=wl["seed"], weighted=wl["weighted"])
    return dict(off=dg.off_ptr, col=dg.col_ptr, w=dg.w_ptr or None, n=dg.n, nnz=dg.nnz, m=dg.nnz // 2, host=None,
                dg=dg)


def cpu_baseline(gr, ctx_state, budget_s=15.0):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    level-0, sweep-1 move decisions (singleton communities) of the movable nodes
    of a random contiguous node-id range (R-MAT ids are randomly relabelled, so
    the range is a uniform node sample and its rows are one contiguous CSR
    slice); rate = sampled undirected edges (entries / 2) per second."""
    import ctypes
    import numpy as np
    import graphgen
    import oracle
    n = gr["n"]
    zeta, volc, _ = ctx_state
    if gr["host"] is not None:
        g = gr["host"]
        off = g.off

        def get_rows(a, b):
            lo, hi = int(off[a]), int(off[b])
            return g.col[lo:hi].copy(), (None if g.w is None else g.w[lo:hi].copy())
    else:
        dg = gr["dg"]
        off = np.zeros(n + 1, np.int64)
        lib = graphgen._gpu_lib()
        lib.ggpu_copy_to_host(off.ctypes.data, ctypes.c_void_p(dg.off_ptr), off.nbytes)

        def get_rows(a, b):
            lo, hi = int(off[a]), int(off[b])
            c = np.zeros(hi - lo, np.int32)
            lib.ggpu_copy_to_host(c.ctypes.data, ctypes.c_void_p(dg.col_ptr + 4 * lo), c.nbytes)
            w = None
            if dg.w_ptr:
                w = np.zeros(hi - lo, np.int32)
                lib.ggpu_copy_to_host(w.ctypes.data, ctypes.c_void_p(dg.w_ptr + 4 * lo), w.nbytes)
            return c, w
    deg = np.diff(off)
    rng = np.random.default_rng(12345)
    vol = volc.astype(np.int64)
    S = int(vol.sum())

    def timed(count):
        count = min(count, n)
        a = int(rng.integers(0, n - count + 1))
        b = a + count
        scol, sw = get_rows(a, b)
        nodes = (a + np.nonzero(deg[a:b] > 0)[0]).astype(np.int32)
        soff = np.zeros(n + 1, np.int64)
        soff[a + 1:b + 1] = np.cumsum(deg[a:b])
        soff[b + 1:] = soff[b]
        sw = np.ones(len(scol), np.int64) if sw is None else sw.astype(np.int64)
        w2 = oracle.double_diagonal(soff, scol, sw)
        t = time.perf_counter()
        oracle.decide_many(nodes, soff, scol.astype(np.int32), w2, zeta, volc, vol, S)
        dt = time.perf_counter() - t
        return len(nodes), int(deg[a:b].sum()), dt

    k, e, dt = timed(min(n, 50_000))
    if dt < budget_s / 5 and k < n:
        k, e, dt = timed(int(min(n, 50_000 * budget_s / max(dt, 1e-3))))
    return {"value": (e / 2) / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"level-0 sweep-1 move decisions (singleton communities) of the {k} movable nodes of a random "
                      f"contiguous node-id range ({e} CSR entries) of the same graph; oracle single-threaded",
            "seconds": dt, "host": host_info()}


def cpu_full_run(P, torch, scale=18):
    """The oracle's whole PLM run (all levels) on R-MAT scale `scale` (unit
    weights, seed 2), single-threaded, phase by phase through its exported
    steps (volumes, colouring, sweeps until one moves nothing or 32, relabel,
    contraction), beside plm_run on the same graph on the GPU; both must give
    the same level trace."""
    import numpy as np
    import graphgen
    import oracle
    g = graphgen.rmat(scale, 16, seed=2, weighted=False)
    m = g.undirected_edges()
    off, col = g.off.astype(np.int64), g.col.astype(np.int32)
    w2 = oracle.double_diagonal(off, col, g.w)
    phases = {"colouring_s": 0.0, "sweeps_s": 0.0, "coarsening_s": 0.0, "volumes_s": 0.0}
    trace = []
    t_all = time.perf_counter()
    level = 0
    while True:
        t = time.perf_counter()
        vol, S = oracle.volumes(off, w2)
        phases["volumes_s"] += time.perf_counter() - t
        t = time.perf_counter()
        colours, C = oracle.colour(off, col, 0, level, 0)
        phases["colouring_s"] += time.perf_counter() - t
        zeta = np.arange(len(vol), dtype=np.int32)
        volC = vol.copy()
        t = time.perf_counter()
        sweeps = 0
        for _ in range(32):
            sweeps += 1
            if oracle.sweep(off, col, w2, vol, S, colours, C, zeta, volC) == 0:
                break
        phases["sweeps_s"] += time.perf_counter() - t
        t = time.perf_counter()
        pi, k = oracle.relabel(zeta)
        trace.append((len(vol), int(C), sweeps, int(k)))
        if k == len(vol):
            break
        off, col, w2 = oracle.contract(off, col, w2, pi, k)
        phases["coarsening_s"] += time.perf_counter() - t
        level += 1
    total = time.perf_counter() - t_all
    dev = torch.device("cuda:0")
    with P.Context(torch.from_numpy(g.off).to(dev), torch.from_numpy(g.col).to(dev), None, n=g.n, nnz=g.nnz,
                   mem_kind=P.PLM_MEM_DEVICE) as ctx:
        lab = torch.empty(g.n, dtype=torch.int32, device=dev)
        ctx.run(lab)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.run(lab)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t
        st = ctx.stats()
    gpu_trace = [(st["n"][i], st["colours"][i], st["sweeps"][i], st["communities"][i]) for i in range(st["levels"])]
    return {"graph": f"R-MAT scale {scale}, edge factor 16, unit weights, seed 2 ({g.n} nodes, {m} edges)",
            "seconds": total, "edges_per_s": m / total, "cores": 1,
            "phases_s": phases, "levels": len(trace), "same_level_trace_as_gpu": trace == gpu_trace,
            "gpu_plm_run_s": tg, "gpu_speedup": total / tg}


COMPILED_BINS = {"bin_lane": 16, "bin_wave": 512, "bin_block": 4096, "hub_row_max": 12288}
BATCH_DESC = ("4,096 SBM graphs, n log-uniform in [100, 100000], k = max(2, n/100) near-equal blocks, "
              "p_in = 20/blocksize, p_out = 1/n, unit weights, seed 4")


def batch_bench(args, P, torch, np):
    """Batched PLM: graphs/s of plm_batch_run over the whole batch, against a
    loop of plm_run over a random sample of the same graphs (contexts created
    beforehand, inputs resident in HBM for both); partitions, Q and levels of
    the sample must be identical.  The oracle's rate (plain C, one graph per
    host thread) is timed on a bounded sample."""
    from concurrent.futures import ThreadPoolExecutor
    import graphgen
    import oracle
    count = args.batch_graphs
    t = time.time()
    n, k, pin, pout, gs = graphgen.batch_params(4, count)
    workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(workers) as ex:
        graphs = list(ex.map(lambda i: graphgen.sbm(int(n[i]), int(k[i]), float(pin[i]), float(pout[i]), int(gs[i])),
                             range(count)))
    nb, off, col, w = P.pack_batch(graphs)
    log(f"batch: {count} graphs, n={nb[-1]} nnz={len(col)} built in {time.time() - t:.1f}s")
    ctx = P.BatchContext(nb, off, col, w, timing=1)  # instrumented step (see main)
    lab = torch.empty(int(nb[-1]), dtype=torch.int32, device="cuda:0")
    ctx.run_batch(lab)
    roof = roofline(ctx.stats())
    ctx.close()
    ctx = P.BatchContext(nb, off, col, w)
    for i in range(args.warmup):
        ctx.run_batch(lab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, q, lv = ctx.run_batch(lab)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    st = ctx.stats()
    o = ctx.options()
    tuned_bins = {k: int(getattr(o, k)) for k in COMPILED_BINS}
    labels = lab.cpu().numpy()
    ctx.close()
    log(f"batch run {tb * 1e3:.1f} ms (bins {tuned_bins})")
    # the same batch with the compiled bin thresholds, for the tuned table's gain
    ctx = P.BatchContext(nb, off, col, w, **COMPILED_BINS)
    lab_d = torch.empty_like(lab)
    for i in range(args.warmup):
        ctx.run_batch(lab_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, q_d, lv_d = ctx.run_batch(lab_d)
    torch.cuda.synchronize()
    td = (time.perf_counter() - t0) / args.steps
    ctx.close()
    same_d = bool(np.array_equal(lab_d.cpu().numpy(), labels) and np.array_equal(q_d, q) and np.array_equal(lv_d, lv))
    del lab_d
    log(f"batch run with compiled bins {td * 1e3:.1f} ms, identical: {same_d}")
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(count, min(args.plain_sample, count), replace=False))
    ctxs = [P.Context(graphs[i].off, graphs[i].col, graphs[i].w) for i in idx]
    outs = [torch.empty(max(graphs[i].n, 1), dtype=torch.int32, device="cuda:0") for i in idx]
    res = [c.run(o) for c, o in zip(ctxs, outs)]  # warm-up pass
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [c.run(o) for c, o in zip(ctxs, outs)]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    same = 0
    for j, i in enumerate(idx):
        a, b = int(nb[i]), int(nb[i + 1])
        same += int(np.array_equal(outs[j].cpu().numpy()[: b - a], labels[a:b]) and res[j][1] == q[i]
                    and res[j][2] == lv[i])
    for c in ctxs:
        c.close()
    log(f"plain loop over {len(idx)} graphs {tp * 1e3:.1f} ms")
    out = {"workload": BATCH_DESC, "graphs": count, "n": int(nb[-1]), "nnz": int(len(col)),
           "graphs_per_s": count / tb, "ms_per_run": tb * 1e3,
           "plain_graphs_per_s": len(idx) / tp, "plain_sample": int(len(idx)),
           "speedup_vs_plain": (count / tb) / (len(idx) / tp),
           "identical_partitions": f"{same}/{len(idx)}", "levels_max": int(lv.max()),
           "tuned_bins": {"bins": tuned_bins, "source": "paper_1304_4453_amd/tuned_bins.txt (batch row)",
                          "compiled_bins": COMPILED_BINS, "graphs_per_s_compiled_bins": count / td,
                          "gain": td / tb, "identical_partitions": same_d},
           "roofline": roof,
           "per_level": {k: st[k] for k in ("n", "nnz", "colours", "sweeps", "sweep_ms", "colour_ms",
                                            "coarsen_ms")}}
    if not args.no_cpu_baseline:
        order = rng.permutation(count)
        done, ge, t0 = 0, 0, time.perf_counter()

        def one(i):
            g = graphs[i]
            oracle.run(g.off, g.col, g.w)
            return g.nnz

        with ThreadPoolExecutor(workers) as ex:
            for s0 in range(0, count, workers):
                ge += sum(ex.map(one, order[s0:s0 + workers]))
                done += len(order[s0:s0 + workers])
                if time.perf_counter() - t0 > args.cpu_budget:
                    break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "graphs/s", "cores": workers, "kind": "oracle",
                               "sample": f"full oracle runs of {done} randomly chosen graphs of the batch "
                                         f"({ge} CSR entries), one graph per host thread",
                               "seconds": dt}
    return out


SERVE_DESC = ("Poisson arrivals at 200 req/s of R-MAT graphs, scale uniform in [12, 22], edge factor 16, "
              "a=.57 b=.19 c=.19 d=.05, unit weights, request seeds from seed 5; HBM budget 200 GB")


def serve_replay(P, torch, np, dgs, arr, check, join, inflight):
    """One open-loop real-time replay of the request stream against the native
    request server (join: level boundaries of a batch at which queued requests
    join it, 0 = fixed batches); returns (latencies, results of the checked
    requests, makespan, server info)."""
    count = len(dgs)
    check_lab = {i: torch.empty(dgs[i].n, dtype=torch.int32, device="cuda:0") for i in check}
    srv = P.Server(200 * 10 ** 9, max_inflight=inflight, join=join)
    ids, lat, done_q = {}, np.full(count, np.nan), {}
    nxt, t0 = 0, time.perf_counter()
    while len(done_q) < count:
        now = time.perf_counter() - t0
        while nxt < count and arr[nxt] <= now:
            d = dgs[nxt]
            ids[nxt] = srv.submit(d.off_ptr, d.col_ptr, None, mem_kind=P.PLM_MEM_DEVICE, n=d.n, nnz=d.nnz)
            nxt += 1
        if srv.info().queued > 0:
            srv.step()  # fixed batches, one in flight: runs a batch; otherwise hands one to a free worker
        tdone = time.perf_counter() - t0
        progressed = False
        for i, rid in list(ids.items()):
            if i in done_q:
                continue
            ready, _, q, lv = srv.result(rid, check_lab.get(i))
            if ready:
                done_q[i] = (q, lv)
                lat[i] = tdone - arr[i]
                progressed = True
        if not progressed:
            pause = 0.0005
            if srv.info().inflight == 0 and nxt < count:
                pause = max(0.0, min(arr[nxt] - (time.perf_counter() - t0), 0.01))
            time.sleep(pause)
    makespan = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    checked = {i: (check_lab[i].cpu().numpy(),) + done_q[i] for i in check}
    return lat, checked, makespan, info


# queued requests join a running batch at its first level boundary only: on the
# overloaded 200 req/s stream, depths 0 / 1 / 2 / 4 measured p50 13.95 / 13.68 /
# 14.19 / 14.38 s at 13.8 / 13.7 / 13.4 / 13.3 graphs/s (deeper joins add their
# level-0 classes to the running batch's later levels)
JOIN_DEPTH = 1


def serve_bench(args, P, torch, np):
    """Served PLM: the request stream of the arrival window is generated on the
    GPU first (client buffers), then replayed open-loop in real time against
    the native request server (plm_server_*), each request submitted at its
    arrival time; a request's latency is its result-ready time minus its
    arrival time.  Two replays of the same stream: continuous batching (join =
    JOIN_DEPTH: a running batch takes the queued requests in at its first level
    boundary and every request completes when its own run ends), then fixed batches (a step
    admits the queued requests that fit as one batch, which reports at its
    end; --serve-inflight batches at once)."""
    import graphgen
    import oracle
    rate = 200.0
    count = max(1, int(round(args.serve_seconds * rate)))
    arr, scales, seeds = graphgen.serve_params(5, count, rate)
    t = time.time()
    dgs = [graphgen.rmat_gpu(int(scales[i]), 16, seed=int(seeds[i]), weighted=False) for i in range(count)]
    torch.cuda.synchronize()
    edges = sum(d.nnz // 2 for d in dgs)
    log(f"serve: {count} requests ({edges} edges) generated in {time.time() - t:.1f}s")
    # a few small requests are checked against the oracle afterwards
    check = [i for i in range(count) if scales[i] <= 13][:3]
    lat, checked, makespan, info = serve_replay(P, torch, np, dgs, arr, check, JOIN_DEPTH, 1)
    log(f"serve (continuous batching): {count} requests in {makespan:.1f}s, {info.batches} batches, "
        f"{info.joined} joined a running batch")
    lat_f, checked_f, makespan_f, info_f = serve_replay(P, torch, np, dgs, arr, check, 0, args.serve_inflight)
    log(f"serve (fixed batches): {count} requests in {makespan_f:.1f}s over {info_f.batches} batches")
    for d in dgs:
        d.free()
    # the same kind of requests one by one through plm_run (random sample,
    # contexts created beforehand, inputs resident in HBM)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(count, min(args.plain_serve_sample, count), replace=False))
    ctxs, outs = [], []
    for i in sample:
        d = graphgen.rmat_gpu(int(scales[i]), 16, seed=int(seeds[i]), weighted=False)
        ctxs.append(P.Context(d.off_ptr, d.col_ptr, None, mem_kind=P.PLM_MEM_DEVICE, n=d.n, nnz=d.nnz))
        outs.append(torch.empty(d.n, dtype=torch.int32, device="cuda:0"))
        d.free()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for c, o in zip(ctxs, outs):
        c.run(o)
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    for c in ctxs:
        c.close()
    ok = 0
    for i in check:
        g = graphgen.rmat(int(scales[i]), 16, seed=int(seeds[i]), weighted=False)
        r = oracle.run(g.off, g.col, g.w)
        for res in (checked[i], checked_f[i]):
            ok += int(np.array_equal(res[0], r.labels[: g.n]) and res[1] == r.q and res[2] == r.levels)
    return {"workload": SERVE_DESC, "arrival_window_s": float(arr[-1]), "requests": count,
            "offered_req_per_s": rate, "offered_edges_per_s": edges / float(arr[-1]),
            "mode": "continuous batching (queued requests join the running batch at its first level boundary)",
            "join_depth": JOIN_DEPTH,
            "completed": int(np.isfinite(lat).sum()), "makespan_s": makespan, "graphs_per_s": count / makespan,
            "edges_per_s": edges / makespan, "p50_latency_s": float(np.nanpercentile(lat, 50)),
            "p99_latency_s": float(np.nanpercentile(lat, 99)), "max_latency_s": float(np.nanmax(lat)),
            "batches": int(info.batches), "joined": int(info.joined),
            "fixed_batches": {"max_inflight": args.serve_inflight, "makespan_s": makespan_f,
                              "graphs_per_s": count / makespan_f,
                              "p50_latency_s": float(np.nanpercentile(lat_f, 50)),
                              "p99_latency_s": float(np.nanpercentile(lat_f, 99)),
                              "batches": int(info_f.batches)},
            "plain_graphs_per_s": len(sample) / tp, "plain_sample": int(len(sample)),
            "speedup_vs_plain": (count / makespan) / (len(sample) / tp),
            "hbm_budget_bytes": 200 * 10 ** 9,
            "verified_vs_oracle": f"{ok}/{2 * len(check)} small requests over both replays (labels, Q, levels)",
            "note": "the offered load exceeds one GPU's throughput, so latency grows over the window; the window "
                    "is bounded (--serve-seconds, default 2 s of the 60 s stream) so that the run ends within "
                    "minutes: the full 60 s stream is not measured"}


def plmr_bench(gr, P, torch, q_plm, st_plm):
    """PLMR (Algorithm 4) on the same resident graph: one warm-up and one timed
    full run with refinement; its modularity beside PLM's."""
    ctx = P.Context(gr["off"], gr["col"], gr["w"], mem_kind=P.PLM_MEM_DEVICE, n=gr["n"], nnz=gr["nnz"], refine=1)
    lab = torch.empty(max(gr["n"], 1), dtype=torch.int32, device="cuda:0")
    ctx.run(lab)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, q, lv = ctx.run(lab)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    st = ctx.stats()
    ctx.close()
    m0 = (st["nnz"][0] - st["loops"][0]) // 2 + st["loops"][0]
    log(f"plmr step {dt:.2f}s q={q}")
    return {"ms_per_run": dt * 1e3, "full_run_edges_per_s": m0 / dt, "q": q, "q_plm": q_plm, "levels": lv,
            "refinement_ms": sum(st["ref_ms"]), "ref_sweeps": st["ref_sweeps"], "ref_moves": st["ref_moves"]}


def plp_bench(gr, P, torch):
    """Label propagation (Algorithm 1) on the same resident graph: one run with
    every decide dispatch event-timed (it gives the first iteration's
    roofline: every node is active there, so its algorithmic bytes are the
    whole graph's: per entry column, weight and neighbour label, per node 32
    bytes, no community volumes) and one timed run without events."""
    mk = lambda **kw: P.Context(gr["off"], gr["col"], gr["w"], mem_kind=P.PLM_MEM_DEVICE, n=gr["n"], nnz=gr["nnz"],
                                validate=0, **kw)
    lab = torch.empty(max(gr["n"], 1), dtype=torch.int32, device="cuda:0")
    ctx = mk(timing=1)
    ctx.plp(64, lab)
    st = ctx.stats()
    ctx.close()
    first_gbs = st["lp_first_bytes"] / (st["lp_first_ms"] * 1e6) if st["lp_first_ms"] else 0.0
    ctx = mk(timing=0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, q, it, upd = ctx.plp(64, lab)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    st2 = ctx.stats()
    ctx.close()
    m0 = gr["m"]
    log(f"plp {dt:.2f}s iterations={it} q={q}")
    return {"ms_per_run": dt * 1e3, "edges_per_s": m0 / dt, "iterations": it, "updates": upd, "q": q,
            "colouring_and_iterations_ms_host": st2["lp_ms"],
            "first_iteration": {"bound": "hbm", "achieved": first_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": first_gbs / HBM_PEAK_GBS, "decide_ms": st["lp_first_ms"],
                                "algorithmic_bytes": st["lp_first_bytes"],
                                "timing": "HIP events on every decide dispatch of the instrumented run"},
            "paper_context": "PLP >53M edges/s (uk-2007-05, 3.3e9 edges, 2x Xeon E5-2680, 32 threads)"}


def epp_bench(gr, P, torch, q_plm):
    """EPP(4, PLP, PLMR) (Algorithm 5) on the same resident graph: one timed run
    (the kernels are warm from the label-propagation runs before it)."""
    ctx = P.Context(gr["off"], gr["col"], gr["w"], mem_kind=P.PLM_MEM_DEVICE, n=gr["n"], nnz=gr["nnz"], validate=0)
    lab = torch.empty(max(gr["n"], 1), dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, q, lv, cores = ctx.epp(4, 64, lab)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    st = ctx.stats()
    ctx.close()
    log(f"epp {dt:.2f}s cores={cores} q={q}")
    return {"ensemble_size": 4, "ms_per_run": dt * 1e3, "edges_per_s": gr["m"] / dt, "q": q, "q_plm": q_plm,
            "core_groups": cores, "plmr_levels": lv, "plp_iterations": st["lp_iterations"],
            "plp_ms_host": st["lp_ms"], "core_group_ms_host": st["ens_ms"],
            "paper_context": "EPP(4,PLP,PLMR) about 219 s on uk-2007-05 (2x Xeon E5-2680, 32 threads)"}


def gamma_bench(P, torch):
    """Resolution gamma on R-MAT 20 (unit weights, seed 2) resident in HBM: one
    warm-up and one timed full run per gamma; time, Q and communities."""
    import graphgen
    dg = graphgen.rmat_gpu(20, 16, seed=2, weighted=False)
    out = []
    for num, den in [(1, 2), (1, 1), (2, 1)]:
        ctx = P.Context(dg.off_ptr, dg.col_ptr, None, mem_kind=P.PLM_MEM_DEVICE, n=dg.n, nnz=dg.nnz,
                        gamma_num=num, gamma_den=den)
        lab = torch.empty(dg.n, dtype=torch.int32, device="cuda:0")
        ctx.run(lab)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, q, lv = ctx.run(lab)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = ctx.stats()
        ctx.close()
        out.append({"gamma": f"{num}/{den}", "ms_per_run": dt * 1e3, "q": q, "levels": lv,
                    "communities": st["communities"][-1]})
    dg.free()
    return {"workload": "R-MAT scale 20, edge factor 16, unit weights, seed 2", "runs": out}


def sweep_probe(P, torch, level=0):
    """One move sweep of the R-MAT 26 workload at a level (level 1: after the
    level-0 move phase and its contraction) with every move-decide kernel
    timed, after a 1 GiB device copy that calibrates the HBM byte counters;
    for rocprofv3 --pmc runs.  Prints the sweep's per-kernel algorithmic bytes
    and launch counts as one JSON line."""
    import ctypes
    import graphgen
    wl = WORKLOADS["rmat26"]
    dg = graphgen.rmat_gpu(wl["scale"], 16, seed=wl["seed"], weighted=wl["weighted"])
    ctx = P.Context(dg.off_ptr, dg.col_ptr, dg.w_ptr, mem_kind=P.PLM_MEM_DEVICE, n=dg.n, nnz=dg.nnz, timing=1,
                    validate=0)
    dg.free()
    if level > 0:
        for _ in range(level):
            while ctx.move_sweep() > 0 and ctx.level_info().sweeps < 32:
                pass
            ctx.coarsen()
    x = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")  # 1 GiB
    y = x.clone()                                                # copy: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    del x, y
    st = P.plm_stats_t()
    P.plm_get_stats(ctx._c, ctypes.byref(st))
    b0 = (list(st.bin_bytes[level]), list(st.bin_ms[level]), st.hub_single_bytes[level], st.hub_single_ms[level],
          list(st.kernel_launches[level]))
    moves = ctx.move_sweep()
    P.plm_get_stats(ctx._c, ctypes.byref(st))
    bb = [a - b for a, b in zip(st.bin_bytes[level], b0[0])]
    bm = [a - b for a, b in zip(st.bin_ms[level], b0[1])]
    hb, hm = st.hub_single_bytes[level] - b0[2], st.hub_single_ms[level] - b0[3]
    out = {"workload": wl["desc"], "level": level, "sweep": ctx.level_info().sweeps, "moves": moves,
           "kernels": KERNELS, "kernel_bytes": [bb[0], bb[1], bb[2], hb, bb[3] - hb],
           "kernel_ms": [bm[0], bm[1], bm[2], hm, bm[3] - hm],
           "kernel_launches": [a - b for a, b in zip(st.kernel_launches[level], b0[4])],
           "calibration_copy_bytes": 1 << 30}
    ctx.close()
    print(json.dumps(out), flush=True)


GROUP_OF = {"k_decide_lane": "k_decide_lane", "k_decide_quad": "k_decide_wave", "k_decide_wave": "k_decide_wave",
            "k_decide_block": "k_decide_block", "k_hub_single": "k_hub_single", "k_hub_part": "k_hub_part+k_hub_agg",
            "k_hub_agg": "k_hub_part+k_hub_agg"}


def _kernel_base(name):
    """(base name, first template argument) of a kernel name in a rocprofv3 CSV."""
    short = name.replace("void ", "").replace("plm::", "").split("(")[0]
    base = short.split("<")[0]
    arg = short[len(base) + 1:].split(",")[0].split(">")[0] if "<" in short else ""
    return base, arg


def reduce_counters(fetch_dir, write_dir, probe_file, level):
    """Reduces two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
    `bench.py --sweep-probe LEVEL` to the HBM traffic of each move-decide kernel
    group in the probed sweep (the level's instantiations: weight kind 1 at
    level 0, 2 above), scaled by what the counters read for the probe's 1 GiB
    device copy (the dispatch that wrote 1 GiB and read the most); prints the
    JSON that profiles/decide_traffic_rmat26.md carries."""
    import csv
    import glob
    import hashlib

    def per_dispatch(d, counter):
        agg = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") == counter:
                        k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                        agg[k] = agg.get(k, 0.0) + float(r["Counter_Value"])
        return agg

    wk = "2" if level > 0 else "1"

    def groups(agg):
        acc = {}
        for (_, name), v in agg.items():
            base, arg = _kernel_base(name)
            if base in GROUP_OF and arg == wk:
                acc[GROUP_OF[base]] = acc.get(GROUP_OF[base], 0.0) + v
        return acc

    fd, wd = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    cands = [kv for kv in wd.items() if abs(kv[1] - (1 << 20)) < (1 << 14)]
    cal = max(cands, key=lambda kv: fd.get(kv[0], 0.0))
    fs, ws = (1 << 20) / fd[cal[0]], (1 << 20) / cal[1]
    fa, wa = groups(fd), groups(wd)
    probe = json.loads([l for l in open(probe_file) if l.startswith("{")][-1])
    src = os.path.join(ROOT, "paper_1304_4453_amd", "csrc", "move.hip")
    out = {"workload": probe["workload"], "level": level, "sweep": probe["sweep"], "moves": probe["moves"],
           "calibration_kernel": cal[0][1][:60], "fetch_copy_kib": fd[cal[0]], "write_copy_kib": cal[1],
           "fetch_scale": fs, "write_scale": ws,
           "move_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(), "kernels": []}
    for i, k in enumerate(probe["kernels"]):
        la = probe["kernel_launches"][min(i, 4)]
        fb, wb = fa.get(k, 0.0) * 1024 * fs, wa.get(k, 0.0) * 1024 * ws
        alg = probe["kernel_bytes"][i]
        out["kernels"].append({"kernel": k, "launches": la, "fetch_bytes": fb, "write_bytes": wb,
                               "traffic_bytes_per_launch": (fb + wb) / max(la, 1),
                               "algorithmic_bytes_per_launch": alg / max(la, 1),
                               "traffic_over_algorithmic": (fb + wb) / alg if alg else None})
    print(json.dumps(out))


def reduce_trace(trace_dir, level):
    """Per-dispatch durations of the move-decide kernels of a level in a
    rocprofv3 --kernel-trace of `bench.py --steps 1 --warmup 0 ...` (the
    instrumented step, then the timed step, each with the same dispatches):
    average duration per dispatch in each half; prints JSON."""
    import csv
    import glob
    import statistics
    wk = "2" if level > 0 else "1"
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    out = {}
    for base in GROUP_OF:
        ds = [(e - s) / 1000 for s, e, n in rows if _kernel_base(n) == (base, wk)]
        if not ds:
            continue
        h = len(ds) // 2
        out[base] = {"dispatches_per_step": h, "instrumented_avg_us": statistics.mean(ds[:h]) if h else None,
                     "timed_avg_us": statistics.mean(ds[h:])}
    print(json.dumps(out))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--reduce-counters":
        reduce_counters(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--reduce-trace":
        reduce_trace(sys.argv[2], int(sys.argv[3]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat26", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=256)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-plmr", action="store_true")
    ap.add_argument("--no-gamma", action="store_true")
    ap.add_argument("--no-plp", action="store_true")
    ap.add_argument("--no-epp", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the served workload")
    ap.add_argument("--plain-serve-sample", type=int, default=40)
    ap.add_argument("--serve-inflight", type=int, default=1, help="batches the server may run at once")
    ap.add_argument("--sweep-probe", type=int, default=None, metavar="LEVEL",
                    help="one instrumented sweep of R-MAT 26 at this level for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1304_4453_amd as P

    torch.cuda.set_device(0)
    if args.sweep_probe is not None:
        sweep_probe(P, torch, args.sweep_probe)
        return
    t = time.time()
    gr = make_graph(args.workload)
    log(f"graph {args.workload}: n={gr['n']} nnz={gr['nnz']} built in {time.time() - t:.1f}s")
    # Instrumented step: every move-decide kernel carries start/stop HIP events
    # on its dispatch (the library's stream); it gives the dominant kernel and
    # its average launch duration.  Events slow the timed kernels on this
    # stack (up to ~2x), so the timed steps below run without them and the
    # roofline from the instrumented step is a lower bound.
    mk = lambda **kw: P.Context(gr["off"], gr["col"], gr["w"], mem_kind=P.PLM_MEM_DEVICE, n=gr["n"], nnz=gr["nnz"],
                                **kw)
    ctx = mk(timing=1)
    state0 = ctx.state()  # level-0 singleton state, for the CPU sample
    lab = torch.empty(max(gr["n"], 1), dtype=torch.int32, device="cuda:0")
    t = time.time()
    ctx.run(lab)
    st_probe = ctx.stats()
    dl, dk = dominant(st_probe)
    roof = roofline(st_probe, dl, dk)
    log(f"instrumented step {time.time() - t:.2f}s: dominant {roof['kernel']}")
    ctx.close()
    ctx = mk(timing=0)
    for i in range(args.warmup):
        t = time.time()
        ctx.run(lab)
        log(f"warmup {i}: {time.time() - t:.2f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q = lv = None
    for i in range(args.steps):
        t = time.perf_counter()
        _, q, lv = ctx.run(lab)
        log(f"step {i}: {time.perf_counter() - t:.3f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.stats()  # of the last step
    ms_per_step = elapsed * 1e3 / args.steps

    L = st["levels"]
    m_l = [(st["nnz"][l] - st["loops"][l]) // 2 + st["loops"][l] for l in range(L)]
    # executed sweeps only: sweeps fast-forwarded over a period-2 cycle did not run
    run_sweeps = [st["sweeps"][l] - st["cycle_sweeps"][l] for l in range(L)]
    sweep_edges = sum(run_sweeps[l] * m_l[l] for l in range(L))
    value = sweep_edges / (ms_per_step / 1e3)
    sweep_ms = sum(st["sweep_ms"])
    roof["timing"] = ("HIP events attached to each move-decide dispatch (hipExtLaunchKernelGGL) on the library's "
                      "stream, in one instrumented step before the timed steps; the timed steps run without events")
    roof["measured_copy"] = copy_peak(torch)
    roof["per_level"] = level_summary(st_probe)
    if args.workload == "rmat26":
        tr = counter_traffic(roof["kernel"], roof["level"])
        if tr is not None:
            roof["traffic"] = tr["bytes_per_launch"]
            roof["traffic_detail"] = tr
    out = {
        "metric": "PLM move-sweep edges/s",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload]["desc"], "n": gr["n"], "nnz": gr["nnz"], "m": m_l[0],
                   "schedule": "Jones-Plassmann colour classes, <=32 sweeps per level", "parallelism": "single-gpu"},
        "roofline": roof,
        "sweep_only_edges_per_s": sweep_edges / (sweep_ms / 1e3) if sweep_ms else None,
        "full_run_edges_per_s": m_l[0] / (ms_per_step / 1e3),
        "q": q,
        "levels": lv,
        "per_level": {k: st[k] for k in ("n", "nnz", "colours", "sweeps", "cycle_sweeps", "moves", "schedule_ms",
                                         "colour_ms", "schedule_rounds", "sweep_ms", "coarsen_ms")},
        "paper_context": "PLM full run >21M edges/s (uk-2007-05, 3.3e9 edges, 2x Xeon E5-2680, 32 threads)",
    }
    if not args.no_cpu_baseline:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(gr, state0, args.cpu_budget)
        log(f"cpu baseline {time.time() - t:.1f}s")
        t = time.time()
        out["cpu_baseline"]["full_run"] = cpu_full_run(P, torch)
        log(f"oracle full run {time.time() - t:.1f}s")
    ctx.close()
    if not args.no_plmr:
        out["plmr"] = plmr_bench(gr, P, torch, q, st)
    if not args.no_plp:
        out["plp"] = plp_bench(gr, P, torch)
    if not args.no_epp:
        out["epp"] = epp_bench(gr, P, torch, q)
    if not args.no_gamma:
        out["gamma"] = gamma_bench(P, torch)
    if gr["dg"] is not None:
        gr["dg"].free()
    if not args.no_batch:
        out["batched"] = batch_bench(args, P, torch, np)
    if not args.no_serve:
        out["served"] = serve_bench(args, P, torch, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
