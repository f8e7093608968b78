"""Autotuner of the degree-bin thresholds of the move sweep.

The decide kernels split a colour class's nodes by row length into bins
(one lane per node up to bin_lane entries, a wavefront up to bin_wave, a
workgroup up to bin_block, one 1024-thread workgroup up to hub_row_max, several
workgroups per node above).  Any setting gives the same partition; the best one
depends on the degree mix of the workload and on the device.  This tuner times
candidate settings on the GPU and writes the fastest for each workload class
into ``tuned_bins.txt`` beside ``libplm.so``, which ``plm_create`` and
``plm_batch_create`` read for every threshold left at 0 (the default):

* ``batch``: ``plm_batch_run`` on graphs of the batched workload's recipe (SBM,
  n log-uniform in [100, 1e5], k = max(2, n/100) blocks, p_in = 20/blocksize,
  p_out = 1/n, seed 4);
* ``single``, up to 2^27 entries: ``plm_run`` on R-MAT scale 20 (unit weights,
  seed 2);
* ``single`` above: ``plm_run`` on R-MAT scale 26 (weights 1..100, seed 3), built
  on the GPU.

Search: coordinate descent over (bin_block, bin_wave, bin_lane, hub_row_max)
from the compiled defaults, each candidate timed as the median of ``--reps``
runs after a warm-up; a candidate must beat the incumbent by ``--margin`` to
replace it.  Every candidate's labels are compared with those of the compiled
defaults and must be identical.

    python -m paper_1304_4453_amd.tune [--out FILE] [--classes batch,small,large]
"""
from __future__ import annotations

import argparse
import os
import platform
import statistics
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT = {"bin_lane": 16, "bin_wave": 512, "bin_block": 4096, "hub_row_max": 12288}
CANDIDATES = {
    "bin_block": [1024, 2048, 4096],
    "bin_wave": [64, 128, 256, 512],
    "bin_lane": [4, 8, 12, 16],
    "hub_row_max": [6144, 8192, 12288],
}
SMALL_MAX_NNZ = 1 << 27


def valid(s: dict) -> bool:
    return 1 <= s["bin_lane"] <= s["bin_wave"] <= s["bin_block"] and s["bin_lane"] <= 16 and \
        s["bin_wave"] <= 512 and s["bin_block"] <= 4096 and 1 <= s["hub_row_max"] <= 12288


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


class Workload:
    """A timed run of one workload class with given bin settings; returns
    (seconds, labels as numpy)."""

    def __init__(self, kind: str, P, torch, batch_graphs: int):
        import graphgen
        self.kind, self.P, self.torch = kind, P, torch
        self.dg = None
        if kind == "batch":
            graphs = graphgen.sbm_batch(4, batch_graphs)
            self.nb, self.off, self.col, self.w = P.pack_batch(graphs)
            self.desc = f"{batch_graphs} SBM graphs of the batched workload's recipe (seed 4)"
            self.n = int(self.nb[-1])
        elif kind == "small":
            g = graphgen.rmat20(seed=2)
            self.off, self.col, self.w, self.n = g.off, g.col, g.w, g.n
            self.desc = "R-MAT scale 20, unit weights, seed 2"
        else:
            self.dg = graphgen.rmat_gpu(26, 16, seed=3, weighted=True)
            self.n = self.dg.n
            self.desc = "R-MAT scale 26, weights 1..100, seed 3"
        self.lab = torch.empty(max(self.n, 1), dtype=torch.int32, device="cuda:0")

    def ctx(self, s: dict):
        P = self.P
        if self.kind == "batch":
            return P.BatchContext(self.nb, self.off, self.col, self.w, **s)
        if self.kind == "small":
            return P.Context(self.off, self.col, self.w, **s)
        return P.Context(self.dg.off_ptr, self.dg.col_ptr, self.dg.w_ptr, mem_kind=P.PLM_MEM_DEVICE, n=self.dg.n,
                         nnz=self.dg.nnz, validate=0, **s)

    def time(self, s: dict, reps: int):
        torch = self.torch
        c = self.ctx(s)
        try:
            run = (lambda: c.run_batch(self.lab)) if self.kind == "batch" else (lambda: c.run(self.lab))
            run()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                run()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
        finally:
            c.close()
        return statistics.median(ts), self.lab.cpu().numpy()

    def close(self):
        if self.dg is not None:
            self.dg.free()


def tune(w: Workload, reps: int, passes: int, margin: float):
    best = dict(DEFAULT)
    t_def, ref = w.time(best, reps)
    t_best = t_def
    log(f"{w.kind}: defaults {best} {t_def * 1e3:.1f} ms")
    tried = {tuple(sorted(best.items())): t_def}
    for p in range(passes):
        changed = False
        for key, vals in CANDIDATES.items():
            for v in vals:
                s = dict(best, **{key: v})
                k = tuple(sorted(s.items()))
                if not valid(s) or k in tried:
                    continue
                t, lab = w.time(s, reps)
                tried[k] = t
                if not np.array_equal(lab, ref):
                    raise RuntimeError(f"{w.kind}: labels with {s} differ from the defaults' labels")
                log(f"{w.kind}: {s} {t * 1e3:.1f} ms")
                if t < t_best * (1 - margin):
                    best, t_best, changed = s, t, True
        if not changed:
            break
    return best, t_best, t_def, len(tried)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuned_bins.txt"))
    ap.add_argument("--classes", default="batch,small,large")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--margin", type=float, default=0.01)
    ap.add_argument("--batch-graphs", type=int, default=1024)
    a = ap.parse_args(argv)
    import torch
    import paper_1304_4453_amd as P
    assert torch.cuda.is_available(), "the tuner times kernels on the GPU"
    dev = torch.cuda.get_device_name(0)
    rows, notes = [], []
    for kind in a.classes.split(","):
        w = Workload(kind, P, torch, a.batch_graphs)
        try:
            reps = a.reps if kind != "large" else max(1, a.reps - 1)
            passes = a.passes if kind != "large" else 1
            best, t_best, t_def, n = tune(w, reps, passes, a.margin)
        finally:
            w.close()
        row_kind = "batch" if kind == "batch" else "single"
        max_nnz = SMALL_MAX_NNZ if kind == "small" else 0
        rows.append((kind, f"{row_kind} {max_nnz} {best['bin_lane']} {best['bin_wave']} {best['bin_block']} "
                           f"{best['hub_row_max']}"))
        notes.append(f"# {kind}: {w.desc}: tuned {t_best * 1e3:.1f} ms, compiled defaults {t_def * 1e3:.1f} ms "
                     f"({n} settings timed)")
        log(notes[-1][2:])
    order = {"batch": 0, "small": 1, "large": 2}
    rows.sort(key=lambda r: order[r[0]])
    with open(a.out + ".tmp", "w") as f:
        f.write(f"# degree-bin thresholds written by paper_1304_4453_amd/tune.py on "
                f"{time.strftime('%Y-%m-%d')} ({dev}, {platform.node() or 'host'})\n")
        f.write("# kind max_nnz bin_lane bin_wave bin_block hub_row_max (max_nnz 0 = any size)\n")
        for n_ in notes:
            f.write(n_ + "\n")
        for _, r in rows:
            f.write(r + "\n")
    os.replace(a.out + ".tmp", a.out)
    log(f"wrote {a.out}")


if __name__ == "__main__":
    main()
