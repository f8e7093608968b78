"""Writes tests/golden/rmat26_oracle.json: the oracle's PLM run on R-MAT scale 26
(edge factor 16, a/b/c/d = .57/.19/.19/.05, weights uniform in [1, 100],
seed 3), level by level and sweep by sweep.  Calls only the oracle and the
input generators; every recorded value is the oracle's.

Recorded per level: n, nnz, S, SHA-256 of the level's CSR arrays, the colour
count and the SHA-256 of the colour array, and for every sweep the move count
and the SHA-256 of the community ids (int32) and community volumes (int64)
after it; then the community count.  At the end: SHA-256 of the canonical
labels, Q (and its integers N and S^2, Equation (3.1)), the level count, and
the single-threaded oracle seconds of every phase on this host.

The run follows the oracle's full run (orc_run) step for step, through the
oracle's exported steps: volumes, colouring, sweeps until one moves nothing or
32 have run, relabel, contraction while communities merged, composition of the
fine-to-coarse maps, canonical labels, modularity on the input graph.  It
needs about 55 GB of host memory at the level-0 contraction.  The decisions
of each colour class may be spread over threads (orc_sweep_mt: same result as
the oracle's plain sweep); single-threaded, one level-0 sweep takes about half
an hour.

    python tests/golden/make_rmat26_golden.py [--ckpt DIR] [--threads T]

--ckpt DIR keeps each finished level's state on disk and resumes from it.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

EF, MAX_SWEEPS = 16, 32
SCALE, SEED = 26, 3
OUT = os.path.join(HERE, "rmat26_oracle.json")
P64, P32 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)


def sha(a) -> str:
    h = hashlib.sha256()
    mv = memoryview(np.ascontiguousarray(a)).cast("B")
    step = 1 << 28
    for i in range(0, len(mv), step):
        h.update(mv[i:i + step])
    return h.hexdigest()


def p(a, t):
    return a.ctypes.data_as(t)


def say(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def host():
    cpu = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": cpu, "logical_cores": os.cpu_count()}


def generate():
    """Level-0 CSR: off int64, col int32, input weights int32 and the
    doubled-diagonal int64 weights the oracle works on."""
    g = graphgen.rmat(SCALE, EF, graphgen.RMAT_ABCD, SEED, weighted=True)
    w2 = np.empty(g.nnz, np.int64)
    w2[:] = g.w
    oracle.lib().orc_double_diagonal(g.n, p(g.off, P64), p(g.col, P32), p(w2, P64), p(w2, P64))
    return g, w2


def save(rec):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ckpt", default=None, help="directory for per-level checkpoints (resume)")
    ap.add_argument("--scale", type=int, default=26, help="smaller scales write rmat<scale>_oracle.json (trial runs)")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--threads", type=int, default=1, help="threads of the class decisions (same result)")
    args = ap.parse_args()
    global SCALE, SEED, OUT
    SCALE, SEED = args.scale, args.seed
    OUT = os.path.join(HERE, f"rmat{SCALE}_oracle.json")
    L = oracle.lib()
    rec = {"workload": f"R-MAT scale {SCALE}, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, loops and "
                       f"duplicates removed, integer weights uniform in [1,100], seed {SEED}",
           "options": {"max_sweeps": MAX_SWEEPS, "max_levels": 0, "schedule": 0, "colour_seed": 0, "gamma": [1, 1]},
           "host": dict(host(), decision_threads=args.threads), "complete": False, "levels": []}
    t0 = time.time()
    say("generate")
    g, w2 = generate()
    n0 = g.n
    rec["graph"] = {"n": g.n, "nnz": g.nnz, "off_sha256": sha(g.off), "col_sha256": sha(g.col),
                    "w_sha256": sha(g.w), "generate_seconds": time.time() - t0}
    say("graph", rec["graph"])
    off, col, lw = g.off, g.col, w2
    del g, w2                       # only off/col/lw hold the level-0 graph now
    lab = np.arange(n0, dtype=np.int32)   # input node -> current-level node
    level = 0
    ck = args.ckpt
    if ck:
        os.makedirs(ck, exist_ok=True)
    while True:
        ln, lnnz = off.shape[0] - 1, col.shape[0]
        ckf = os.path.join(ck, f"level{level}.npz") if ck else None
        ckj = os.path.join(ck, f"level{level}.json") if ck else None
        if ckf and os.path.exists(ckf) and os.path.exists(ckj):
            lv = json.load(open(ckj))
            z = np.load(ckf)
            zeta = z["zeta"]
            say(f"level {level}: resumed from checkpoint")
        else:
            vol = np.empty(max(ln, 1), np.int64)
            t = time.time()
            S = int(L.orc_volumes(ln, p(off, P64), p(lw, P64), p(vol, P64)))
            cks = os.path.join(ck, f"level{level}_sweeps.npz") if ck else None
            if cks and os.path.exists(cks) and os.path.exists(cks + ".json"):
                # resume inside the level: colouring and the state after the last finished sweep
                lv = json.load(open(cks + ".json"))
                z = np.load(cks)
                colour, zeta, volC = z["colour"], z["zeta"], z["volC"]
                ncol = lv["colours"]
                say(f"level {level}: resumed after sweep {len(lv['sweeps'])}")
            else:
                lv = {"level": level, "n": ln, "nnz": lnnz}
                if level > 0:
                    lv.update(off_sha256=sha(off), col_sha256=sha(col), w_sha256=sha(lw))
                lv["S"] = S
                lv["vol_sha256"] = sha(vol[:ln])
                colour = np.empty(max(ln, 1), np.int32)
                ncol = int(L.orc_colour(ln, p(off, P64), p(col, P32), 0, level, 0, p(colour, P32)))
                lv["colour_seconds"] = time.time() - t
                lv["colours"] = ncol
                lv["colour_sha256"] = sha(colour[:ln])
                lv["class_sizes_sha256"] = sha(np.bincount(colour[:ln], minlength=ncol).astype(np.int64))
                say(f"level {level}: n={ln} nnz={lnnz} S={S} colours={ncol} ({lv['colour_seconds']:.0f} s)")
                zeta = np.arange(max(ln, 1), dtype=np.int32)
                volC = vol.copy()
                lv["sweeps"] = []
            for s in range(len(lv["sweeps"]), MAX_SWEEPS):
                if lv["sweeps"] and lv["sweeps"][-1]["moves"] == 0:
                    break
                t = time.time()
                mv = int(L.orc_sweep_mt(ln, p(off, P64), p(col, P32), p(lw, P64), p(vol, P64), S, 1, 1,
                                        p(colour, P32), ncol, p(zeta, P32), p(volC, P64), args.threads))
                dt = time.time() - t
                lv["sweeps"].append({"moves": mv, "zeta_sha256": sha(zeta[:ln]), "volc_sha256": sha(volC[:ln]),
                                     "seconds": dt})
                say(f"level {level} sweep {s + 1}: moves={mv} ({dt:.0f} s)")
                rec["levels_partial"] = rec["levels"] + [lv]
                save(rec)
                if cks and ln > (1 << 20):
                    np.savez(cks + ".tmp.npz", colour=colour, zeta=zeta, volC=volC)
                    os.replace(cks + ".tmp.npz", cks)
                    json.dump(lv, open(cks + ".json", "w"))
                if mv == 0:
                    break
            del vol, volC, colour
            zeta = zeta[:ln]
            if ckf:
                np.savez(ckf, zeta=zeta)
                json.dump(lv, open(ckj, "w"))
        pi = np.empty(max(ln, 1), np.int32)
        k = int(L.orc_relabel(ln, p(zeta, P32), p(pi, P32)))
        lv["communities"] = k
        rec["levels"].append(lv)
        rec.pop("levels_partial", None)
        save(rec)
        level += 1
        if k == ln:
            lab = zeta[lab]
            break
        del zeta
        t = time.time()
        coff = np.empty(k + 1, np.int64)
        ccol = np.empty(max(lnnz, 1), np.int32)     # untouched pages past the coarse size stay unmapped
        cw = np.empty(max(lnnz, 1), np.int64)
        cnnz = int(L.orc_contract(ln, p(off, P64), p(col, P32), p(lw, P64), p(pi, P32), k, p(coff, P64),
                                  p(ccol, P32), p(cw, P64)))
        lv["contract_seconds"] = time.time() - t
        save(rec)
        say(f"contracted to n={k} nnz={cnnz} ({lv['contract_seconds']:.0f} s)")
        lab = pi[lab]
        del pi
        off, col, lw = coff, ccol[:cnnz], cw[:cnnz]
        if cnnz < lnnz // 2:            # hand back the unused tail of the capacity
            col, lw = col.copy(), lw.copy()
        del ccol, cw
    labels = np.empty(n0, np.int32)
    L.orc_canonical(n0, p(lab, P32), p(labels, P32))
    del lab, off, col, lw
    rec["levels_count"] = level
    rec["labels_sha256"] = sha(labels)
    rec["communities"] = int(labels.max()) + 1 if n0 else 0
    save(rec)
    say("modularity on the input graph (regenerated)")
    g, w2 = generate()
    g.w = None
    N, D, q = oracle.modularity_parts(g.off, g.col, w2, labels)
    rec.update(q=q, q_hex=float(q).hex(), N=str(N), D=str(D), complete=True, total_seconds=time.time() - t0)
    save(rec)
    say("done", q, level)


if __name__ == "__main__":
    main()
