"""Writes the oracle's full-run results (PLM, and PLMR under the "_plmr" keys)
for the named workloads to
tests/golden/oracle_runs.json: a SHA-256 of the canonical label array, Q and
the per-level trace.  Calls only the oracle and the input generators.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype=np.int32).tobytes()).hexdigest()


def main():
    out = {}
    work = {
        "planted_partition_1000_seed1": lambda: graphgen.planted_partition_1000(seed=1),
        "rmat20_seed2_unit": lambda: graphgen.rmat20(seed=2),
    }
    for name, make in work.items():
        g = make()
        for refine in (False, True):
            r = oracle.run(g.off, g.col, None if g.w is None else g.w, refine=refine)
            key = name + ("_plmr" if refine else "")
            out[key] = {"n": g.n, "nnz": g.nnz, "q": r.q, "q_hex": float(r.q).hex(), "levels": r.levels,
                        "labels_sha256": digest(r.labels), "communities": len(set(r.labels.tolist())),
                        "trace": {"n": r.n, "nnz": r.nnz, "colours": r.colours, "sweeps": r.sweeps,
                                  "communities": r.communities, "moves": [sum(m) for m in r.moves]}}
            if refine:
                out[key]["trace"]["ref_sweeps"] = r.ref_sweeps
                out[key]["trace"]["ref_moves"] = r.ref_moves
            print(key, out[key]["q"], out[key]["levels"], flush=True)
    with open(os.path.join(HERE, "oracle_runs.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
