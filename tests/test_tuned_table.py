"""The tuned degree-bin table (tuned_bins.txt beside libplm.so, or the file
PLM_TUNED_TABLE names), read once per process: which row applies to a context
of a given kind and size, how zero thresholds are filled, and how invalid rows
or mixes with the caller's own values fall back to the compiled defaults.
Runs without a GPU (plm_resolve_options does no device work); each case runs
in a fresh process, since the table is read once."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1304_4453_amd", "libplm.so")

PROBE = r"""
import json, sys
sys.path.insert(0, %r)
import paper_1304_4453_amd as P
cases = json.loads(sys.argv[1])
out = {"table": P.plm_tuned_table().decode(), "res": []}
for batched, nnz, kw in cases:
    try:
        o = P.resolve_options(batched, nnz, **kw)
        out["res"].append([o.bin_lane, o.bin_wave, o.bin_block, o.hub_row_max])
    except P.PLMError as e:
        out["res"].append(str(e.status))
print(json.dumps(out))
""" % ROOT


def _probe(table_text, cases, tmp_path):
    env = dict(os.environ)
    if table_text is None:
        env["PLM_TUNED_TABLE"] = str(tmp_path / "missing.txt")
    else:
        p = tmp_path / "tuned.txt"
        p.write_text(table_text)
        env["PLM_TUNED_TABLE"] = str(p)
    r = subprocess.run([sys.executable, "-c", PROBE, json.dumps(cases)], capture_output=True, text=True, env=env,
                       check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.fixture(scope="module")
def built():
    assert os.path.exists(LIB), "libplm.so missing: run __graft_entry__.build()"


def test_no_table_gives_compiled_defaults(built, tmp_path):
    out = _probe(None, [[False, 1000, {}], [True, 1000, {}], [False, 1000, {"bin_wave": 64}]], tmp_path)
    assert out["table"] == ""
    assert out["res"] == [[16, 512, 4096, 12288], [16, 512, 4096, 12288], [16, 64, 4096, 12288]]


def test_rows_by_kind_and_size(built, tmp_path):
    table = ("# comment\n"
             "batch 0 8 64 1024 8192\n"
             "single 1000 4 16 256 6144\n"
             "single 0 12 128 2048 12288\n")
    cases = [[True, 5, {}], [True, 10**9, {}], [False, 1000, {}], [False, 1001, {}],
             [False, 1000, {"bin_block": 4096}], [False, 10**9, {"hub_row_max": 100}]]
    out = _probe(table, cases, tmp_path)
    assert out["table"].endswith("tuned.txt")
    assert out["res"] == [[8, 64, 1024, 8192], [8, 64, 1024, 8192], [4, 16, 256, 6144], [12, 128, 2048, 12288],
                          [4, 16, 4096, 6144], [12, 128, 2048, 100]]


def test_invalid_rows_ignored_and_bad_mix_falls_back(built, tmp_path):
    table = ("single 0 32 64 128 100\n"        # bin_lane > 16: ignored
             "single 0 8 4 128 100\n"          # lane > wave: ignored
             "batch -1 8 64 1024 8192\n"       # negative size: ignored
             "bogus 0 8 64 1024 8192\n"        # unknown kind: ignored
             "single 0 8 64 1024\n"            # short row: ignored
             "single 0 2 32 512 4096\n")
    cases = [[False, 10, {}], [True, 10, {}],
             [False, 10, {"bin_block": 64}],   # tuned (2, 32) fits below 64
             [False, 10, {"bin_block": 16}],   # tuned wave 32 > 16, compiled 512 > 16 too: PLM_E_ARG
             [False, 10, {"bin_wave": 16}],    # tuned block 512 >= 16: kept
             [False, 10, {"bin_lane": 17}]]    # out of range: PLM_E_ARG
    out = _probe(table, cases, tmp_path)
    assert out["res"][0] == [2, 32, 512, 4096]
    assert out["res"][1] == [16, 512, 4096, 12288]
    assert out["res"][2] == [2, 32, 64, 4096]
    assert out["res"][3] == "-1"
    assert out["res"][4] == [2, 16, 512, 4096]
    assert out["res"][5] == "-1"
