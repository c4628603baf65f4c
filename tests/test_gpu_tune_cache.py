"""The autotuner's winner file (PBM_TUNE_CACHE, "key variant" per line).

A process that finds its keys in the file uses the stored variants without
timing; an entry that names no variant (a stale or corrupt file) is timed
again, and the new winner is appended.  Each step runs in a child process,
since the file is read once per process."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import inputs
import paper_2108_10481_amd as pbm
m = inputs.icosphere(6, 2.0)
c = inputs.charges_ball(2, 5, 1.0)
r = pbm.pb_solve(m.xyz, m.tri, c.xyz, c.q,
                 pbm.pb_default_options(precision=pbm.PB_FP32, operator_mode=pbm.PB_ASSEMBLED))
print(json.dumps({"status": r["status"], "iterations": r["iterations"], "dG": r["dG"]}), flush=True)
"""


def _child(cache):
    env = dict(os.environ, PBM_TUNE_CACHE=str(cache))
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def _entries(cache):
    rows = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    return [(k, int(v)) for k, v in rows]


def test_tune_cache_file_reuse_and_stale_entries(tmp_path):
    cache = tmp_path / "tune.txt"
    first = _child(cache)
    assert first["status"] == 0 and first["iterations"] > 0
    tuned = _entries(cache)
    assert tuned and all(k.startswith("gemv/") and 0 <= v < 6 for k, v in tuned)
    # a later process reads the winners: same variants, bitwise the same result, nothing appended
    assert _child(cache) == first
    assert _entries(cache) == tuned
    # entries naming no variant: timed again, valid winners appended, same solution
    cache.write_text("".join(f"{k} {bad}\n" for (k, _), bad in zip(tuned, [99, -1] * len(tuned))))
    again = _child(cache)
    assert again["status"] == 0 and again["iterations"] == first["iterations"]
    assert abs(again["dG"] - first["dG"]) <= 1e-6 * abs(first["dG"])
    redo = _entries(cache)[len(tuned):]
    assert sorted(k for k, _ in redo) == sorted(k for k, _ in tuned)
    assert all(0 <= v < 6 for _, v in redo)
    # the appended winners, read last, now serve a fourth process
    assert _child(cache) == again
