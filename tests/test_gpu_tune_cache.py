"""The autotuner's schedule cache persists across processes (JSON file named
by FSI_TUNE_CACHE): a first process times the candidates and writes its
choice, a second one takes the same schedule from the file without timing."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
from paper_2601_01903_amd import fsi
bp = fsi.BatchPlan({ds!r}, {ls!r}, dtype={dtype!r}, autotune=True)
print("SCHED " + json.dumps(bp.schedule()), flush=True)
bp.close()
"""

# register-phase orders; and orders above 4 only, where the autotuner also
# chooses between the two algorithms
LOW = ([14, 13, 12], [3, 2, 4], "f32")
HIGH = ([12, 11], [6, 8], "f64")


def _child(path, spec=LOW):
    env = dict(os.environ, FSI_TUNE_CACHE=path)
    ds, ls, dtype = spec
    code = CHILD.format(root=ROOT, ds=ds, ls=ls, dtype=dtype)
    out = subprocess.run([sys.executable, "-c", code], env=env,
                         capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stdout + out.stderr
    line = [x for x in out.stdout.splitlines() if x.startswith("SCHED ")][-1]
    return json.loads(line[6:])


def test_tune_cache_persists_across_processes(tmp_path):
    path = str(tmp_path / "tune.json")
    first = _child(path)
    assert first["autotuned"] == 1 and first["tuned_ms"] > 0
    with open(path) as f:
        doc = json.load(f)
    assert doc["format"] == "fsi-autotune-1"
    keys = [e["key"] for e in doc["entries"]]
    assert any(k.startswith("gfx950-") and "14,3x1" in k for k in keys), keys
    second = _child(path)
    assert second["autotuned"] == 1 and second["tuned_ms"] == 0.0
    for k in ("fast_instances", "tiles_per_item", "tile_shift", "mob_group"):
        assert second[k] == first[k], k


def test_tune_cache_disabled_by_empty_path(tmp_path):
    first = _child("")
    second = _child("")
    assert first["tuned_ms"] > 0 and second["tuned_ms"] > 0


def test_tune_cache_algorithm_choice_and_older_entries(tmp_path):
    """The schedule of a plan whose orders are all above 4 records the
    algorithm the autotuner chose (mob_group > 0: two-pass), and a second
    process builds the same; entries written without the algorithm field
    still read (as the option's algorithm)."""
    import re
    path = str(tmp_path / "tune.json")
    first = _child(path, HIGH)
    assert first["autotuned"] == 1 and first["tuned_ms"] > 0
    text = open(path).read()
    assert re.search(r'"algo": [12]\}', text), text
    second = _child(path, HIGH)
    assert second["autotuned"] == 1 and second["tuned_ms"] == 0.0
    assert second["mob_group"] == first["mob_group"]
    low = _child(path, LOW)
    with open(path) as f:
        text = f.read()
    with open(path, "w") as f:
        f.write(re.sub(r', "algo": -?[0-9]+', "", text))
    again = _child(path, LOW)
    assert again["autotuned"] == 1 and again["tuned_ms"] == 0.0
    for k in ("fast_instances", "tiles_per_item", "tile_shift", "mob_group"):
        assert again[k] == low[k], k
