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
bp = fsi.BatchPlan([14, 13, 12], [3, 2, 4], dtype="f32", autotune=True)
print("SCHED " + json.dumps(bp.schedule()), flush=True)
bp.close()
"""


def _child(path):
    env = dict(os.environ, FSI_TUNE_CACHE=path)
    out = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env,
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
