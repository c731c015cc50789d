"""Host-side checks of bench.py: the one-GPU guard, and the committed HBM
counter summary it reads the measured traffic from."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_is_well_formed():
    path = os.path.join(ROOT, "profiles", "tile11_kernel_d20_l4_x256_hbm_traffic.txt")
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert kv["workload"].startswith("256x(d=20,l=4)")
    assert len(kv["source_sha256"]) == 64
    fetch = float(kv["fetch_bytes_per_launch"])
    write = float(kv["write_bytes_per_launch"])
    alg = 1 << 30   # each FP32 coalition value read once
    # the kernel reads its input once: FETCH within a few percent of the
    # algorithmic bytes, WRITE (FP64 partial sums) a small fraction of them
    assert alg <= fetch <= 1.05 * alg
    assert 0 < write <= 0.1 * alg
