"""Host-side behaviour of bench.py that needs no GPU: the refusal of more
than one GPU, and the CPU-oracle baseline leg on a small lattice."""

import os
import subprocess
import sys

import numpy as np

import fieldgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr and p.stdout == ""


def test_cpu_baseline_fields():
    import bench
    dims = (4, 4, 4, 8)
    U = fieldgen.gauge_haar(dims, 1)
    psi = fieldgen.spinor_gauss(int(np.prod(dims)) // 2, 2)
    r = bench.cpu_baseline(dims, U, psi, 0.16, (1.0, 0.0, 0.0, 0.0), 0.05)
    assert r["kind"] == "oracle" and r["unit"] == "GFlop/s"
    assert r["value"] > 0 and r["value_1_thread"] > 0 and r["cores"] >= 1
    assert r["min_ms_per_application"] <= r["median_ms_per_application"]
