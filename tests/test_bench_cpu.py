"""Host-side pieces of the benchmark that must hold without a GPU: the
kernel-source hashes that tie a traffic measurement to a kernel resolve for
every kernel that has one, and the --gpus guard."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_kernel_source_hashes_resolve():
    for (kname, _, _), meas in bench.MEASURED_TRAFFIC.items():
        h = bench.kernel_source_hash(kname)
        assert isinstance(h, str) and len(h) == 16, kname
        assert isinstance(meas["bytes"], int) and len(meas["src"]) == 16
    assert bench.kernel_source_hash("no_such_kernel") is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]
