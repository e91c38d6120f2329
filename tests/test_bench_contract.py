"""The benchmark's host-side contract (no GPU): one GPU only, the algorithmic
byte count of the headline step, the committed traffic summary it reads and
the walk-length histogram's bins."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes_of_the_graded_step():
    # 2,002,225 feet x (16 B coordinates + 4 B start + 4 B element + 2 x 16 x 4 B
    # values) + 3,998,792 triangles x 12 B vertex ids
    assert bench.algorithmic_bytes(2_002_225, 3_998_792, 16, 4, 16) == 352_323_704
    # one field, FP32 coordinates
    assert bench.algorithmic_bytes(10, 7, 8, 4, 1) == 10 * (8 + 4 + 4 + 8) + 7 * 12
    # P2: six DOF ids per triangle and an 8-byte start/element pair per DOF
    assert bench.algorithmic_bytes(10, 7, 16, 8, 2, order=2) == 10 * (16 + 8 + 32) + 7 * 24


def test_traffic_summary_is_readable_and_plausible():
    txt = Path(bench.TRAFFIC_SUMMARY).read_text()
    assert "kernel_source_sha256_16:" in txt and "hbm_bytes_per_launch:" in txt
    t = bench.measured_traffic()
    if t is not None:  # taken on the current kernel source
        alg = bench.algorithmic_bytes(2_002_225, 3_998_792, 16, 4, 16)
        assert alg < t < 4 * alg


def test_step_histogram_bins():
    h = bench.hist_dict(list(range(16)))
    assert len(h) == 16 and h["[0,1)"] == 0 and h["[1,2)"] == 1 and h["[16384,inf)"] == 15
    assert sum(h.values()) == sum(range(16))
