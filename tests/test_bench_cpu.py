"""Host-side checks of the benchmark: its refusal of more than one GPU, the
algorithmic work it prices the roofline with, and that the committed HBM
traffic record was taken on the current kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2110_01614_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "only --gpus 1" in r.stderr and r.stdout == ""


def test_algorithmic_work_per_point_in_closed_form():
    """4 sum_l K_l width_l: every multiply-add of every affine map, once per
    sweep.  3->256x8->1 with x re-fed at layer 5: 768 + 6 * 65536 + 256 * 259
    + 256 multiply-adds per sweep; the same at width 512."""
    assert bench.flops_per_point(I.NetSpec((256,) * 8, 5)) == 4 * (768 + 6 * 65536 + 256 * 259 + 256) == 1842176
    assert bench.flops_per_point(I.NetSpec((512,) * 8, 5)) == 4 * (1536 + 6 * 262144 + 512 * 515 + 512) == 7354368
    # the sphere workload: 3->64x3->1, no skip
    assert bench.flops_per_point(I.NetSpec((64,) * 3)) == 4 * (192 + 2 * 4096 + 64)


def test_traffic_record_matches_the_current_kernel_sources():
    """The FETCH/WRITE record behind roofline.traffic names the hash of the
    device sources it was measured on; bench.py reports null otherwise, so
    a stale record would silently drop the figure."""
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["source_hash"] == bench.kernel_source_hash()
    assert rec["kernel"] == bench.K16_NAME % bench.PREC_ID[rec["precision"]]
    # algorithmic bytes of a launch (12 B in, 28 B out per vertex) are a lower bound
    assert rec["bytes_per_launch"] >= 40e6
