"""bench.py's host logic, without a GPU: the link-update count of each sweep
order, and the refusal of more than one GPU before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_grouped_count_is_two_updates_per_link_and_sweep():
    V = 20 ** 4
    assert bench.link_updates("grouped", V, 128, 2500, 0.3) == 2 * 4 * V * 128 * 2500
    # independent of the acceptance
    assert bench.link_updates("grouped", V, 128, 1, 0.0) == bench.link_updates("grouped", V, 128, 1, 1.0)


@pytest.mark.parametrize("acc", [0.0, 0.25, 0.68, 1.0])
def test_interleaved_count_leaves_out_the_relabelled_overrelaxation(acc):
    V = 8 ** 4
    per_sweep = 8 * (V // 2)           # class links of one chain over the 8 fused passes
    got = bench.link_updates("interleaved", V, 3, 10, acc)
    assert got == pytest.approx((acc * 1 + (1 - acc) * 2) * per_sweep * 3 * 10)
    # all classes rejected: as many updates as the grouped order; all accepted: half
    assert bench.link_updates("interleaved", V, 1, 1, 0.0) == bench.link_updates("grouped", V, 1, 1, 0.0)
    assert bench.link_updates("interleaved", V, 1, 1, 1.0) == 0.5 * bench.link_updates("grouped", V, 1, 1, 0.0)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_staggered_order_counts_as_grouped():
    import bench
    V, n, sw = 20 ** 4, 128, 10
    assert bench.link_updates("staggered", V, n, sw, 0.3) == bench.link_updates("grouped", V, n, sw, 0.9)
    assert bench.link_updates("staggered", V, n, sw, 0.3) == 2 * 4 * V * n * sw
