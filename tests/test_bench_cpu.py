"""Host-side pieces of bench.py: the counted-traffic record is reported only for
the kernel source, precision and launch shape it was taken on."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import pytest  # noqa: E402

import bench  # noqa: E402
from paper_1310_4218_amd.autotune import tuned_params  # noqa: E402


def test_traffic_record_matches_current_kernel_and_launch():
    for w in ("moving", "precision", "large"):
        path = os.path.join(ROOT, "profiles", f"traffic_{w}.json")
        with open(path) as f:
            rec = json.load(f)
        launch = tuned_params(w, "fp32")
        if rec["kernel_source_hash"] != bench.kernel_source_hash():
            pytest.skip(f"traffic_{w}.json was taken on an earlier kernel source (bench reports null)")
        assert rec["launch"] == launch, w
        got = bench.measured_traffic(w, "fp32", launch)
        assert got == rec["hbm_bytes_per_launch"]
        # the algorithmic bytes are a lower bound of what the counters see
        wl_bytes = {"moving": 8 * 256 * 256 * 64, "precision": 8 * 1024 * 1024 * 64,
                    "large": 8 * 2048 * 2048 * 80}[w]
        assert got > wl_bytes


def test_traffic_record_not_reported_for_other_precision_or_launch():
    launch = tuned_params("moving", "fp32")
    assert bench.measured_traffic("moving", "fp64", launch) is None
    other = dict(launch, tile_y=launch.get("tile_y", 8) * 2)
    assert bench.measured_traffic("moving", "fp32", other) is None
    assert bench.measured_traffic("no-such-workload", "fp32", launch) is None


def test_kahan_takes_the_fp32_launch_shape():
    for w in ("moving", "precision", "large"):
        assert tuned_params(w, "fp32_kahan") == tuned_params(w, "fp32")
    assert tuned_params("no-such-workload", "fp32_kahan") == {}


def test_vertical_physics_takes_its_own_launch_where_tuned():
    """The 2048x2048x80 grid's vertical physics runs its two-step launch with 5 levels
    per thread (16 lanes per column); the pointwise launch keeps 4.  Workloads without a
    vertical entry take their pointwise one."""
    from paper_1310_4218_amd import _abi
    from paper_1310_4218_amd import workloads as W
    vert = tuned_params("large", "fp32", physics="vertical")
    assert vert.get("lane_levels") == 5 and "lane_levels" not in tuned_params("large", "fp32")
    assert {k: v for k, v in vert.items() if k != "lane_levels"} == tuned_params("large", "fp32")
    assert tuned_params("large", "fp32_kahan", physics="vertical") == vert
    _abi.query(_abi.config_from_workload(W.get("large").replace(vertical=1), **vert)[0])
    assert tuned_params("precision", "fp32", physics="vertical") == tuned_params("precision", "fp32")


def test_valu_count_reported_only_for_its_kernel_and_launch():
    """The vector-instruction count behind roofline.issue comes from the committed counter
    record of the 2048x2048x80 two-step launch, and only for the kernel source, precision
    and launch shape it was taken on."""
    launch = tuned_params("large", "fp32")
    path = os.path.join(ROOT, "profiles", "counters_large.json")
    with open(path) as f:
        rec = json.load(f)
    if rec["kernel_source_hash"] != bench.kernel_source_hash():
        pytest.skip("counters_large.json was taken on an earlier kernel source (bench reports null)")
    got = bench.measured_valu("large", "fp32", launch)
    assert got == rec["means_per_dispatch"]["SQ_INSTS_VALU"] and got > 1e8
    assert bench.measured_valu("large", "fp64", launch) is None
    assert bench.measured_valu("large", "fp32", dict(launch, tile_y=12)) is None
    # issue slots of one launch: 1024 SIMDs, 4 cycles per wave instruction, 2.4 GHz
    assert bench.SIMDS * bench.CLOCK_HZ / bench.CYCLES_PER_WAVE_INSTRUCTION == 614.4e9
