"""The committed rocprofv3 summaries and the roofline calibration in bench.py
describe the same kernel sources: every counter summary names the digest the
calibration was taken on, and bench.py reports no roofline fraction for any
other sources (no GPU needed)."""
import glob
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_summaries_name_the_calibrated_digest():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "phase_*_kernel_*.md")))
    assert len(files) >= 6
    for f in files:
        m = re.search(r"digest `([0-9a-f]{16})`", open(f).read())
        assert m and m.group(1) == bench.PROFILED_KERNEL_DIGEST, f


def test_roofline_fraction_only_for_the_profiled_sources():
    d = bench._roofline("sphere", False, 200.0, 131072.0, 3.7e-4, "phase_sphere_kernel")
    assert d["frac"] is None and d["achieved"] is None and d["traffic"] is None
    d = bench._roofline("sphere", True, 212.05 * 131072, 131072.0, 3.7e-4, "phase_sphere_kernel")
    p = bench.PROFILE["sphere"]
    want = (p["a_dep"] * 212.05 * 131072 + p["b_move"] * 131072) / 3.7e-4 / bench.VALU_PEAK_LANE_OPS
    assert abs(d["frac"] - want) < 1e-12 and 0.0 < d["frac"] < 1.0
