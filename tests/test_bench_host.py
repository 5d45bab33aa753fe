"""Host-side logic of bench.py that its figures rest on (no device): the launch period its timed
windows align to, the algorithmic bytes of the roofline, the traffic lookup keyed by the kernel
source, and the names the profile summaries use."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1912_02018_amd.config import config2, sweep_configs  # noqa: E402


def test_launch_period_is_the_lcm_of_the_buffer_period_and_the_sampling_periods():
    c2 = config2()
    assert bench.launch_period([c2]) == 20                  # diag_every 20 (even)
    assert bench.launch_period([c2.replace(diag_every=7)]) == 14
    assert bench.launch_period([c2.replace(diag_every=0)]) == 2
    assert bench.launch_period([c2.replace(diag_every=6), c2.replace(diag_every=10)]) == 30
    assert bench.launch_period(sweep_configs(64, 2018)) == 100


def test_algorithmic_bytes_per_node():
    # stream-and-collide: 9 populations read and written in the storage type, T read in the compute
    # type; temperature: T read and written
    assert bench.kernel_bytes_per_lup(0, 1) == 76 and bench.kernel_bytes_per_lup(1, 1) == 8
    assert bench.kernel_bytes_per_lup(0, 0) == 152 and bench.kernel_bytes_per_lup(1, 0) == 16
    assert bench.kernel_bytes_per_lup(0, 2) == 40 and bench.kernel_bytes_per_lup(0, 3) == 40


def test_measured_traffic_only_for_the_profiled_source():
    """profiles/traffic.json is read only when its source digest is that of the kernels built here,
    so a stale profile never feeds the roofline."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    tj = json.load(open(path))
    key, rec = next(iter(sorted(tj.items())))
    variant, workload = key.split("@")
    got = bench.measured_traffic(variant, workload)
    if rec["source_sha"] == bench.source_digest():
        assert got == rec["bytes_per_launch"]
    else:
        assert got is None
    assert bench.measured_traffic("k_lbm<no such variant>", workload) is None


def test_profile_names_of_launch_variants():
    assert bench.variant_name(0, (32, 8, 256, 6), 4) == "k_lbm<32x8x256,w6>"
    assert bench.variant_name(0, (64, 16, 512, 0), 4) == "k_lbm<64x16x512>"
    assert bench.variant_name(1, (240, 0, 256, 2), 4) == "k_thermal<240x0x256,w2,rk4>"
    assert bench.variant_name(1, (64, 32, 1024, 0), 2) == "k_thermal<64x32x1024,rk2>"
