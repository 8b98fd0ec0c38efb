"""Host-side helpers of bench.py that read committed measurement summaries."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_lds_atomic_ceiling_is_read_from_the_probe_summary():
    peak = bench.measured_lds_atomic_peak()
    assert peak is not None
    # conflict-free 64-bit atomic adds: below the nominal LDS bandwidth, above
    # what random addresses reach (about 5 lanes per clock per CU)
    assert 5 * 8 * 256 * 2.4 < peak < bench.PEAK_LDS_GBS


def test_traffic_summary_parses_for_the_spreading_kernel():
    t = bench.measured_traffic("k_nu_spread", "clutter_50k")
    # None only when the kernel's sources changed since the counters were taken
    assert t is None or t > 0
    assert bench.measured_traffic("k_nu_spread", "icosphere_20k") is None
