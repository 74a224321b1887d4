"""The roofline probes return throughputs of the right order for the device
(256 CUs x 64 lanes x 2.4 GHz = 39.3e12 INT32 lane-ops/s and 128 B per clock
per CU = 78.6e12 LDS bytes/s from the unit counts; a probe's own loop reaches
a fraction of that, never ten times it)."""
import pytest

from paper_1601_00636_amd import binding as cb

pytestmark = pytest.mark.gpu


def test_peak_probes_are_plausible():
    h = cb.cuboid_create(0)
    try:
        pk = cb.cuboid_probe_peaks(h)
    finally:
        assert cb.cuboid_destroy(h) == cb.OK
    assert 0.1 * 39.3e12 < pk["valu_lane_ops_per_s"] < 10 * 39.3e12
    assert 0.05 * 78.6e12 < pk["lds_bytes_per_s"] < 10 * 78.6e12
