"""The device calibration entry point returns the seven access rates, each in
a plausible range for a device with HBM (diagnostic only)."""
import pytest

import paper_2606_09318_amd as lr

pytestmark = pytest.mark.gpu


def test_calibrate_rates():
    r = lr.calibrate()
    assert len(r) == 7
    assert r["copy_gb_s"] > 500                       # streaming: far above random access
    assert 1 < r["gather4_1gib_g_s"] < 1000
    assert all(v > 0.5 for v in r.values())
    # a random 4 B gather moves a whole line: far fewer gathers per second than
    # the copy moves 4 B words
    assert r["gather4_1gib_g_s"] * 4 < r["copy_gb_s"]
