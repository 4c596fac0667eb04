"""The oracle against its pins (see ``oracle_pins.py`` for what each rests on)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_threaded_equals_serial(orc):
    from paper_1905_00565_amd import synth
    import numpy as np
    w = synth.workload_small()
    a = orc.ccm(w.X[:300], w.Y[:300], 2, 1, [50, 299], 3, 5)
    b = orc.ccm_threaded(w.X[:300], w.Y[:300], 2, 1, [50, 299], 3, 5, threads=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
