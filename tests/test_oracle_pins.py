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


def test_realization_split_equals_serial(orc):
    """The query-split helper gives the serial realization's rho exactly."""
    from paper_1905_00565_amd import synth
    x, y = synth.coupled_logistic(3000)
    for E, tau, L, ri, excl in ((2, 1, 500, 3, 0), (5, 2, 2990, 0, 0), (3, 3, 800, 1, 4),
                                (1, 1, 120, 7, -1)):
        want = orc.realization(y, x, E, tau, L, ri, 9, excl=excl)[0]
        got = orc.realization_split(y, x, E, tau, L, ri, 9, excl=excl, threads=3, chunk=257)
        assert got == want, (E, tau, L, ri, excl)
