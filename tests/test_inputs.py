"""The workloads' synthetic inputs are pinned by fixtures: the small
workload's series as a file and every workload's series by SHA-256
(written by tests/golden/make_input_fixtures.py, which calls only the
seeded generators).  A generator that drifts changes every measured input,
so it fails here first."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
sys.path.insert(0, os.path.dirname(HERE))

import make_input_fixtures as fx  # noqa: E402
from paper_1905_00565_amd import synth  # noqa: E402


def test_coupled_logistic_first_step():
    # x1 = 0.4 (3.8 - 3.8*0.4 - 0.02*0.2), y1 = 0.2 (3.5 - 3.5*0.2 - 0.1*0.4)
    x, y = synth.coupled_logistic(2)
    assert x[0] == 0.4 and y[0] == 0.2
    assert x[1] == 0.4 * (3.8 - 3.8 * 0.4 - 0.02 * 0.2)
    assert y[1] == 0.2 * (3.5 - 3.5 * 0.2 - 0.1 * 0.4)
    assert abs(x[1] - 0.9104) < 1e-15 and abs(y[1] - 0.552) < 1e-15


def test_small_workload_file_fixture():
    raw = np.fromfile(os.path.join(HERE, "golden", "c1_coupled_logistic_N1000.bin"), dtype="<f8")
    w = synth.workload_small()
    assert raw.shape == (2000,)
    assert np.array_equal(raw[:1000], w.X) and np.array_equal(raw[1000:], w.Y)


def test_every_workload_digest():
    with open(os.path.join(HERE, "golden", "inputs_sha256.json")) as f:
        want = json.load(f)
    assert fx.digests() == want
