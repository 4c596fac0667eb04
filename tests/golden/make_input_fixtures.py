"""Write the input fixtures of the workloads (run from the repository root):

    python tests/golden/make_input_fixtures.py

* ``c1_coupled_logistic_N1000.bin``: the small workload's series, x then y,
  1000 little-endian float64 values each;
* ``inputs_sha256.json``: SHA-256 of the float64 bytes of every workload's
  series (small, sweep, long noisy series, causal-matrix network, the first
  jobs of the served job stream), so that a change of a generator shows up
  as a test failure rather than as a silent change of every measured input.

Only the seeded generators of ``paper_1905_00565_amd.synth`` are called (no
method arithmetic).
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from paper_1905_00565_amd import synth  # noqa: E402

N_JOBS = 8


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def digests() -> dict:
    out = {}
    w = synth.workload_small()
    out["small.x"], out["small.y"] = sha(w.X), sha(w.Y)
    w = synth.workload_sweep()
    out["sweep.x"], out["sweep.y"] = sha(w.X), sha(w.Y)
    w = synth.workload_long()
    out["long.x"], out["long.y"] = sha(w.X), sha(w.Y)
    m = synth.workload_matrix()
    out["matrix.S"] = sha(m["S"])
    for k, j in enumerate(synth.job_stream(N_JOBS, 1.0, seed=4)):
        x, y = j["make"]()
        out[f"job{k}"] = {"N": int(len(x)), "E": j["E"], "tau": j["tau"], "L": list(j["L"]),
                          "r": j["r"], "x": sha(x), "y": sha(y)}
    return out


def main():
    w = synth.workload_small()
    np.concatenate([w.X, w.Y]).astype("<f8").tofile(os.path.join(HERE, "c1_coupled_logistic_N1000.bin"))
    with open(os.path.join(HERE, "inputs_sha256.json"), "w") as f:
        json.dump(digests(), f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
