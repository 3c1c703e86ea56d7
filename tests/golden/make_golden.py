"""Writes tests/golden/*.json from the oracle only (never from the HIP path).

    python tests/golden/make_golden.py

square4x4_U4_b2_3sweeps.json: the 4x4 square, U=4, beta=2, dtau=0.1,
n_wrap=10, seed 0 chain after three oracle sweeps (field, G(0), bin sums,
acceptance).  It guards the oracle against unintended changes; its physics is
pinned separately by the closed-form and Fock-space tests.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import square_lattice  # noqa: E402
from oracle import hubbard, sweep  # noqa: E402


def main():
    lat = square_lattice(4, 4)
    m = hubbard.hubbard_model(lat.K, 4.0, 2.0, 0.1, 10, trotter="sym", seed=0)
    ch = sweep.Chain(m, hubbard.init_field(m)).init()
    for _ in range(3):
        ch.sweep()
    out = {
        "workload": "square 4x4, U=4, beta=2, dtau=0.1, n_wrap=10, seed 0, symmetric split, 3 sweeps",
        "field": ch.field.astype(int).tolist(),
        "G0": ch.G.tolist(),
        "bins": ch.bins.tolist(),
        "proposals": ch.proposals,
        "accepted": ch.accepted,
    }
    with open(os.path.join(HERE, "square4x4_U4_b2_3sweeps.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
