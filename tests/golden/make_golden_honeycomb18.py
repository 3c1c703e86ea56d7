"""Writes tests/golden/honeycomb18_U5_b20_sweep1.npz from the oracle only
(never from the HIP path).

    python tests/golden/make_golden_honeycomb18.py

The honeycomb 18x18 chain (N = 648, U = 5, beta = 20, dtau = 0.1, L = 200,
n_wrap = 10, two-valued field, seed 0, asymmetric split) after one oracle
sweep with the equal-time estimators on every slice, from its seeded initial
field.  Stored: the field after the sweep (signs, bit-packed), the diagonal of
G(0) and 24 of its rows (a fixed sample of indices; the full matrix is 3.4 MB),
the bin sums, the proposal and acceptance counts, the largest stabilisation
deviation and the smallest |R - u| over all proposals (near-tie guard).
The full oracle sweep takes several minutes on the host cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import WORKLOADS  # noqa: E402
from oracle import hubbard, sweep  # noqa: E402

OUT = os.path.join(HERE, "honeycomb18_U5_b20_sweep1.npz")
N_ROWS = 24


def sample_rows(n: int) -> np.ndarray:
    """The fixed row sample: first, last, and rows spread over the matrix."""
    rows = np.unique(np.concatenate([[0, 1, 31, 32, n - 1], np.random.default_rng(648).choice(n, N_ROWS - 5,
                                                                                              replace=False)]))
    return rows[:N_ROWS]


def main():
    w = WORKLOADS["honeycomb18_U5_b20"]
    lat = w.lattice()
    m = hubbard.hubbard_model(lat.K, w.U, w.beta, w.dtau, w.n_wrap, trotter=w.trotter, seed=w.seed)
    f0 = hubbard.init_field(m)
    ch = sweep.Chain(m, f0).init()
    t0 = time.time()
    ch.sweep(measure=True)
    dt = time.time() - t0
    rows = sample_rows(m.N)
    np.savez_compressed(
        OUT,
        workload=np.array("honeycomb 18x18, N=648, U=5, beta=20, dtau=0.1, L=200, n_wrap=10, Ising field, seed 0, "
                          "asymmetric split, one sweep with equal-time estimators"),
        field_bits=np.packbits(ch.field.ravel() > 0),
        field_shape=np.array(ch.field.shape),
        init_bits=np.packbits(f0.ravel() > 0),
        G_diag=np.diag(ch.G).copy(),
        G_rows_index=rows,
        G_rows=ch.G[rows].copy(),
        bins=ch.bins.copy(),
        proposals=np.array(ch.proposals),
        accepted=np.array(ch.accepted),
        prec_max=np.array(max(ch.prec)),
        min_tie=np.array(ch.min_tie),
    )
    print("wrote %s: %d proposals, %d accepted, prec_max %.3g, min |R - u| %.3g, %.0f s"
          % (OUT, ch.proposals, ch.accepted, max(ch.prec), ch.min_tie, dt))


if __name__ == "__main__":
    main()
