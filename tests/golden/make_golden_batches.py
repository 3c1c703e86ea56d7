"""Writes the oracle's values for sampled chains of the two batched workloads,
from the oracle only (never from the HIP path).

    python tests/golden/make_golden_batches.py [c3] [c4]

c3 -> batched512_U4_b8_chains.npz: chains {0, 1, 255, 256, 383, 384, 511} of
the 512-chain mixed batch (256 x 8x8, 128 x 6x6, 128 x 10x10; U = 4,
beta = 8, dtau = 0.1, L = 80, n_wrap = 10, two-valued field, symmetric split,
seed = chain index) after the sweeps the batch workload runs: four
unmeasured sweeps (the autotuner's trials: one per GEMM kernel) and one sweep
with the equal-time estimators (the captured sweep).  Per chain: the field
(signs, bit-packed), the diagonal of G(0) and 8 of its rows, the bin sums,
the counts and the smallest |R - u| (near-tie guard).

c4 -> gauss10x10_U4_b4_chains.npz: chains of the 64-chain Gaussian batch
(10x10 square, U = 4, beta = 4, L = 40, n_wrap = 10, seed = chain index):
the gradient d log det / d phi of the initial field at every fourth slice for
chains {0, 1, 17, 32, 48, 63}, and for chains {0, 31, 63} the field after one
Monte Carlo step (one local sweep, then ten Langevin steps with eps = 1e-3
and steps 0..9), with the local sweep's smallest |R - u|.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import batched_chain_layout, square_lattice  # noqa: E402
from oracle import gradient, hubbard, sweep  # noqa: E402

C3_CHAINS = (0, 1, 255, 256, 383, 384, 511)
C4_GRAD_CHAINS = (0, 1, 17, 32, 48, 63)
C4_STEP_CHAINS = (0, 31, 63)
GRAD_SLICES = tuple(range(1, 41, 4)) + (40,)


def g_rows(n):
    return np.unique(np.array([0, 1, n // 3, n // 2, (2 * n) // 3, n - 2, n - 1, 31 % n]))[:8]


def make_c3():
    lay = batched_chain_layout(512)
    out = {"chains": np.array(C3_CHAINS)}
    for c in C3_CHAINS:
        seed, L1, L2 = lay[c]
        lat = square_lattice(L1, L2)
        m = hubbard.hubbard_model(lat.K, 4.0, 8.0, 0.1, 10, trotter="sym", seed=seed)
        f0 = hubbard.init_field(m)
        ch = sweep.Chain(m, f0).init()
        t0 = time.time()
        for _ in range(4):
            ch.sweep(measure=False)
        ch.sweep(measure=True)
        rows = g_rows(m.N)
        out["field_bits_%d" % c] = np.packbits(ch.field.ravel() > 0)
        out["G_diag_%d" % c] = np.diag(ch.G).copy()
        out["G_rows_index_%d" % c] = rows
        out["G_rows_%d" % c] = ch.G[rows].copy()
        out["bins_%d" % c] = ch.bins.copy()
        out["counts_%d" % c] = np.array([ch.proposals, ch.accepted])
        out["min_tie_%d" % c] = np.array(ch.min_tie)
        print("c3 chain %d (N = %d): %d accepted, min |R - u| %.3g, %.0f s"
              % (c, m.N, ch.accepted, ch.min_tie, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "batched512_U4_b8_chains.npz"), **out)


def make_c4():
    lat = square_lattice(10, 10)
    out = {"grad_chains": np.array(C4_GRAD_CHAINS), "step_chains": np.array(C4_STEP_CHAINS),
           "grad_slices": np.array(GRAD_SLICES)}
    for c in sorted(set(C4_GRAD_CHAINS) | set(C4_STEP_CHAINS)):
        m = hubbard.hubbard_model(lat.K, 4.0, 4.0, 0.1, 10, field_kind="gauss", seed=c)
        f0 = hubbard.init_field(m)
        t0 = time.time()
        if c in C4_GRAD_CHAINS:
            out["grad_%d" % c] = gradient.grad_logdet(m, f0, GRAD_SLICES)
        if c in C4_STEP_CHAINS:
            ch = sweep.Chain(m, f0).init()
            ch.sweep(measure=False)
            f = ch.field.copy()
            for k in range(10):
                f = gradient.langevin_step(m, f, 1e-3, k)
            out["field_after_step_%d" % c] = f
            out["min_tie_%d" % c] = np.array(ch.min_tie)
        print("c4 chain %d: %.0f s" % (c, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "gauss10x10_U4_b4_chains.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c4"]
    if "c3" in which:
        make_c3()
    if "c4" in which:
        make_c4()
