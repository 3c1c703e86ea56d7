"""Helpers of the GPU parity tests: build both sides from the same inputs."""
import numpy as np

from inputs import honeycomb_lattice, square_lattice
from oracle import hubbard as ohub


def lattice(kind, L1, L2):
    return square_lattice(L1, L2) if kind == "square" else honeycomb_lattice(L1, L2)


def pair(kind, L1, L2, U, beta, dtau, n_wrap, trotter="sym", seed=0, field="ising"):
    """(oracle model, product chain) for the same workload."""
    import paper_1704_00131_amd as pa
    lat = lattice(kind, L1, L2)
    om = ohub.hubbard_model(lat.K, U, beta, dtau, n_wrap, field_kind=field, trotter=trotter, seed=seed)
    lam = pa.hubbard_coupling(U, dtau, field)
    pm = pa.make_model(lat.n, beta, dtau, n_wrap, lam, U=U, field=field, trotter=trotter, seed=seed)
    return om, pa.Chain(pm, lat.K), lat


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
