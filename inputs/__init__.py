"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds only input construction: lattice hopping matrices, the
workload parameter sets and chain-to-lattice assignments.  It contains none of
the method's arithmetic (no Hubbard-Stratonovich constants, no matrix
exponentials, no Green's functions), so that the oracle and the GPU path stay
independent of each other.
"""
from .lattices import Lattice, bonds_of, bonds_sharing_a_site, honeycomb_lattice, square_lattice  # noqa: F401
from .workloads import WORKLOADS, Workload, batched_chain_layout  # noqa: F401
