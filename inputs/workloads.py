"""The synthetic Hubbard workloads (parameters only).

Each workload is a half-filled Hubbard model (t = 1, mu = 0) on a periodic
lattice.  The paper runs no public dataset; these parameter sets are the
benchmark inputs themselves.
"""
from dataclasses import dataclass, field as dc_field
from typing import Callable, Optional, Tuple

from .lattices import Lattice, honeycomb_lattice, square_lattice


@dataclass
class Workload:
    name: str
    lattice: Callable[[], Lattice]
    U: float
    beta: float
    dtau: float
    n_wrap: int
    field_kind: str = "ising"     # "ising" (s = +-1) or "gauss" (continuous phi)
    trotter: str = "sym"          # measurement split
    seed: int = 0
    n_chains: int = 1
    extra: dict = dc_field(default_factory=dict)

    @property
    def n_slices(self) -> int:
        return int(round(self.beta / self.dtau))


WORKLOADS = {
    # 4x4 square, N=16, U=4, beta=2, L=20, 200 sweeps, symmetric split
    "square4x4_U4_b2": Workload("square4x4_U4_b2", lambda: square_lattice(4, 4), 4.0, 2.0, 0.1, 10,
                                extra={"sweeps": 200, "bins": 20}),
    # honeycomb 12x12 cells, N=288, U=4, beta=10, L=100
    "honeycomb12_U4_b10": Workload("honeycomb12_U4_b10", lambda: honeycomb_lattice(12, 12), 4.0, 10.0,
                                   0.1, 10, trotter="asym"),
    # batched: 256 x 8x8, 128 x 6x6, 128 x 10x10, U=4, beta=8, L=80
    "batched512_U4_b8": Workload("batched512_U4_b8", lambda: square_lattice(8, 8), 4.0, 8.0, 0.1, 10,
                                 n_chains=512),
    # continuous field, 10x10 square, U=4, beta=4, L=40, 64 chains
    "gauss10x10_U4_b4": Workload("gauss10x10_U4_b4", lambda: square_lattice(10, 10), 4.0, 4.0, 0.1, 10,
                                 field_kind="gauss", n_chains=64),
    # honeycomb 18x18 cells, N=648, U=5, beta=20, L=200, time-displaced G
    "honeycomb18_U5_b20": Workload("honeycomb18_U5_b20", lambda: honeycomb_lattice(18, 18), 5.0, 20.0,
                                   0.1, 10, trotter="asym"),
}


def batched_chain_layout(n_chains: int = 512) -> Tuple[Tuple[int, int, int], ...]:
    """(chain seed, L1, L2) for the mixed-size batch: the first half of the
    chains on 8x8, the next quarter on 6x6, the last quarter on 10x10."""
    out = []
    for c in range(n_chains):
        if c < n_chains // 2:
            out.append((c, 8, 8))
        elif c < (3 * n_chains) // 4:
            out.append((c, 6, 6))
        else:
            out.append((c, 10, 10))
    return tuple(out)


def lattice_for(L1: int, L2: int, kind: str = "square") -> Optional[Lattice]:
    return square_lattice(L1, L2) if kind == "square" else honeycomb_lattice(L1, L2)
