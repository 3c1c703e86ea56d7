"""Hopping matrices of the lattices used by the workloads.

Conventions follow the paper's worked examples:

* Square lattice (section "The SU(2)-Hubbard model on a square lattice", the
  hopping-term paragraph): unit vectors a1 = (1, 0), a2 = (0, 1); periodic
  torus; T[I, I+a1] = T[I+a1, I] = T[I, I+a2] = T[I+a2, I] = -t and
  T[I, I] = -mu.  The matrix elements are *assigned*, not accumulated, so on a
  lattice of extent 2 a bond that wraps twice is counted once.
* Honeycomb lattice (section "Working with multi-orbital unit cells" and its
  hopping-term listing): triangular Bravais lattice a1 = (1, 0),
  a2 = (1/2, sqrt(3)/2), two orbitals per unit cell, super-index
  nc = 2*I + no (0-based here).  Orbital A of cell I hops to orbital B of
  cells I, I + a1 - a2 and I - a2 with amplitude -t.

Unit cell I has coordinates (i1, i2) with I = i1 + L1*i2 and position
R_I = i1*a1 + i2*a2.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Lattice:
    name: str
    L1: int
    L2: int
    norb: int
    a1: np.ndarray
    a2: np.ndarray
    K: np.ndarray            # N x N hopping matrix, fp64, symmetric
    cell_of: np.ndarray      # [N] unit-cell index of each orbital
    orb_of: np.ndarray       # [N] orbital index within the cell
    cell_pos: np.ndarray     # [Ncell, 2] real-space position of each cell

    @property
    def n(self) -> int:
        return self.K.shape[0]

    @property
    def n_cells(self) -> int:
        return self.L1 * self.L2

    def reciprocal(self):
        """Reciprocal vectors g1, g2 with a_i . g_j = 2 pi delta_ij."""
        A = np.stack([self.a1, self.a2])            # rows a1, a2
        G = 2.0 * np.pi * np.linalg.inv(A).T        # rows g1, g2
        return G[0], G[1]

    def sublattice_sign(self) -> np.ndarray:
        """(-1)^x staggering of a bipartite lattice (+1 on A, -1 on B)."""
        if self.name == "honeycomb":
            return np.where(self.orb_of == 0, 1.0, -1.0)
        i1 = self.cell_of % self.L1
        i2 = self.cell_of // self.L1
        return np.where((i1 + i2) % 2 == 0, 1.0, -1.0)


def bonds_of(K: np.ndarray):
    """The bonds of a hopping matrix: pairs (a, b), a < b, with K[a, b] != 0,
    in row-major order (the structure of the bond vertices of the
    transverse-Ising example, Eq. (hubbard_sun_Ising))."""
    n = K.shape[0]
    return [(a, b) for a in range(n) for b in range(a + 1, n) if K[a, b] != 0.0]


def bonds_sharing_a_site(bonds):
    """Pairs (i, j), i < j, of bond indices whose bonds share a site."""
    return [(i, j) for i in range(len(bonds)) for j in range(i + 1, len(bonds))
            if set(bonds[i]) & set(bonds[j])]


def _cell(i1, i2, L1, L2):
    return (i1 % L1) + L1 * (i2 % L2)


def square_lattice(L1: int, L2: int, t: float = 1.0, mu: float = 0.0) -> Lattice:
    n = L1 * L2
    K = np.zeros((n, n))
    for i2 in range(L2):
        for i1 in range(L1):
            I = _cell(i1, i2, L1, L2)
            Ix = _cell(i1 + 1, i2, L1, L2)
            Iy = _cell(i1, i2 + 1, L1, L2)
            K[I, Ix] = -t
            K[Ix, I] = -t
            K[I, Iy] = -t
            K[Iy, I] = -t
            K[I, I] = -mu
    cells = np.arange(n)
    pos = np.stack([cells % L1, cells // L1], axis=1).astype(float)
    return Lattice("square", L1, L2, 1, np.array([1.0, 0.0]), np.array([0.0, 1.0]),
                   K, cells.copy(), np.zeros(n, dtype=np.int64), pos)


def honeycomb_lattice(L1: int, L2: int, t: float = 1.0, mu: float = 0.0) -> Lattice:
    ncell = L1 * L2
    n = 2 * ncell
    K = np.zeros((n, n))
    a1 = np.array([1.0, 0.0])
    a2 = np.array([0.5, np.sqrt(3.0) / 2.0])
    for i2 in range(L2):
        for i1 in range(L1):
            I = _cell(i1, i2, L1, L2)
            A = 2 * I
            K[A, A] = -mu
            K[A + 1, A + 1] = -mu
            for (d1, d2) in ((0, 0), (1, -1), (0, -1)):
                B = 2 * _cell(i1 + d1, i2 + d2, L1, L2) + 1
                K[A, B] = -t
                K[B, A] = -t
    cells = np.arange(ncell)
    i1 = cells % L1
    i2 = cells // L1
    pos = i1[:, None] * a1[None, :] + i2[:, None] * a2[None, :]
    cell_of = np.repeat(cells, 2)
    orb_of = np.tile(np.arange(2), ncell)
    return Lattice("honeycomb", L1, L2, 2, a1, a2, K, cell_of, orb_of, pos)
