"""Periodic chain and square lattices (paper section 2.3, standard models).

Sites are numbered x + Lx*y.  Bonds are unordered nearest-neighbour pairs
listed once each; the hopping term of the Hamiltonian uses every bond in both
directions.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Lattice:
    kind: str                 # "chain" or "square"
    Lx: int
    Ly: int
    coords: np.ndarray        # [n_sites, 2] int
    bonds: np.ndarray         # [n_bonds, 2] int32, i < j not required

    @property
    def n_sites(self) -> int:
        return self.Lx * self.Ly

    def displacement(self, i: int, j: int) -> tuple[int, int]:
        """(dx, dy) from site i to site j, each reduced mod the period."""
        xi, yi = self.coords[i]
        xj, yj = self.coords[j]
        return int((xj - xi) % self.Lx), int((yj - yi) % self.Ly)

    def min_image(self, i: int, j: int) -> tuple[int, int]:
        """Absolute minimum-image separation (|dx|, |dy|)."""
        dx, dy = self.displacement(i, j)
        dx = min(dx, self.Lx - dx)
        dy = min(dy, self.Ly - dy)
        return dx, dy


def chain(L: int) -> Lattice:
    if L < 3:
        raise ValueError("periodic chain needs L >= 3")
    coords = np.stack([np.arange(L), np.zeros(L, dtype=int)], axis=1)
    bonds = np.array([(i, (i + 1) % L) for i in range(L)], dtype=np.int32)
    return Lattice("chain", L, 1, coords, bonds)


def square(L: int) -> Lattice:
    if L < 3:
        raise ValueError("periodic square lattice needs L >= 3")
    n = L * L
    coords = np.array([(s % L, s // L) for s in range(n)], dtype=int)
    bonds = []
    for s in range(n):
        x, y = coords[s]
        bonds.append((s, ((x + 1) % L) + L * y))
        bonds.append((s, x + L * ((y + 1) % L)))
    return Lattice("square", L, L, coords, np.array(bonds, dtype=np.int32))
