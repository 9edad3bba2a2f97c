"""Lattice geometries as explicit bond lists.

The paper encodes the geometry in a hopping matrix v (Sec. 2.1): any pair of
sites may be connected, periodic boundaries are just extra matrix elements, and
on-site energies sit on its diagonal.  Here a geometry is a list of undirected
bonds (i, j, t_ij, dx_ij) where t_ij = |v_ij| > 0 and dx_ij is the projection of
R_i - R_j on the field direction.  On a periodic wrap bond dx uses the minimum
image, so that a ring threaded by a uniform A(t) carries a net flux.  The
on-site array holds epsilon_i, the energy of one electron on site i.

These are plain data; evaluating Peierls phases from them is left to whoever
builds the Hamiltonian.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple


@dataclass(frozen=True)
class Lattice:
    name: str
    n_sites: int
    bonds: Tuple[Tuple[int, int, float, float], ...]  # (i, j, t, dx)
    onsite: Optional[Tuple[float, ...]] = None
    positions: Tuple[Tuple[float, float], ...] = field(default=())

    @property
    def n_bonds(self) -> int:
        return len(self.bonds)

    def arrays(self):
        """Bond endpoints, amplitudes and displacements as four lists."""
        bi = [b[0] for b in self.bonds]
        bj = [b[1] for b in self.bonds]
        bt = [float(b[2]) for b in self.bonds]
        bdx = [float(b[3]) for b in self.bonds]
        return bi, bj, bt, bdx

    def with_onsite(self, eps) -> "Lattice":
        return Lattice(self.name + "+onsite", self.n_sites, self.bonds,
                       tuple(float(e) for e in eps), self.positions)

    def with_hopping(self, t: float) -> "Lattice":
        return Lattice(f"{self.name}(t={t})", self.n_sites,
                       tuple((i, j, float(t), dx) for (i, j, _, dx) in self.bonds),
                       self.onsite, self.positions)


def _min_image(d: float, period: int) -> float:
    """Shortest signed displacement on a circle of length `period`."""
    d = d % period
    if d > period / 2:
        d -= period
    return float(d)


def ring(n: int, t: float = 1.0) -> Lattice:
    """Periodic 1D ring, nearest-neighbour bonds (i, i+1 mod n), field along the ring."""
    if n < 3:
        raise ValueError("a ring needs at least 3 sites (use two_site for 2)")
    bonds = []
    for i in range(n):
        j = (i + 1) % n
        bonds.append((i, j, t, _min_image(i - j, n)))
    pos = tuple((float(i), 0.0) for i in range(n))
    return Lattice(f"ring{n}", n, tuple(bonds), None, pos)


def chain(n: int, t: float = 1.0) -> Lattice:
    """Open 1D chain (open boundary conditions), field along the chain."""
    bonds = tuple((i, i + 1, t, -1.0) for i in range(n - 1))
    pos = tuple((float(i), 0.0) for i in range(n))
    return Lattice(f"chain{n}", n, bonds, None, pos)


def two_site(t: float = 1.0) -> Lattice:
    """A single bond between two sites (the smallest open chain)."""
    return Lattice("two_site", 2, ((0, 1, t, -1.0),), None, ((0.0, 0.0), (1.0, 0.0)))


def cluster_2d(lx: int, ly: int, t: float = 1.0, periodic: bool = True,
               field_dir: Tuple[float, float] = (1.0, 0.0)) -> Lattice:
    """Rectangular lx-by-ly cluster, site index x + lx*y (lexicographic).

    Nearest-neighbour bonds along x and y; with `periodic` the wrap bonds are
    included (minimum-image displacement).  A dimension of length 2 with
    periodic wrap would duplicate its bond, so wraps are only added for
    lengths >= 3.  dx is the bond displacement projected on `field_dir`.
    """
    ex, ey = field_dir
    bonds: List[Tuple[int, int, float, float]] = []

    def idx(x, y):
        return x + lx * y

    for y in range(ly):
        for x in range(lx):
            # bond to +x neighbour
            if x + 1 < lx or (periodic and lx >= 3):
                x2 = (x + 1) % lx
                ddx = _min_image(x - x2, lx) if periodic else float(x - x2)
                bonds.append((idx(x, y), idx(x2, y), t, ddx * ex))
    for y in range(ly):
        for x in range(lx):
            if y + 1 < ly or (periodic and ly >= 3):
                y2 = (y + 1) % ly
                ddy = _min_image(y - y2, ly) if periodic else float(y - y2)
                bonds.append((idx(x, y), idx(x, y2), t, ddy * ey))
    pos = tuple((float(x), float(y)) for y in range(ly) for x in range(lx))
    kind = "pbc" if periodic else "obc"
    return Lattice(f"cluster{lx}x{ly}{kind}", lx * ly, tuple(bonds), None, pos)


def ring_nnn(n: int, t: float = 1.0, t2: float = 0.4) -> Lattice:
    """Periodic ring with nearest (t) and next-nearest (t2) neighbour bonds,
    field along the ring (minimum-image displacements)."""
    if n < 5:
        raise ValueError("next-nearest bonds need at least 5 sites")
    bonds = []
    for i in range(n):
        for step, amp in ((1, t), (2, t2)):
            j = (i + step) % n
            bonds.append((i, j, amp, _min_image(i - j, n)))
    pos = tuple((float(i), 0.0) for i in range(n))
    return Lattice(f"ring{n}nnn", n, tuple(bonds), None, pos)


def random_graph(n: int, n_bonds: int, seed: int, amplitudes=(1.0, 0.5), displacements=(-1.0, 0.0, 1.0)) -> Lattice:
    """Seeded graph of n sites and n_bonds distinct bonds between arbitrary
    site pairs (the paper's hopping matrix allows any pair), amplitudes and
    field displacements drawn from the given small sets, random on-site
    energies in [-0.5, 0.5]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    pick = rng.choice(len(pairs), size=n_bonds, replace=False)
    bonds = tuple((pairs[k][0], pairs[k][1], float(rng.choice(amplitudes)), float(rng.choice(displacements)))
                  for k in sorted(pick))
    onsite = tuple(float(e) for e in rng.uniform(-0.5, 0.5, n))
    return Lattice(f"graph{n}_{n_bonds}_{seed}", n, bonds, onsite, tuple((float(i), 0.0) for i in range(n)))
