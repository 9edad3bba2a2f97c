"""Map between the paper's interleaved basis and the spin-separated tile layout.

The paper notes (below Eq. (creation-annihilation)) that the operator order
defining a basis state is a convention.  The oracle uses the interleaved order
of Eq. (statedef).  Results are compared in the spin-separated convention:
the state is c^dag_{up...} (all up creators, site 0 leftmost) times
c^dag_{down...} (all down creators) on the vacuum, and a vector is a
dim_up x dim_down tile indexed by (a, b), where a is the position of the
up-occupation string among all such strings sorted as integers (bit i =
site i) and b likewise for the down string.

Reordering the creators from interleaved to separated order moves every up
creator on site i past every down creator on a site j < i, so
|state>_interleaved = S |state>_separated with
S = (-1)^{sum over occupied (j, down) of #{i > j : (i, up) occupied}}.
Hence psi_separated[a, b] = S * psi_interleaved[k].

Only the test-suite uses this map; the rank here is a plain sort position, not
the combinatorial ranking formula of Eq. (hashing).
"""
from __future__ import annotations

import numpy as np

from .fock import UP, DOWN, mode_index


def _spin_strings(states: np.ndarray, n_sites: int, spin: int) -> np.ndarray:
    out = np.zeros(states.shape, dtype=np.int64)
    for i in range(n_sites):
        out |= ((states >> mode_index(i, spin)) & 1) << i
    return out


def canonical_map(states: np.ndarray, n_sites: int):
    """For each interleaved basis state: (flat tile index a*dim_dn + b, sign S,
    dim_up, dim_dn, sorted up strings, sorted down strings)."""
    states = np.asarray(states, dtype=np.int64)
    ups = _spin_strings(states, n_sites, UP)
    dns = _spin_strings(states, n_sites, DOWN)
    up_sorted = np.unique(ups)
    dn_sorted = np.unique(dns)
    a = np.searchsorted(up_sorted, ups)
    b = np.searchsorted(dn_sorted, dns)
    dim_dn = len(dn_sorted)
    # crossing count: for each occupied down site j, the up electrons on sites > j
    cross = np.zeros(states.shape, dtype=np.int64)
    for j in range(n_sites):
        dn_j = (dns >> j) & 1
        ups_above = np.zeros(states.shape, dtype=np.int64)
        for i in range(j + 1, n_sites):
            ups_above += (ups >> i) & 1
        cross += dn_j * ups_above
    sign = np.where(cross % 2 == 0, 1.0, -1.0)
    return a * dim_dn + b, sign, len(up_sorted), dim_dn, up_sorted, dn_sorted


def to_canonical(psi: np.ndarray, states: np.ndarray, n_sites: int) -> np.ndarray:
    """Interleaved-basis vector(s) (..., dim) -> flat separated tile (..., dim)."""
    flat, sign, _, _, _, _ = canonical_map(states, n_sites)
    out = np.empty_like(psi)
    out[..., flat] = sign * psi
    return out


def from_canonical(psi_c: np.ndarray, states: np.ndarray, n_sites: int) -> np.ndarray:
    """Inverse of `to_canonical`."""
    flat, sign, _, _, _, _ = canonical_map(states, n_sites)
    return sign * psi_c[..., flat]
