"""Occupation-number basis and fermionic ladder operators.

Paper Sec. 2.3: a state is |n_{1up} n_{1down} n_{2up} ... n_{Ns down}>, built
from the vacuum by creation operators in exactly that order (Eq. (statedef)).
The particle-number sectors H^{n_up}_{n_down} of Eq. (directsum) are spanned by
the basis states with the given number of up and down electrons, and their
dimension is C(Ns, n_up) C(Ns, n_down) (Eq. (statedim)).

A basis state is an integer: bit 2*i holds n_{i,up}, bit 2*i+1 holds
n_{i,down} (sites 0-based).  Mode k = 2*i + sigma is the k-th operator from
the left in Eq. (statedef).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

UP, DOWN = 0, 1


def mode_index(site: int, spin: int) -> int:
    """Position of (site, spin) in the operator order of Eq. (statedef)."""
    return 2 * site + spin


def popcount(x: np.ndarray) -> np.ndarray:
    """Number of set bits of each entry (int64 input, any shape)."""
    x = np.asarray(x, dtype=np.int64)
    return np.bitwise_count(x).astype(np.int64)


def sector_states(n_sites: int, n_up: int, n_dn: int) -> np.ndarray:
    """All basis states of H^{n_up}_{n_dn}(n_sites), ascending as integers.

    Built as every placement of n_up up electrons combined with every
    placement of n_dn down electrons (the tensor-product structure noted under
    Eq. (statedim)); the result is sorted so lookups can bisect.
    """
    if not (0 <= n_up <= n_sites and 0 <= n_dn <= n_sites):
        raise ValueError("particle numbers out of range")

    def spread(sites, spin):
        v = 0
        for s in sites:
            v |= 1 << mode_index(s, spin)
        return v

    ups = np.array([spread(c, UP) for c in combinations(range(n_sites), n_up)], dtype=np.int64)
    dns = np.array([spread(c, DOWN) for c in combinations(range(n_sites), n_dn)], dtype=np.int64)
    states = (ups[:, None] | dns[None, :]).ravel()
    states.sort()
    return states


def apply_ladder(states: np.ndarray, mode: int, dagger: bool):
    """Act with c_mode (dagger=False) or c^dagger_mode on each basis state.

    Eq. (creation-annihilation): c^dagger gives zero on an occupied mode, c on
    an empty one; otherwise the mode is flipped and the amplitude is
    (-1)^{c_mode}, where c_mode counts occupied modes strictly before `mode`
    in the operator order (the anticommutations needed to bring the operator
    to its place).  The square-root factors are 1 for fermions.

    Returns (valid, new_states, signs): `valid` marks states with a non-zero
    result; new_states/signs are meaningful where valid.
    """
    states = np.asarray(states, dtype=np.int64)
    bit = np.int64(1) << np.int64(mode)
    occupied = (states & bit) != 0
    valid = ~occupied if dagger else occupied
    before = states & (bit - 1)
    sign = np.where(popcount(before) % 2 == 0, 1.0, -1.0)
    new = states ^ bit
    return valid, new, sign


def lookup(sorted_states: np.ndarray, targets: np.ndarray) -> np.ndarray:
    """Index of each target in the sorted basis (bisection; the paper's
    'linear search or hash', Sec. 3.6-3.7).  Raises if a target is missing."""
    idx = np.searchsorted(sorted_states, targets)
    idx_c = np.minimum(idx, len(sorted_states) - 1)
    if len(targets) and not np.all(sorted_states[idx_c] == targets):
        raise KeyError("state not in target sector")
    return idx


def ladder_matrix(states_from: np.ndarray, states_to: np.ndarray, mode: int,
                  dagger: bool):
    """Sparse matrix of c_mode / c^dagger_mode from one sector to another."""
    import scipy.sparse as sp
    valid, new, sign = apply_ladder(states_from, mode, dagger)
    cols = np.nonzero(valid)[0]
    rows = lookup(states_to, new[valid])
    return sp.csr_matrix((sign[valid], (rows, cols)),
                         shape=(len(states_to), len(states_from)))


def docc_weights(states: np.ndarray, n_sites: int) -> np.ndarray:
    """Weight vector w_d of Sec. 3.5: number of doubly occupied sites per state."""
    states = np.asarray(states, dtype=np.int64)
    w = np.zeros(states.shape, dtype=np.int64)
    for i in range(n_sites):
        up = (states >> mode_index(i, UP)) & 1
        dn = (states >> mode_index(i, DOWN)) & 1
        w += up & dn
    return w


def site_occupations(states: np.ndarray, n_sites: int, spin: int) -> np.ndarray:
    """n_{i,spin} for every state, shape (len(states), n_sites)."""
    states = np.asarray(states, dtype=np.int64)
    return np.stack([(states >> mode_index(i, spin)) & 1 for i in range(n_sites)], axis=1)
