"""The paper's matrix-assembly route, kept literally for small cross-checks.

Sec. 3.2: Hermitian H stored as the upper triangle in CSR (val, col, row),
1-based, non-zeros only (the worked 5x5 example).  Alg. 2 builds the pattern
by comparing every pair of basis states (O(N^2)); Alg. 3 fills the values:
the diagonal is U times the number of doubly occupied sites, each
off-diagonal entry is a hop between two sites alpha, beta of one spin with
the fermionic sign (-1)^delta of Eq. (sign-explanation), delta being the
number of electrons strictly between the two modes in the order of
Eq. (statedef).  Time-dependent hops go into H_Re / H_Im so that
H(t) = H_stat + Re f(t) H_Re + i Im f(t) H_Im (Eq. (hamimplementation)).

Readings: the hop amplitude carries the minus sign of
Eq. (hubbardhamiltonian) (Alg. 3 prints +v); a hop beta -> alpha along a
bond with displacement dx = x_alpha - x_beta in {-1, 0, +1} has value
-t exp(i A dx) = -t (Re f + i dx Im f) with f = exp(iA), so dx = 0 bonds are
time independent; Alg. 2's final row pointer is the count plus one in
1-based numbering (row_{N+1} = k).  Only small sectors: the pattern pass is
quadratic.
"""
from __future__ import annotations

import numpy as np

from .fock import UP, DOWN, mode_index, sector_states, docc_weights


def csr_upper(M: np.ndarray):
    """Upper-triangle CSR of a Hermitian matrix, 1-based, non-zeros only."""
    n = M.shape[0]
    val, col, row = [], [], []
    for i in range(n):
        row.append(len(val) + 1)
        for j in range(i, n):
            if M[i, j] != 0:
                val.append(M[i, j])
                col.append(j + 1)
    row.append(len(val) + 1)
    return np.array(val), np.array(col), np.array(row)


def csr_upper_to_dense(val, col, row, n):
    M = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for k in range(row[i] - 1, row[i + 1] - 1):
            j = col[k] - 1
            M[i, j] = val[k]
            M[j, i] = np.conj(val[k])
    return M


def differ_bits(a: int, b: int) -> int:
    return bin(int(a) ^ int(b)).count("1")


def alg2_structure(states):
    """Alg. 2: (row, col), 1-based; a pair enters when the states differ in at
    most two occupation entries.  Vectorised per row, same output."""
    states = np.asarray(states, dtype=np.int64)
    n = len(states)
    row = np.zeros(n + 1, dtype=np.int64)
    cols = []
    k = 1
    for i in range(n):
        row[i] = k
        x = states[i:] ^ states[i]
        cnt = np.zeros(x.shape, dtype=np.int64)
        y = x.copy()
        while np.any(y):
            cnt += y & 1
            y >>= 1
        js = np.nonzero(cnt <= 2)[0] + i + 1
        cols.append(js)
        k += len(js)
    row[n] = k
    return row, np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)


def _hop_sites(a: int, b: int):
    """For states a (row) and b (column) differing by one hop: the mode that is
    occupied in a only (destination) and in b only (source)."""
    x = int(a) ^ int(b)
    m1 = (x & -x).bit_length() - 1
    m2 = x.bit_length() - 1
    if (int(a) >> m1) & 1:
        return m1, m2
    return m2, m1


def alg3_assembly(states, n_sites, U, bonds, row, col):
    """Alg. 3 values (H_stat, H_Re, H_Im) on the Alg. 2 pattern."""
    states = np.asarray(states, dtype=np.int64)
    nnz = len(col)
    Hs = np.zeros(nnz, dtype=np.complex128)
    Hr = np.zeros(nnz, dtype=np.complex128)
    Hi = np.zeros(nnz, dtype=np.complex128)
    bond_of = {}
    for (i, j, t, dx) in bonds:
        bond_of[(i, j)] = (t, dx)
        bond_of[(j, i)] = (t, -dx)
    w = docc_weights(states, n_sites)
    n = len(states)
    for r in range(n):
        for k in range(row[r] - 1, row[r + 1] - 1):
            c = col[k] - 1
            if c == r:
                Hs[k] += U * w[r]
                continue
            md, ms = _hop_sites(states[r], states[c])
            if md % 2 != ms % 2:
                continue  # would flip a spin: not a Hubbard hop
            alpha, beta = md // 2, ms // 2
            if (alpha, beta) not in bond_of:
                continue  # pruned: zero hopping amplitude
            t, dx = bond_of[(alpha, beta)]
            lo, hi = min(md, ms), max(md, ms)
            between = (int(states[c]) >> (lo + 1)) & ((1 << (hi - lo - 1)) - 1)
            sgn = -1.0 if bin(between).count("1") % 2 else 1.0
            if dx == 0:
                Hs[k] += sgn * (-t)
            else:
                Hr[k] = sgn * (-t)
                Hi[k] = sgn * (-t) * dx
    return Hs, Hr, Hi


def literal_H(states, n_sites, U, bonds, A: float):
    """Dense H(A) assembled through Alg. 2 + Alg. 3 + Eq. (hamimplementation)."""
    row, col = alg2_structure(states)
    Hs, Hr, Hi = alg3_assembly(states, n_sites, U, bonds, row, col)
    f = np.exp(1j * A)
    val = Hs + np.real(f) * Hr + 1j * np.imag(f) * Hi
    # the stored triangle is the row >= column half of the hop list: entry
    # (r, c) with c > r is <r|H|c>
    return csr_upper_to_dense(val, col, row, len(states)), len(col)
