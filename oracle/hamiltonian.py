"""Sparse FP64 matrix of the time-dependent Hubbard Hamiltonian in one sector.

Eq. (hubbardhamiltonian): H = - sum_{i,j,sigma} v_ji c^dag_{i sigma} c_{j sigma}
+ U sum_i n_{i up} n_{i down}, with the hopping matrix carrying the geometry
(Sec. 2.1) and the light pulse entering through the Peierls substitution of
Eq. (peierls).  With a uniform vector potential A(t) along the field the line
integral from R_i to R_j is A(t) (R_j - R_i); the electron charge is absorbed
in A, so a directed hop j -> i picks up exp(i A(t) dx_ij), dx_ij = (R_i - R_j)
along the field.  Each bond (i, j, t, dx) of the geometry therefore gives

    -t exp(+i A dx) c^dag_i c_j  -  t exp(-i A dx) c^dag_j c_i   (both spins).

Like the split of Eq. (hamimplementation), the matrix is stored once as
time-independent pieces: the diagonal D (interaction plus on-site energies)
and, for every distinct displacement d, the hopping matrix K_d summing the
directed hops with that displacement (amplitude -t, no phase), so that

    H(A) = D + sum_d exp(i A d) K_d.

Each directed hop is built as the product c^dag_{i sigma} c_{j sigma} of the
ladder operators of Eq. (creation-annihilation) (see `fock.apply_ladder`).

On-site energies: the lattice's `onsite[i]` = epsilon_i enters as
epsilon_i (n_{i up} + n_{i down}).  In the paper's notation this is the
diagonal of the hopping matrix with epsilon_i = -v_ii.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fock import UP, DOWN, mode_index, sector_states, apply_ladder, lookup, docc_weights


def pulse_A(pulse, t: float) -> float:
    """Vector potential (or Peierls phase per unit displacement) at time t.

    kind 0: A(t) = A0 exp(-(t-t0)^2/(2 sigma^2)) sin(omega (t-t0)), the
            Gaussian-windowed sine of Eq. (efield) used as the vector potential.
    kind 1: the phase of Eq. (vt): f(t) = exp(i a [cos(omega (t-t_p)) - b]
            exp(-(t-t_p)^2/(2 sigma^2))); returned is the exponent's real
            factor, so that bonds with dx = 1 carry f(t).
    """
    kind, A0, omega, t0, sigma, b = pulse.as_tuple() if hasattr(pulse, "as_tuple") else pulse
    s = t - t0
    env = np.exp(-s * s / (2.0 * sigma * sigma))
    if int(kind) == 0:
        return float(A0 * env * np.sin(omega * s))
    if int(kind) == 1:
        return float(A0 * (np.cos(omega * s) - b) * env)
    raise ValueError("unknown pulse kind")


class HubbardOracle:
    """H(A) = D + sum_d e^{iAd} K_d on the sector (n_up, n_dn) of a lattice."""

    def __init__(self, lattice, U: float, n_up: int, n_dn: int, states=None):
        self.lattice = lattice
        self.n_sites = lattice.n_sites
        self.U = float(U)
        self.n_up, self.n_dn = n_up, n_dn
        # `states` overrides the sector (e.g. the whole Fock space, Eq. (directsum))
        self.states = (sector_states(self.n_sites, n_up, n_dn) if states is None
                       else np.sort(np.asarray(states, dtype=np.int64)))
        self.dim = len(self.states)
        self.w_docc = docc_weights(self.states, self.n_sites)

        diag = self.U * self.w_docc.astype(np.float64)
        if lattice.onsite is not None:
            for i, eps in enumerate(lattice.onsite):
                for spin in (UP, DOWN):
                    diag = diag + eps * ((self.states >> mode_index(i, spin)) & 1)
        self.diag = diag

        # K_d for every displacement d
        pieces = {}
        for (i, j, t, dx) in lattice.bonds:
            if i == j:
                raise ValueError("on-site terms belong in lattice.onsite")
            for (dst, src, d) in ((i, j, dx), (j, i, -dx)):
                for spin in (UP, DOWN):
                    r, c, v = self._hop(dst, src, spin)
                    pieces.setdefault(float(d) + 0.0, []).append((r, c, -float(t) * v))
        self.K = {}
        for d, lst in pieces.items():
            r = np.concatenate([p[0] for p in lst])
            c = np.concatenate([p[1] for p in lst])
            v = np.concatenate([p[2] for p in lst])
            self.K[d] = sp.csr_matrix((v.astype(np.complex128), (r, c)),
                                      shape=(self.dim, self.dim))
        self.D = sp.diags(self.diag.astype(np.complex128), format="csr")

    def _hop(self, dst: int, src: int, spin: int):
        """Matrix entries of c^dag_{dst,spin} c_{src,spin}: rows, cols, values."""
        st = self.states
        v1, s1, g1 = apply_ladder(st, mode_index(src, spin), dagger=False)
        v2, s2, g2 = apply_ladder(s1, mode_index(dst, spin), dagger=True)
        ok = v1 & v2
        cols = np.nonzero(ok)[0]
        rows = lookup(st, s2[ok])
        vals = (g1 * g2)[ok]
        return rows, cols, vals

    def H(self, A: float) -> sp.csr_matrix:
        out = self.D.copy()
        for d, Kd in self.K.items():
            out = out + np.exp(1j * A * d) * Kd
        return out.tocsr()

    def apply(self, A: float, x: np.ndarray) -> np.ndarray:
        y = self.diag * x
        for d, Kd in self.K.items():
            y = y + np.exp(1j * A * d) * (Kd @ x)
        return y

    def norm_inf(self) -> float:
        """Max absolute row sum; independent of A because phases have modulus 1."""
        acc = np.abs(self.diag).astype(np.float64)
        for Kd in self.K.values():
            acc = acc + np.asarray(abs(Kd).sum(axis=1)).ravel()
        return float(acc.max())

    def row(self, A: float, k: int):
        """Row k of H(A), computed from the ladder action on basis state k alone.

        Used to check single outputs at sizes where the full matrix is costly:
        returns (column indices, values) of the non-zeros of row k.
        """
        st = self.states
        target = np.array([st[k]], dtype=np.int64)
        cols, vals = [k], [self.diag[k] + 0j]
        for (i, j, t, dx) in self.lattice.bonds:
            # row k collects the hops whose result is state k: the source is
            # obtained from state k by the adjoint hop.
            for (dst, src, d) in ((i, j, dx), (j, i, -dx)):
                for spin in (UP, DOWN):
                    v1, s1, g1 = apply_ladder(target, mode_index(dst, spin), dagger=False)
                    v2, s2, g2 = apply_ladder(s1, mode_index(src, spin), dagger=True)
                    if v1[0] and v2[0]:
                        c = int(lookup(st, s2)[0])
                        # <k| c^dag_dst c_src |c> = <c| c^dag_src c_dst |k>^*, real signs
                        cols.append(c)
                        vals.append(-t * g1[0] * g2[0] * np.exp(1j * A * d))
        return np.array(cols, dtype=np.int64), np.array(vals, dtype=np.complex128)
