"""Non-interacting (U = 0) reference for the midpoint stepper.

At U = 0 the Hamiltonian of Eq. (hubbardhamiltonian) with the Peierls phases
of Eq. (peierls) is the second quantisation of the one-particle matrix
h(A)_{ij} = -t_ij exp(i A dx_ij) (plus epsilon_i on the diagonal), separately
for each spin.  exp(-i tau H) maps a Slater determinant with orbitals Phi to
the determinant with orbitals exp(-i tau h) Phi, so the many-body midpoint
stepper of Eq. (time-stepping) reduces exactly to propagating Phi with
exp(-i tau h(A_mid)).  Observables follow from the one-body density
<c^dag_i c_j> = (Phi Phi^dag)_{ji}: E = tr(h rho)/Ns summed over spins, and
d_i = <n_{i up}><n_{i down}> because the state is a product of an up and a
down determinant.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.linalg as sla

from .hamiltonian import pulse_A


def one_body(lattice, A: float) -> np.ndarray:
    n = lattice.n_sites
    h = np.zeros((n, n), dtype=np.complex128)
    for (i, j, t, dx) in lattice.bonds:
        h[i, j] += -t * np.exp(1j * A * dx)
        h[j, i] += -t * np.exp(-1j * A * dx)
    if lattice.onsite is not None:
        h += np.diag(np.asarray(lattice.onsite, dtype=np.float64))
    return h


def ground_orbitals(lattice, n_el: int, A: float = 0.0):
    """Lowest n_el eigenvectors of h(A) and the gap at the Fermi level."""
    w, U = np.linalg.eigh(one_body(lattice, A))
    gap = w[n_el] - w[n_el - 1] if 0 < n_el < len(w) else np.inf
    return U[:, :n_el], w, gap


def step(lattice, phis, t: float, tau: float, pulse):
    h = one_body(lattice, pulse_A(pulse, t + 0.5 * tau))
    P = sla.expm(-1j * tau * h)
    return [P @ p for p in phis]


def observables(lattice, phis, A: float):
    """(energy per site, docc per site, site docc) for the up/down determinants."""
    h = one_body(lattice, A)
    n = lattice.n_sites
    E = 0.0
    dens = []
    for p in phis:
        rho = p @ p.conj().T          # rho[j, i] = <c^dag_i c_j>
        E += float(np.real(np.sum(h * rho.T)))
        dens.append(np.real(np.diag(rho)))
    site = dens[0] * dens[1]
    return E / n, float(site.sum()) / n, site


def slater_vector(phi_up, phi_dn, ham):
    """Many-body amplitude of the product of two Slater determinants on the
    oracle's interleaved basis: psi[k] = <k| prod_a c^dag(phi_up[:,a]) prod_b
    c^dag(phi_dn[:,b]) |0>, with the determinants' creators in the order
    (all up, then all down) and each basis state's creators in the order of
    Eq. (statedef).  Small sectors only (explicit minors)."""
    from .fock import UP, DOWN, mode_index
    n = ham.n_sites
    out = np.zeros(ham.dim, dtype=np.complex128)
    for k, s in enumerate(ham.states):
        ups = [i for i in range(n) if (s >> mode_index(i, UP)) & 1]
        dns = [i for i in range(n) if (s >> mode_index(i, DOWN)) & 1]
        du = np.linalg.det(phi_up[ups, :]) if ups else 1.0
        dd = np.linalg.det(phi_dn[dns, :]) if dns else 1.0
        # reorder from (ups ascending, dns ascending) to the interleaved order
        cross = sum(1 for j in dns for i in ups if i > j)
        out[k] = (-1) ** cross * du * dd
    return out
