"""Two-time Green's functions on the diagonal (Eq. (Glg)), FP64 CPU reference.

Sec. 2.5: G^<_{ii sigma}(t, t') = i <psi(t')| c^dag_{i sigma} T exp(-i int_t^t' H)
c_{i sigma} |psi(t)>, obtained (Sec. 3.7) by applying c to psi(t), evolving the
result in the sector with one electron less, and projecting on c psi(t'):

    G^<(t, t + s) = i  < c psi(t+s) | U(t+s, t) c psi(t) >
    G^>(t + s, t) = -i < c^dag psi(t+s) | U(t+s, t) c^dag psi(t) >

(for G^> the same construction with c^dag, in the sector with one electron
more).  U is the same midpoint stepper as for psi (Eq. (time-stepping)) on the
same time grid, each exponential evaluated to machine precision.  The overlap
is a scalar, so it does not depend on the operator-order convention of the
basis.
"""
from __future__ import annotations

import numpy as np

from .fock import UP, DOWN, mode_index, ladder_matrix
from .hamiltonian import HubbardOracle
from .stepper import midpoint_step_exact


def op_sector(n_up: int, n_dn: int, spin: int, dagger: bool):
    d = 1 if dagger else -1
    return (n_up + d, n_dn) if spin == UP else (n_up, n_dn + d)


def greens_diag(ham: HubbardOracle, psi0: np.ndarray, pulse, t0: float, dt: float, start_step: int,
                n_rel: int, site: int, spin: int, dagger: bool, ham_target: HubbardOracle = None):
    """Overlaps o(s) = < op psi(t'+s) | U(t'+s, t') op psi(t') > for s = 0..n_rel
    steps, t' = t0 + start_step dt, psi(t0) = psi0.  G^< = i o (op = c),
    G^> = -i o (op = c^dag)."""
    nu, nd = op_sector(ham.n_up, ham.n_dn, spin, dagger)
    if ham_target is None:
        ham_target = HubbardOracle(ham.lattice, ham.U, nu, nd)
    Op = ladder_matrix(ham.states, ham_target.states, mode_index(site, spin), dagger)
    psi = psi0.copy()
    t = t0
    for n in range(start_step):
        psi = midpoint_step_exact(ham, psi, t, dt, pulse)
        t = t0 + (n + 1) * dt
    phi = Op @ psi
    out = np.empty(n_rel + 1, dtype=np.complex128)
    out[0] = np.vdot(Op @ psi, phi)
    for s in range(n_rel):
        psi = midpoint_step_exact(ham, psi, t, dt, pulse)
        phi = midpoint_step_exact(ham_target, phi, t, dt, pulse)
        t = t0 + (start_step + s + 1) * dt
        out[s + 1] = np.vdot(Op @ psi, phi)
    return out


def lehmann_overlap(ham: HubbardOracle, psi0: np.ndarray, E0: float, ham_target: HubbardOracle,
                    site: int, spin: int, dagger: bool, times: np.ndarray):
    """Equilibrium (time-independent H, psi0 an eigenstate with energy E0):
    o(s) = sum_phi |<phi| op |psi0>|^2 exp(-i (E_phi - E0) s), from a full
    eigendecomposition of the target sector (the Lehmann sum behind
    Eq. (spectralfunction))."""
    Op = ladder_matrix(ham.states, ham_target.states, mode_index(site, spin), dagger)
    w, V = np.linalg.eigh(ham_target.H(0.0).toarray())
    amp = V.conj().T @ (Op @ psi0)
    wts = np.abs(amp) ** 2
    return np.array([np.sum(wts * np.exp(-1j * (w - E0) * s)) for s in times])
