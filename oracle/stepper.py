"""Exponential midpoint stepper, ground state and observables (FP64, CPU).

Eq. (time-stepping): v^(n+1) = exp(-i tau H(n tau + tau/2)) v^(n), the
lowest-order Magnus step with the integral of Eq. (magnus) taken by the
midpoint rule of Eq. (midpoint-rule).  Here every exponential is evaluated to
machine precision (dense expm for small sectors, scipy's expm_multiply
otherwise), so the oracle computes the same discrete scheme as the Krylov
method but without the Krylov truncation.

Ground state (Sec. 3.4, "Ground state"): the eigenvector of the smallest
eigenvalue of H; obtained with dense or sparse Hermitian eigensolvers instead
of the power iteration of Alg. 4/5, which `power_iteration_ground_state`
keeps for small cross-checks.

Observables (Sec. 2.4 Eqs. (observable), (docc), (energy); Sec. 3.5): the
double occupation per site via the weight vector w_d, the energy per site
<psi|H(t)|psi>/Ns at the sample time t, the norm, and the site-resolved
double occupation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .fock import UP, DOWN, site_occupations
from .hamiltonian import pulse_A

DENSE_LIMIT = 2500


def expm_apply(H, v: np.ndarray, tau: float) -> np.ndarray:
    """exp(-i tau H) v to machine precision."""
    n = H.shape[0]
    if n <= DENSE_LIMIT:
        Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
        return sla.expm(-1j * tau * Hd) @ v
    return spla.expm_multiply(-1j * tau * H, v)


def midpoint_step_exact(ham, v: np.ndarray, t: float, tau: float, pulse) -> np.ndarray:
    """One step of Eq. (time-stepping) from time t."""
    A_mid = pulse_A(pulse, t + 0.5 * tau)
    return expm_apply(ham.H(A_mid), v, tau)


def cfet4_step_exact(ham, v: np.ndarray, t: float, tau: float, pulse) -> np.ndarray:
    """One step of the fourth-order commutator-free exponential integrator
    (the higher-order alternative the paper points to in Sec. 3.4): with the
    Gauss nodes c = 1/2 -+ sqrt(3)/6 and a = (3 -+ 2 sqrt(3))/12,
        v <- exp(-i tau (a1 H1 + a2 H2)) exp(-i tau (a2 H1 + a1 H2)) v,
    H_k = H(A(t + c_k tau)), each exponential exact."""
    r3 = np.sqrt(3.0)
    c1, c2 = 0.5 - r3 / 6.0, 0.5 + r3 / 6.0
    a1, a2 = (3.0 - 2.0 * r3) / 12.0, (3.0 + 2.0 * r3) / 12.0
    H1 = ham.H(pulse_A(pulse, t + c1 * tau))
    H2 = ham.H(pulse_A(pulse, t + c2 * tau))
    w = expm_apply(a2 * H1 + a1 * H2, v, tau)
    return expm_apply(a1 * H1 + a2 * H2, w, tau)


def observables(ham, v: np.ndarray, A: float):
    """(norm, energy per site, double occupation per site, site-resolved docc)."""
    p = np.abs(v) ** 2
    norm = float(np.sqrt(p.sum()))
    Hv = ham.apply(A, v)
    energy = float(np.real(np.vdot(v, Hv))) / ham.n_sites
    docc = float(np.dot(ham.w_docc, p)) / ham.n_sites
    nu = site_occupations(ham.states, ham.n_sites, UP)
    nd = site_occupations(ham.states, ham.n_sites, DOWN)
    site = (nu * nd * p[:, None]).sum(axis=0)
    return norm, energy, docc, site


def propagate_exact(ham, v0: np.ndarray, t0: float, tau: float, n_steps: int, pulse,
                    record: bool = True):
    """Run n_steps midpoint steps; returns final vector and, if `record`, the
    observables at every sample time t0 + n tau (n = 0..n_steps)."""
    v = v0.copy()
    obs = []
    t = t0
    for n in range(n_steps):
        if record:
            obs.append((t,) + observables(ham, v, pulse_A(pulse, t))[:3])
        v = midpoint_step_exact(ham, v, t, tau, pulse)
        t = t0 + (n + 1) * tau
    if record:
        obs.append((t,) + observables(ham, v, pulse_A(pulse, t))[:3])
    return v, obs


def fix_phase(v: np.ndarray) -> np.ndarray:
    """Multiply by a unit phase so that the component of largest modulus is
    real and positive (lowest index among components within 1e-12 relative of
    the largest)."""
    a = np.abs(v)
    k = int(np.nonzero(a >= a.max() * (1 - 1e-12))[0][0])
    return v * (np.conj(v[k]) / a[k])


def ground_state(ham, A: float = 0.0, k: int = 3, tol: float = 1e-14):
    """(E0, E1, psi0): lowest two eigenvalues and the ground state of H(A)."""
    H = ham.H(A)
    n = H.shape[0]
    if n <= DENSE_LIMIT:
        w, U = np.linalg.eigh(H.toarray())
        return float(w[0]), float(w[1]) if n > 1 else np.inf, fix_phase(U[:, 0])
    w, U = spla.eigsh(H, k=min(k, n - 1), which="SA", tol=tol)
    order = np.argsort(w)
    w, U = w[order], U[:, order]
    return float(w[0]), float(w[1]), fix_phase(U[:, 0])


def power_iteration(apply_M, n: int, n_max: int, tol: float, rng):
    """Alg. 4: power iteration for the eigenpair of largest |lambda|.

    Reading: the stopping test compares consecutive normalised iterates up to
    a global sign (for a negative dominant eigenvalue the iterates alternate
    in sign otherwise and never pass the printed test)."""
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    lam_prev = 0.0
    lam = 0.0
    for _ in range(n_max):
        w = apply_M(v)
        lam = float(np.real(np.vdot(v, w)))
        w /= np.linalg.norm(w)
        phase = np.vdot(v, w)
        phase = phase / abs(phase) if abs(phase) > 0 else 1.0
        w_al = w / phase
        if abs(lam - lam_prev) <= tol * abs(lam_prev) and \
                np.linalg.norm(w_al - v) <= tol * np.linalg.norm(v):
            v = w
            break
        v = w
        lam_prev = lam
    return lam, v


def power_iteration_ground_state(ham, A: float, n_max: int = 200000, tol: float = 1e-12,
                                 seed: int = 0):
    """Alg. 5: power iteration on H, and on H - E I if the first result is >= 0."""
    rng = np.random.default_rng(seed)
    H = ham.H(A)
    E, v = power_iteration(lambda x: H @ x, H.shape[0], n_max, tol, rng)
    if E < 0:
        return E, v
    E2, v2 = power_iteration(lambda x: H @ x - E * x, H.shape[0], n_max, tol, rng)
    return E + E2, v2
