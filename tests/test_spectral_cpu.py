"""Broadened spectral functions (Eq. (A_noneq_broad)), oracle pins on the CPU.

* the trapezoidal transform of a sum of exponentials equals its closed form
  (geometric series) — catches a wrong weight, sign or conjugation;
* with a fine grid and long window it converges to the Lorentzian Lehmann
  form of Eq. (spectralplot) (divided by pi), removal peaks at E0 - E_phi and
  addition peaks at E_phi - E0;
* from the ground state without a pulse the stepper's overlaps transform to
  the closed form built from the exact eigen-decomposition of the N -+ 1
  sectors, and the removal weights sum to <n_i sigma> = 1/2 at half filling.
"""
import numpy as np
import pytest

from oracle import HubbardOracle, ground_state
from oracle.fock import UP, DOWN, mode_index, ladder_matrix
from oracle.greens import greens_diag
from oracle import spectral as sp
from synth import ring, PulseParams


def _lehmann_parts(h, g, E0, site, spin, dagger):
    nu_, nd_ = (h.n_up + (1 if dagger else -1), h.n_dn) if spin == UP else (h.n_up, h.n_dn + (1 if dagger else -1))
    ht = HubbardOracle(h.lattice, h.U, nu_, nd_)
    Op = ladder_matrix(h.states, ht.states, mode_index(site, spin), dagger)
    w, V = np.linalg.eigh(ht.H(0.0).toarray())
    amp = np.abs(V.conj().T @ (Op @ g)) ** 2
    return amp, w - E0, ht


def test_trapezoid_transform_of_exponentials_closed_form():
    rng = np.random.default_rng(5)
    wts = rng.uniform(0.1, 1.0, 7)
    dE = rng.uniform(-6, 6, 7)
    dt, n, eps = 0.05, 300, 0.3
    s = np.arange(n + 1) * dt
    o = (wts[None, :] * np.exp(-1j * dE[None, :] * s[:, None])).sum(axis=1)
    nu = np.linspace(-8, 8, 41)
    for lesser in (True, False):
        got = sp.spectral_from_overlaps(o, lesser, dt, eps, nu)
        sgn = 1.0 if lesser else -1.0   # conj(o) turns e^{-i dE s} into e^{+i dE s}
        ref = [sp.trapezoid_of_exponentials(wts, -eps + 1j * (v + sgn * dE), n, dt).real / np.pi for v in nu]
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-13)


def test_fine_grid_converges_to_lorentzian_lehmann():
    wts = np.array([0.3, 0.5, 0.2])
    dE = np.array([1.5, 3.0, -2.0])
    dt, T, eps = 0.002, 40.0, 0.5
    n = int(round(T / dt))
    s = np.arange(n + 1) * dt
    o = (wts[None, :] * np.exp(-1j * dE[None, :] * s[:, None])).sum(axis=1)
    nu = np.linspace(-6, 6, 25)
    lesser = sp.spectral_from_overlaps(o, True, dt, eps, nu)
    greater = sp.spectral_from_overlaps(o, False, dt, eps, nu)
    assert np.allclose(lesser, sp.lorentzian_lehmann(wts, -dE, eps, nu), atol=2e-5)
    assert np.allclose(greater, sp.lorentzian_lehmann(wts, dE, eps, nu), atol=2e-5)


def test_equilibrium_greens_transform_matches_eigendecomposition():
    lat = ring(6)
    h = HubbardOracle(lat, 4.0, 3, 3)
    E0, _, g = ground_state(h, 0.0)
    p = PulseParams(0, 0.0, 1.0, 0.0, 1.0)   # no field
    dt, n, eps = 0.05, 120, 0.4
    nu = np.linspace(-8, 8, 33)
    for site, spin, dagger in ((0, UP, False), (2, DOWN, True)):
        amp, dE, ht = _lehmann_parts(h, g, E0, site, spin, dagger)
        o = greens_diag(h, g, p, 0.0, dt, 0, n, site, spin, dagger, ham_target=ht)
        got = sp.spectral_from_overlaps(o, not dagger, dt, eps, nu)
        sgn = 1.0 if not dagger else -1.0
        ref = [sp.trapezoid_of_exponentials(amp, -eps + 1j * (v + sgn * dE), n, dt).real / np.pi for v in nu]
        assert np.allclose(got, ref, atol=1e-10)
    # removal weights sum to <n_{i sigma}> = 1/2 on the half-filled ring
    amp, _, _ = _lehmann_parts(h, g, E0, 3, DOWN, False)
    assert amp.sum() == pytest.approx(0.5, abs=1e-12)
