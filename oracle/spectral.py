"""Broadened spectral functions from the diagonal Green's functions, FP64 CPU
reference (Eq. (A_noneq_broad), Eq. (spectralplot)).

TEST INFRASTRUCTURE ONLY (see the package header).

Overlaps o(s) as returned by `greens.greens_diag` on the stepper grid s_k = k dt,
k = 0..n:  o<(s) = <c psi(t+s)| U c psi(t)>,  o>(s) = <c^dag psi(t+s)| U c^dag psi(t)>.
Then G<(t, t+s) = i o<(s) and G>(t+s, t) = -i o>(s).  Reading of the transform:
the lesser part integrates G<(t+s, t) = -conj G<(t, t+s) and the greater part
carries the sign that makes it non-negative, so that in equilibrium

    A<(nu) = (1/pi) sum_phi |<phi|c|psi0>|^2   eps / ((nu - (E0 - E_phi))^2 + eps^2)
    A>(nu) = (1/pi) sum_phi |<phi|c^dag|psi0>|^2 eps / ((nu - (E_phi - E0))^2 + eps^2),

the Lorentzian Lehmann form of Eq. (spectralplot) (there without the 1/pi):

    A<(nu, t) = (1/pi) Re int_0^T e^{-eps s} e^{i nu s} conj(o<(s)) ds
    A>(nu, t) = (1/pi) Re int_0^T e^{-eps s} e^{i nu s} o>(s) ds,   T = n dt,

with the integral taken by the trapezoidal rule on the stepper grid.
"""
from __future__ import annotations

import numpy as np


def trapezoid_weights(n: int, dt: float) -> np.ndarray:
    w = np.full(n + 1, dt)
    w[0] = w[-1] = 0.5 * dt
    if n == 0:
        w[0] = 0.0
    return w


def spectral_from_overlaps(o: np.ndarray, lesser: bool, dt: float, eps: float, nu: np.ndarray) -> np.ndarray:
    """A<(nu) (lesser=True, o from c) or A>(nu) (o from c^dag) for one member."""
    o = np.asarray(o, dtype=np.complex128)
    n = len(o) - 1
    s = np.arange(n + 1) * dt
    z = np.conj(o) if lesser else o
    w = trapezoid_weights(n, dt) * np.exp(-eps * s)
    out = np.empty(len(nu))
    for k, v in enumerate(nu):
        out[k] = np.real(np.sum(w * np.exp(1j * v * s) * z)) / np.pi
    return out


def lorentzian_lehmann(weights: np.ndarray, centers: np.ndarray, eps: float, nu: np.ndarray) -> np.ndarray:
    """(1/pi) sum_k w_k eps / ((nu - c_k)^2 + eps^2)."""
    d = np.asarray(nu)[:, None] - np.asarray(centers)[None, :]
    return (np.asarray(weights)[None, :] * eps / (d * d + eps * eps)).sum(axis=1) / np.pi


def trapezoid_of_exponentials(weights: np.ndarray, rates: np.ndarray, n: int, dt: float) -> complex:
    """Closed form of the trapezoidal rule applied to sum_k w_k e^{r_k s} on
    s = 0, dt, ..., n dt: dt (sum_{l=0}^{n} q^l - (1 + q^n) / 2), q = e^{r dt}."""
    q = np.exp(np.asarray(rates) * dt)
    geo = np.where(np.abs(q - 1) > 1e-14, (1 - q ** (n + 1)) / (1 - q), n + 1.0)
    return complex(np.sum(np.asarray(weights) * dt * (geo - 0.5 * (1 + q ** n))))
