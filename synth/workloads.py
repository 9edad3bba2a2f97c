"""Workload presets and seeded random inputs.

Each preset names a lattice, the interaction U, the particle-number sector, a
pulse parameter set and the stepping parameters.  Pulse parameters are stored,
never evaluated here: A(t) = A0 exp(-(t-t0)^2 / (2 sigma^2)) sin(omega (t-t0))
(kind 0, the vector potential used directly as the Peierls phase, the
configurations' form of Eq. (efield)), or the paper's phase factor of
Eq. (vt) (kind 1, parameters a, b, omega, t_p, sigma).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, Optional, Tuple

import numpy as np

from .lattices import Lattice, ring, cluster_2d

SEED = 13498


@dataclass(frozen=True)
class PulseParams:
    kind: int = 0           # 0: Gaussian-sine vector potential, 1: Eq. (vt) phase
    A0: float = 0.0         # amplitude (kind 0) or a (kind 1)
    omega: float = 0.0
    t0: float = 0.0         # pulse centre (t_p in the paper)
    sigma: float = 1.0
    b: float = 0.0          # kind 1 only

    def as_tuple(self):
        return (self.kind, self.A0, self.omega, self.t0, self.sigma, self.b)


@dataclass(frozen=True)
class Workload:
    name: str
    lattice: Lattice
    U: float
    n_up: int
    n_dn: int
    pulse: PulseParams
    dt: float
    n_steps: int
    tol: float
    m_max: int = 30
    extra: Dict = field(default_factory=dict)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def draw_amplitudes(n: int, low: float = 0.2, high: float = 1.0, seed: int = SEED) -> np.ndarray:
    """The seeded pulse amplitudes A0 ~ U[low, high], in draw order."""
    return np.random.default_rng(seed).uniform(low, high, size=n)


def controller_draws(n: int, seed: int = SEED + 1):
    """Seeded (U, A0, omega) triples for controller training runs:
    U ~ U[4, 12], A0 ~ U[0.2, 1.2], omega ~ U[U/2, 2U], drawn in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        U = float(rng.uniform(4.0, 12.0))
        A0 = float(rng.uniform(0.2, 1.2))
        om = float(rng.uniform(0.5 * U, 2.0 * U))
        out.append((U, A0, om))
    return out


def controller_groups(n_groups: int, members: int, seed: int):
    """Seeded draws for controller runs in groups sharing U (one basis per
    group): U ~ U[4, 12] per group, then per member A0 ~ U[0.2, 1.2] and
    omega ~ U[U/2, 2U]; [(U, [(A0, omega), ...]), ...]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_groups):
        U = float(rng.uniform(4.0, 12.0))
        out.append((U, [(float(rng.uniform(0.2, 1.2)), float(rng.uniform(0.5 * U, 2.0 * U))) for _ in range(members)]))
    return out


def random_state(dim: int, seed: int = 1, nvec: int = 1) -> np.ndarray:
    """Complex standard-normal vectors, each normalised to 1; shape (nvec, dim)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nvec, dim)) + 1j * rng.standard_normal((nvec, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def workloads() -> Dict[str, Workload]:
    """The five workload presets (ring8, cluster3x4, ring10 batch, ring14 block, controller)."""
    a0 = draw_amplitudes(8)
    ring_pulse = PulseParams(0, 0.5, 8.0, 1.0, 0.3)
    out = {
        # 8-site ring at half filling, Lanczos ground state of H(0), 200 steps
        "ring8": Workload("ring8", ring(8), 8.0, 4, 4, ring_pulse,
                          dt=0.01, n_steps=200, tol=1e-12, m_max=30),
        # 12-site 3x4 periodic cluster, field along x, 1000 steps
        "cluster3x4": Workload("cluster3x4", cluster_2d(3, 4), 8.0, 6, 6,
                               PulseParams(0, float(a0[0]), 8.0, 2.5, 0.5),
                               dt=0.005, n_steps=1000, tol=1e-10, m_max=30,
                               extra={"A0_batch": tuple(float(v) for v in a0)}),
        # 10-site ring, ground sector (5,5), 64 excited members in the N+-1 sectors
        "ring10_greens": Workload("ring10_greens", ring(10), 8.0, 5, 5, ring_pulse,
                                  dt=0.01, n_steps=400, tol=1e-10, m_max=30,
                                  extra={"sites": (0, 3, 6, 9),
                                         "t_primes": (0.5, 1.0, 1.5, 2.0)}),
        # 14-site ring at half filling, block of 8 pulse amplitudes
        "ring14_block": Workload("ring14_block", ring(14), 8.0, 7, 7, ring_pulse,
                                 dt=0.01, n_steps=200, tol=1e-10, m_max=30,
                                 extra={"A0_batch": tuple(0.1 * k for k in range(1, 9))}),
        # controller training logs: 10-site ring runs under seeded (U, A0, omega)
        "controller": Workload("controller", ring(10), 8.0, 5, 5, ring_pulse,
                               dt=0.01, n_steps=400, tol=1e-8, m_max=30,
                               extra={"draws": tuple(controller_draws(16))}),
    }
    return out
