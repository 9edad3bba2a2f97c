"""The paper's own set-ups through the library (NEXT-4 of the build plan):
open 8x1 chain and the 4x2 box (Sec. 4), the phase pulse of Eq. (vt)
(pulse kind 1) and on-site energies v_ii, propagated from the ground state
against the exact-exponential oracle (psi, d(t), E(t) within 1e-10)."""
import math

import numpy as np
import pytest

import paper_2005_13498_amd as hub
from oracle import HubbardOracle, to_canonical, from_canonical, pulse_A, ground_state
from oracle.stepper import midpoint_step_exact, observables
from synth import chain, cluster_2d, PulseParams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    # 8x1 open chain, half filling, Eq. (vt) pulse (a = 0.8, omega = 9, t_p = 0.6, sigma = 0.2, b = cos(omega t_p))
    ("chain8", chain(8), 8.0, 4, 4, PulseParams(1, 0.8, 9.0, 0.6, 0.2, math.cos(9.0 * 0.6))),
    # 4x2 box with open boundaries, field along x, on-site energies
    ("box4x2", cluster_2d(4, 2, periodic=False).with_onsite([0.3, -0.2, 0.1, 0.0, -0.1, 0.2, -0.3, 0.05]), 6.0, 4, 4,
     PulseParams(0, 0.7, 6.0, 0.5, 0.25)),
]


@pytest.mark.parametrize("name,lat,U,nu,nd,pulse", CASES)
def test_paper_geometry_propagation(name, lat, U, nu, nd, pulse):
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd, device=0)
    try:
        A0 = pulse_A(pulse, 0.0)
        v = torch.empty(B.dim, dtype=torch.complex128, device=DEV)
        st, e0, gap = hub.hub_ground_state(B.handle, A0, v, hub.make_opts(tol=1e-13, m_max=60))
        E0, _, _ = ground_state(ham, A0)
        assert e0 == pytest.approx(E0, abs=1e-10 * abs(E0))
        psi = from_canonical(v.cpu().numpy(), ham.states, lat.n_sites)
        dt, n = 0.01, 120
        st, obs, log = hub.hub_propagate(B.handle, [pulse], 0.0, dt, n, hub.make_opts(tol=1e-13, m_max=30), v)
        ref = []
        x = psi.copy()
        for k in range(n + 1):
            t = k * dt
            _, e, d, _ = observables(ham, x, pulse_A(pulse, t))
            ref.append((e, d))
            if k < n:
                x = midpoint_step_exact(ham, x, t, dt, pulse)
        ref = np.array(ref)
        got = v.cpu().numpy()
        r = to_canonical(x, ham.states, lat.n_sites)
        assert np.linalg.norm(got - r) / np.linalg.norm(r) < 1e-10
        assert np.max(np.abs(obs[:, 0, 2] - ref[:, 0])) < 1e-10 * np.max(np.abs(ref[:, 0]))
        assert np.max(np.abs(obs[:, 0, 3] - ref[:, 1])) < 1e-10 * max(np.max(np.abs(ref[:, 1])), 1e-3)
    finally:
        B.close()
