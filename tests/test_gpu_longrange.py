"""Hoppings beyond nearest neighbours (Sec. 2.1: the hopping matrix may
connect any two sites) through the library against the oracle:

* an 8-site ring with next-nearest-neighbour bonds (t' = 0.4, displacement
  2 along the field), half filling;
* a seeded graph of 7 sites with 12 bonds between arbitrary pairs, two
  amplitudes, three field displacements and random on-site energies.

H x of single vectors and blocks within 1e-13 (complex128) of the oracle's
sparse H, and 60 midpoint steps under a pulse against the exact-exponential
stepper within 1e-10 (psi, d(t), E(t))."""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import ring_nnn, random_graph, random_state, PulseParams
from oracle import HubbardOracle, to_canonical, from_canonical, pulse_A, observables, midpoint_step_exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [("ring8nnn", ring_nnn(8, 1.0, 0.4), 6.0, 4, 4), ("graph7", random_graph(7, 12, seed=21), 4.0, 3, 4)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name,lat,U,nu,nd", CASES)
def test_long_range_apply(name, lat, U, nu, nd):
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd)
    try:
        n = lat.n_sites
        for nvec in (1, 8):
            xs = random_state(ham.dim, seed=60 + nvec, nvec=nvec)
            As = list(np.linspace(-0.9, 1.4, nvec))
            ref = [to_canonical(ham.apply(A, x), ham.states, n) for A, x in zip(As, xs)]
            x = torch.from_numpy(np.concatenate([to_canonical(v, ham.states, n) for v in xs])).to(DEV)
            for path in (-1, 0, 1):
                hub.hub_set_apply_path(B.handle, path)
                y = torch.empty_like(x)
                hub.hub_apply_H(B.handle, As, x, y)
                got = y.cpu().numpy().reshape(nvec, -1)
                for k in range(nvec):
                    assert _rel(got[k], ref[k]) < 1e-13, (name, nvec, path, k)
    finally:
        hub.hub_set_apply_path(B.handle, -1)
        B.close()


@pytest.mark.parametrize("name,lat,U,nu,nd", CASES)
def test_long_range_propagation(name, lat, U, nu, nd):
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd)
    try:
        n = lat.n_sites
        pulses = [PulseParams(0, 0.9, 6.0, 0.3, 0.2), PulseParams(0, 0.4, 9.0, 0.2, 0.15)]
        xs = random_state(ham.dim, seed=77, nvec=2)
        x = torch.from_numpy(np.concatenate([to_canonical(v, ham.states, n) for v in xs])).to(DEV)
        steps, dt = 60, 0.01
        st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, dt, steps, hub.make_opts(tol=1e-13, m_max=30), x)
        got = x.cpu().numpy().reshape(2, -1)
        for k in range(2):
            v = xs[k].copy()
            ref = []
            for s in range(steps + 1):
                _, e, d, _ = observables(ham, v, pulse_A(pulses[k], s * dt))
                ref.append((e, d))
                if s < steps:
                    v = midpoint_step_exact(ham, v, s * dt, dt, pulses[k])
            r = np.array(ref)
            assert _rel(from_canonical(got[k], ham.states, n), v) < 1e-10
            assert np.max(np.abs(obs[:, k, 2] - r[:, 0])) < 1e-10 * max(1.0, np.max(np.abs(r[:, 0])))
            assert np.max(np.abs(obs[:, k, 3] - r[:, 1])) < 1e-10
    finally:
        B.close()
