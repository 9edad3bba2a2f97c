"""The resident stepper of small sectors (hub_set_propagate_path 1, the
automatic choice where it applies), through the C ABI.

One launch runs every midpoint step (Eq. (time-stepping)) of each vector in
one workgroup with its tile in LDS.  It must reproduce:

* the exact-exponential oracle (states, d(t), E(t)) at the 1e-10 bar in
  complex128 and 1e-5 in complex64, on sectors with on-site energies, an
  empty spin species and next-nearest-neighbour hops;
* the launch path (path 0) on the same inputs: states, observables and the
  Krylov dimension of every step, for single vectors and batches with
  different pulses, across its instantiations (1 to 16 elements per thread,
  ragged tiles up to 15,876 states);
* the fourth-order scheme and substeps (several Krylov solves per step)
  against the launch path and the oracle's exact exponentials;
* the stopping rules: m_max (HUB_E_NOT_CONVERGED, that step's approximation
  kept, later observables NaN), a non-finite input (HUB_E_INVALID), a zero
  vector (stays zero), no steps (observables of the input only);
* the argument checks of a forced path, and the automatic choice (the
  resident stepper where nvec * 6144 covers the sector's dimension, the
  launch path otherwise: seen in the launch counters).
"""
import numpy as np
import pytest
import torch

import paper_2005_13498_amd as hub
from oracle import HubbardOracle, to_canonical, from_canonical, pulse_A
from oracle.stepper import midpoint_step_exact, observables
from synth import PulseParams, chain, cluster_2d, random_state, ring, ring_nnn, two_site, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _vecs(dim, nv, seed, dtype):
    x = np.concatenate(random_state(dim, seed=seed, nvec=nv))
    return torch.from_numpy(x).to(DEV).to(dtype).contiguous()


def _pulses(nv):
    return [PulseParams(0, 0.4 + 0.15 * k, 8.0, 0.1, 0.3) for k in range(nv)]


def _run(B, path, pulses, x0, dt, n, opts, allow_nc=False):
    hub.hub_set_propagate_path(B.handle, path)
    try:
        v = x0.clone()
        st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, dt, n, opts, v, allow_not_converged=allow_nc)
    finally:
        hub.hub_set_propagate_path(B.handle, -1)
    return st, v, obs, log


CASES = [
    # lattice, U, n_up, n_dn, dtype, nvec, steps
    (ring(8), 8.0, 4, 4, torch.complex128, 3, 40),
    (ring(8), 8.0, 4, 4, torch.complex64, 2, 40),
    (chain(7).with_onsite([0.3, -0.2, 0.0, 0.5, 0.1, -0.4, 0.2]), 3.0, 3, 4, torch.complex128, 2, 30),
    (cluster_2d(3, 2), 8.0, 3, 3, torch.complex64, 3, 30),
    (ring_nnn(8), 6.0, 3, 4, torch.complex128, 1, 30),
    (ring(6), 4.0, 0, 3, torch.complex128, 2, 20),
    (two_site(), 8.0, 1, 1, torch.complex128, 2, 20),
    (ring(4), 4.0, 4, 4, torch.complex128, 2, 5),     # full sector: one state, no hops
    (chain(5), 3.0, 5, 2, torch.complex128, 2, 10),   # up species full: down hops only
    (ring(9), 8.0, 3, 3, torch.complex128, 1, 10),   # 7,056 states: 8 per thread
    (ring(9), 8.0, 4, 4, torch.complex64, 1, 10),    # 15,876 states: 16 per thread
]


@pytest.mark.parametrize("lat,U,nu,nd,dtype,nv,n", CASES)
def test_resident_matches_launch_path(lat, U, nu, nd, dtype, nv, n):
    B = hub.Basis(lat, U, nu, nd, device=0)
    try:
        x0 = _vecs(B.dim, nv, 91, dtype)
        opts = hub.make_opts(tol=1e-12 if dtype == torch.complex128 else 1e-7, m_max=30)
        pulses = _pulses(nv)
        _, v0, o0, l0 = _run(B, 0, pulses, x0, 0.02, n, opts)
        _, v1, o1, l1 = _run(B, 1, pulses, x0, 0.02, n, opts)
        c128 = dtype == torch.complex128
        bar = 1e-12 if c128 else 1e-5
        a, b = v1.cpu().numpy().reshape(nv, -1), v0.cpu().numpy().reshape(nv, -1)
        for k in range(nv):
            assert np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) < bar
        assert np.max(np.abs(o1[:, :, 1:] - o0[:, :, 1:])) < bar
        assert np.array_equal(o1[:, :, 0], o0[:, :, 0])
        same_m = np.mean(l1[:, :, 0] == l0[:, :, 0])
        assert same_m == 1.0 if c128 else same_m >= 0.9, same_m
        assert (l1[:, :, 2] == 1).all()
        if B.dim > 1:
            assert (l1[:, :, 5] > 0).all()
    finally:
        B.close()


@pytest.mark.parametrize("dtype,scheme,subs", [(torch.complex128, 1, 1), (torch.complex128, 0, 3),
                                               (torch.complex128, 1, 2), (torch.complex64, 1, 1)])
def test_resident_substeps_and_fourth_order_match_launch_path(dtype, scheme, subs):
    """The fourth-order scheme (two exponentials per step) and substeps (equal
    Krylov solves per exponential) on both paths: states, observables, the
    per-step log (largest m of the solves)."""
    B = hub.Basis(ring(8), 8.0, 4, 4, device=0)
    try:
        x0 = _vecs(B.dim, 2, 102, dtype)
        c128 = dtype == torch.complex128
        opts = hub.make_opts(tol=1e-12 if c128 else 1e-7, m_max=30, scheme=scheme, substeps=subs)
        _, v0, o0, l0 = _run(B, 0, _pulses(2), x0, 0.04, 20, opts)
        _, v1, o1, l1 = _run(B, 1, _pulses(2), x0, 0.04, 20, opts)
        bar = 1e-12 if c128 else 1e-5
        a, b = v1.cpu().numpy().reshape(2, -1), v0.cpu().numpy().reshape(2, -1)
        for k in range(2):
            assert np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]) < bar
        assert np.max(np.abs(o1[:, :, 1:] - o0[:, :, 1:])) < bar
        same_m = np.mean(l1[:, :, 0] == l0[:, :, 0])
        assert same_m == 1.0 if c128 else same_m >= 0.9, same_m
        assert (l1[:, :, 1] == subs).all() and (l1[:, :, 2] == 1).all()
    finally:
        B.close()


def test_resident_fourth_order_matches_oracle():
    """The fourth-order scheme on the resident stepper against the oracle's
    exact exponentials of the same scheme (7-site chain with on-site
    energies)."""
    from oracle.stepper import cfet4_step_exact
    lat = chain(7).with_onsite([0.3, -0.2, 0.0, 0.5, 0.1, -0.4, 0.2])
    U, nu, nd = 3.0, 3, 4
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd, device=0)
    try:
        p = PulseParams(0, 0.6, 5.0, 0.3, 0.2)
        psi = random_state(ham.dim, seed=103)[0]
        n, dt = 15, 0.04
        v = psi.copy()
        for k in range(n):
            v = cfet4_step_exact(ham, v, k * dt, dt, p)
        x = torch.from_numpy(to_canonical(psi, ham.states, lat.n_sites)).to(DEV)
        hub.hub_set_propagate_path(B.handle, 1)
        hub.hub_propagate(B.handle, [p], 0.0, dt, n, hub.make_opts(tol=1e-13, m_max=40, scheme=1), x)
        got = from_canonical(x.cpu().numpy(), ham.states, lat.n_sites)
        assert np.linalg.norm(got - v) / np.linalg.norm(v) < 1e-10
    finally:
        B.close()


@pytest.mark.parametrize("dtype,bar", [(torch.complex128, 1e-10), (torch.complex64, 1e-5)])
def test_resident_matches_oracle(dtype, bar):
    """7-site chain with on-site energies (3 up, 4 down), 30 steps of 0.02
    under a pulse, against exact exponentials: psi, d(t), E(t)."""
    lat = chain(7).with_onsite([0.3, -0.2, 0.0, 0.5, 0.1, -0.4, 0.2])
    U, nu, nd = 3.0, 3, 4
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd, device=0)
    try:
        p = PulseParams(0, 0.6, 5.0, 0.3, 0.2)
        psi = random_state(ham.dim, seed=93)[0]
        n, dt = 30, 0.02
        ref_obs = []
        v = psi.copy()
        for k in range(n):
            ref_obs.append(observables(ham, v, pulse_A(p, k * dt))[:3])
            v = midpoint_step_exact(ham, v, k * dt, dt, p)
        ref_obs.append(observables(ham, v, pulse_A(p, n * dt))[:3])
        x = torch.from_numpy(to_canonical(psi, ham.states, lat.n_sites)).to(DEV).to(dtype)
        hub.hub_set_propagate_path(B.handle, 1)
        st, obs, log = hub.hub_propagate(B.handle, [p], 0.0, dt, n, hub.make_opts(tol=1e-13 if dtype == torch.complex128
                                                                                  else 1e-7, m_max=40), x)
        got = from_canonical(x.cpu().numpy().astype(np.complex128), ham.states, lat.n_sites)
        assert np.linalg.norm(got - v) / np.linalg.norm(v) < bar
        r = np.array(ref_obs)
        for col in range(3):
            assert np.max(np.abs(obs[:, 0, 1 + col] - r[:, col])) < bar * max(1.0, np.max(np.abs(r[:, col])))
    finally:
        B.close()


def test_resident_workload_ring8_matches_launch_path_over_the_pulse():
    """The 8-site latency workload (ground state, 200 steps of 0.01, tol
    1e-12) on both paths."""
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    try:
        g = torch.empty(B.dim, dtype=torch.complex128, device=DEV)
        hub.hub_ground_state(B.handle, hub.hub_pulse_A(w.pulse, 0.0), g, hub.make_opts(tol=1e-13, m_max=100))
        opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
        _, v0, o0, l0 = _run(B, 0, [w.pulse], g, w.dt, w.n_steps, opts)
        _, v1, o1, l1 = _run(B, 1, [w.pulse], g, w.dt, w.n_steps, opts)
        assert torch.linalg.norm(v1 - v0).item() < 1e-11
        assert np.max(np.abs(o1[:, 0, 1:] - o0[:, 0, 1:])) < 1e-11
        assert np.array_equal(l1[:, 0, 0], l0[:, 0, 0])
        assert np.max(np.abs(l1[:, 0, 4] - l0[:, 0, 4])) < 1e-3 * w.tol + 1e-18
    finally:
        B.close()


def test_resident_m_max_stop_matches_launch_path():
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    try:
        x0 = _vecs(B.dim, 2, 94, torch.complex128)
        opts = hub.make_opts(tol=1e-15, m_max=3)
        s0, v0, o0, l0 = _run(B, 0, _pulses(2), x0, 0.05, 4, opts, allow_nc=True)
        s1, v1, o1, l1 = _run(B, 1, _pulses(2), x0, 0.05, 4, opts, allow_nc=True)
        assert s0 == s1 == hub.HUB_E_NOT_CONVERGED
        assert (l1[0, :, 0] == 3).all() and (l1[0, :, 2] == 0).all()
        assert torch.linalg.norm(v1 - v0).item() < 1e-12 * torch.linalg.norm(v0).item()
        assert np.max(np.abs(o1[:2, :, 1:] - o0[:2, :, 1:])) < 1e-12
        assert np.isnan(o1[2:, :, 1:]).all()
    finally:
        B.close()


def test_resident_zero_vector_and_no_steps():
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    try:
        hub.hub_set_propagate_path(B.handle, 1)
        x = _vecs(B.dim, 2, 95, torch.complex128)
        x[B.dim:] = 0
        st, obs, log = hub.hub_propagate(B.handle, _pulses(2), 0.0, 0.02, 6, hub.make_opts(tol=1e-12, m_max=30), x)
        assert torch.count_nonzero(x[B.dim:]).item() == 0
        assert np.all(obs[:, 1, 1:] == 0.0)
        assert (log[:, 1, 0] == 1).all() and (log[:, 1, 3] == 1).all()  # m = 1, invariant subspace
        assert np.allclose(obs[:, 0, 1], 1.0, atol=1e-12)
        # no steps: the observables of the input only, state unchanged
        y = _vecs(B.dim, 1, 96, torch.complex128)
        y0 = y.clone()
        st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.3, 0.02, 0, hub.make_opts(tol=1e-12, m_max=30), y)
        assert torch.equal(y, y0) and obs.shape == (1, 1, 4)
        hub.hub_set_propagate_path(B.handle, 0)
        st, obs0, _ = hub.hub_propagate(B.handle, [w.pulse], 0.3, 0.02, 0, hub.make_opts(tol=1e-12, m_max=30), y)
        assert np.max(np.abs(obs - obs0)) < 1e-13
    finally:
        B.close()


@pytest.mark.parametrize("nv,bad", [(1, np.nan), (3, np.inf)])
def test_resident_non_finite_input(nv, bad):
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    try:
        hub.hub_set_propagate_path(B.handle, 1)
        x = _vecs(B.dim, nv, 97, torch.complex128)
        x[(nv - 1) * B.dim + 17] = complex(bad, 0.0)
        with pytest.raises(hub.HubError) as e:
            hub.hub_propagate(B.handle, [w.pulse] * nv, 0.0, w.dt, 5, hub.make_opts(tol=1e-10, m_max=30), x)
        assert e.value.status == hub.HUB_E_INVALID and "non-finite" in str(e.value)
    finally:
        B.close()


def test_resident_single_exponential():
    """hub_krylov_expm_step takes the same path."""
    B = hub.Basis(ring(6), 4.0, 3, 3, device=0)
    try:
        x0 = _vecs(B.dim, 2, 98, torch.complex128)
        out = []
        for path in (0, 1):
            hub.hub_set_propagate_path(B.handle, path)
            v = x0.clone()
            hub.hub_krylov_expm_step(B.handle, [0.3, -0.7], 0.05, hub.make_opts(tol=1e-13, m_max=30), v)
            out.append(v)
        assert torch.linalg.norm(out[1] - out[0]).item() < 1e-12
    finally:
        B.close()


def test_resident_forced_path_checks():
    B = hub.Basis(ring(8), 8.0, 4, 4, device=0)
    big = hub.Basis(ring(10), 8.0, 5, 5, device=0)
    try:
        x = _vecs(B.dim, 1, 99, torch.complex128)
        hub.hub_set_propagate_path(B.handle, 1)
        with pytest.raises(hub.HubError) as e:
            hub.hub_propagate(B.handle, [PulseParams(0, 0.5, 8.0, 0.1, 0.3)], 0.0, 0.01, 2,
                              hub.make_opts(tol=1e-10, m_max=30, reorth=1), x.clone())
        assert e.value.status == hub.HUB_E_INVALID
        hub.hub_set_propagate_path(big.handle, 1)
        y = _vecs(big.dim, 1, 100, torch.complex128)
        with pytest.raises(hub.HubError) as e:
            hub.hub_propagate(big.handle, [PulseParams(0, 0.5, 8.0, 0.1, 0.3)], 0.0, 0.01, 2,
                              hub.make_opts(tol=1e-10, m_max=30), y)
        assert e.value.status == hub.HUB_E_INVALID and "does not fit" in str(e.value)
        for bad in (-2, 2):
            with pytest.raises(hub.HubError):
                hub.hub_set_propagate_path(B.handle, bad)
    finally:
        B.close()
        big.close()


@pytest.mark.parametrize("lat,nu,nd,dtype,nv,resident", [
    (ring(8), 4, 4, torch.complex128, 1, True),      # 4,900 states
    (ring(9), 3, 3, torch.complex128, 1, False),     # 7,056 states, one vector
    (ring(9), 3, 3, torch.complex128, 2, True),
    (ring(9), 3, 3, torch.complex64, 1, False),
    (ring(10), 5, 5, torch.complex128, 16, False),   # does not fit
])
def test_resident_automatic_choice(lat, nu, nd, dtype, nv, resident):
    B = hub.Basis(lat, 8.0, nu, nd, device=0)
    try:
        x = _vecs(B.dim, nv, 101, dtype)
        hub.hub_controller_read_stats(B.handle)
        hub.hub_propagate(B.handle, _pulses(nv), 0.0, 0.02, 3, hub.make_opts(tol=1e-10, m_max=30), x)
        s = hub.hub_controller_read_stats(B.handle)
        assert (s["lanczos_launches"] == 0) == resident, s
        # a forced apply path keeps the launch path
        hub.hub_set_apply_path(B.handle, 0)
        hub.hub_propagate(B.handle, _pulses(nv), 0.0, 0.02, 3, hub.make_opts(tol=1e-10, m_max=30), x)
        assert hub.hub_controller_read_stats(B.handle)["lanczos_launches"] > 0
    finally:
        B.close()
