"""Two-pass block kernels (blocks of 2, 4 or 8 vectors interleaved per tile
element) against the oracle and against the one-pass block kernel.

* H x of every block size in both precisions on lattices with ragged tiles,
  open chains, on-site energies and the 12-site cluster: complex128 within
  1e-13 relative of the oracle's sparse H, complex64 within 1e-5;
* the same products from the one-pass kernel (apply path 0) agree;
* midpoint propagations of several pulses in one call (Lanczos iterations
  with the block epilogue and the step's observables in the first apply)
  against the exact-exponential stepper, per member: psi, d(t), E(t) within
  1e-10 (complex128) and 1e-5 (complex64).
"""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import ring, chain, cluster_2d, random_state, PulseParams, workloads
from oracle import HubbardOracle, to_canonical, from_canonical, pulse_A, observables, midpoint_step_exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    (ring(8), 8.0, 4, 4),
    (ring(10), 8.0, 5, 4),
    (chain(7).with_onsite([0.3, -0.2, 0.0, 0.5, 0.1, -0.4, 0.2]), 3.0, 3, 4),
    (cluster_2d(3, 4), 8.0, 3, 2),
    (ring(6), 4.0, 3, 3),
]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("lat,U,nu,nd", CASES)
@pytest.mark.parametrize("dtype,bar", [(torch.complex128, 1e-13), (torch.complex64, 1e-5)])
def test_block_apply_matches_oracle(lat, U, nu, nd, dtype, bar):
    ham = HubbardOracle(lat, U, nu, nd)
    B = hub.Basis(lat, U, nu, nd)
    try:
        n = lat.n_sites
        for nvec in (2, 4, 8, 7):  # 7 = groups of 4, 2 and 1
            xs = random_state(ham.dim, seed=40 + nvec, nvec=nvec)
            As = list(np.linspace(-1.3, 0.9, nvec))
            xc = np.stack([to_canonical(x, ham.states, n) for x in xs])
            ref = np.stack([to_canonical(ham.apply(A, x), ham.states, n) for A, x in zip(As, xs)])
            x = torch.from_numpy(xc.ravel()).to(DEV).to(dtype)
            got = {}
            for path in (-1, 0):
                hub.hub_set_apply_path(B.handle, path)
                y = torch.empty_like(x)
                hub.hub_apply_H(B.handle, As, x, y)
                got[path] = y.to(torch.complex128).cpu().numpy().reshape(nvec, -1)
            for k in range(nvec):
                assert _rel(got[-1][k], ref[k]) < bar, (nvec, k)
                assert _rel(got[0][k], ref[k]) < bar, (nvec, k)
    finally:
        hub.hub_set_apply_path(B.handle, -1)
        B.close()


def test_block_apply_cluster3x4_full_size():
    """12 sites, 6/6: a block of 8 in both precisions against the oracle."""
    w = workloads()["cluster3x4"]
    ham = HubbardOracle(w.lattice, w.U, 6, 6)
    B = hub.Basis(w.lattice, w.U, 6, 6)
    try:
        xs = random_state(ham.dim, seed=9, nvec=8)
        As = [0.1 * k - 0.3 for k in range(8)]
        ref = [to_canonical(ham.apply(A, x), ham.states, 12) for A, x in zip(As, xs)]
        xc = np.concatenate([to_canonical(x, ham.states, 12) for x in xs])
        for dtype, bar in ((torch.complex128, 1e-13), (torch.complex64, 1e-5)):
            x = torch.from_numpy(xc).to(DEV).to(dtype)
            y = torch.empty_like(x)
            hub.hub_apply_H(B.handle, As, x, y)
            got = y.to(torch.complex128).cpu().numpy().reshape(8, -1)
            for k in range(8):
                assert _rel(got[k], ref[k]) < bar
    finally:
        B.close()


@pytest.mark.parametrize("dtype,bar", [(torch.complex128, 1e-10), (torch.complex64, 1e-5)])
def test_block_propagation_matches_exact(dtype, bar):
    """8-site ring, 8 members (pulse amplitudes 0.1 .. 0.8), 40 midpoint
    steps of 0.01 from seeded states, on the launch path (a block of 8 on
    the two-pass block kernels with fused iterations; the automatic choice
    would take the resident stepper at this size)."""
    w = workloads()["ring8"]
    ham = HubbardOracle(w.lattice, w.U, 4, 4)
    B = hub.Basis(w.lattice, w.U, 4, 4)
    hub.hub_set_propagate_path(B.handle, 0)
    try:
        plan = hub.hub_get_plan(B.handle, hub.HUB_C128 if dtype == torch.complex128 else hub.HUB_C64, 8, True)
        assert plan == [(8, 2)]
        nvec, n, dt = 8, 40, 0.01
        pulses = [PulseParams(0, 0.1 * (k + 1), 8.0, 0.2, 0.15) for k in range(nvec)]
        xs = random_state(ham.dim, seed=5, nvec=nvec)
        x = torch.from_numpy(np.concatenate([to_canonical(v, ham.states, 8) for v in xs])).to(DEV).to(dtype)
        tol = 1e-13 if dtype == torch.complex128 else 1e-8
        st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, dt, n, hub.make_opts(tol=tol, m_max=30), x)
        got = x.to(torch.complex128).cpu().numpy().reshape(nvec, -1)
        for k in (0, 3, 7):
            v = xs[k].copy()
            ref_obs = []
            for s in range(n):
                _, e, d, _ = observables(ham, v, pulse_A(pulses[k], s * dt))
                ref_obs.append((e, d))
                v = midpoint_step_exact(ham, v, s * dt, dt, pulses[k])
            _, e, d, _ = observables(ham, v, pulse_A(pulses[k], n * dt))
            ref_obs.append((e, d))
            r = np.array(ref_obs)
            assert _rel(from_canonical(got[k], ham.states, 8), v) < (bar if dtype == torch.complex128 else 1e-4)
            assert np.max(np.abs(obs[:, k, 2] - r[:, 0])) < bar * max(1.0, np.max(np.abs(r[:, 0])))
            assert np.max(np.abs(obs[:, k, 3] - r[:, 1])) < bar
        assert (log[:, :, 2] == 1).all()
    finally:
        B.close()


def _block_plan(group):
    return {"single_two_pass": 1, "block_two_pass": [0, 1, 1, 1], "apply_group": group, "prop_group": group}


def test_block_propagation_cluster3x4_c64_vs_c128():
    """12 sites: 8 members in complex64 as one block on the two-pass block
    kernels (forced plan) against complex128 single vectors of the same
    pulses, 6 steps in the pulse."""
    w = workloads()["cluster3x4"]
    B = hub.Basis(w.lattice, w.U, 6, 6)
    try:
        pulses = [PulseParams(0, a, 8.0, 0.05, 0.05) for a in w.extra["A0_batch"]]
        g = torch.Generator(device=DEV).manual_seed(3)
        v0 = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
        v0 /= torch.linalg.vector_norm(v0)
        blk = v0.to(torch.complex64).repeat(8).contiguous()
        n = 6
        hub.hub_set_tuning(B.handle, hub.HUB_C64, _block_plan(8))
        assert hub.hub_get_plan(B.handle, hub.HUB_C64, 8, True) == [(8, 2)]
        st, o64, _ = hub.hub_propagate(B.handle, pulses, 0.0, w.dt, n, hub.make_opts(tol=1e-8, m_max=30), blk)
        for k in (0, 4, 7):
            v = v0.clone()
            st, o128, _ = hub.hub_propagate(B.handle, [pulses[k]], 0.0, w.dt, n, hub.make_opts(tol=1e-12, m_max=30), v)
            got = blk[k * B.dim:(k + 1) * B.dim].to(torch.complex128)
            assert float(torch.linalg.vector_norm(got - v)) < 2e-5
            assert np.max(np.abs(o64[:, k, 2:] - o128[:, 0, 2:])) < 1e-5
    finally:
        B.close()


def test_block_propagation_ring14_c64_vs_c128():
    """14 sites (dim 11,778,624): 4 members in complex64 as one block of 4 on
    the two-pass block kernels (the plan the tuner picks there) against
    complex128 single vectors, 3 steps in the pulse."""
    w = workloads()["ring14_block"]
    B = hub.Basis(w.lattice, w.U, 7, 7)
    try:
        pulses = [PulseParams(0, a, w.pulse.omega, 0.02, 0.03) for a in (0.2, 0.5, 0.8, 1.1)]
        g = torch.Generator(device=DEV).manual_seed(4)
        v0 = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
        v0 /= torch.linalg.vector_norm(v0)
        blk = v0.to(torch.complex64).repeat(4).contiguous()
        n = 3
        hub.hub_set_tuning(B.handle, hub.HUB_C64, _block_plan(4))
        assert hub.hub_get_plan(B.handle, hub.HUB_C64, 4, True) == [(4, 2)]
        st, o64, _ = hub.hub_propagate(B.handle, pulses, 0.0, w.dt, n, hub.make_opts(tol=1e-8, m_max=30), blk)
        for k in (0, 3):
            v = v0.clone()
            st, o128, _ = hub.hub_propagate(B.handle, [pulses[k]], 0.0, w.dt, n, hub.make_opts(tol=1e-12, m_max=30), v)
            got = blk[k * B.dim:(k + 1) * B.dim].to(torch.complex128)
            assert float(torch.linalg.vector_norm(got - v)) < 2e-5
            assert np.max(np.abs(o64[:, k, 2:] - o128[:, 0, 2:])) < 1e-5
            del v, got
    finally:
        B.close()
        torch.cuda.empty_cache()
