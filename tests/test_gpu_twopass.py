"""Two-pass H*v (row pass + column pass) against the one-pass kernel and the
oracle, through the C ABI.

* plain applies: bit-identical to the one-pass kernel on ragged tiles, empty
  spins, unequal sectors, both precisions, and against the oracle's H;
* Lanczos propagation with the two-pass kernels matches the one-pass run to
  rounding (alpha is reduced in another order) and the exact oracle;
* the learned controller's schedule stays bit-identical on the two-pass path;
* the 12-site tile (automatic choice: two passes) agrees with the one-pass
  kernel over a few full Krylov steps.
"""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from paper_2005_13498_amd import controller as ctl
from synth import ring, chain, cluster_2d, random_state, workloads
from oracle import HubbardOracle, to_canonical, pulse_A, ground_state
from oracle.stepper import midpoint_step_exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    (ring(8), 8.0, 4, 4),        # 70 x 70
    (ring(5), 8.0, 2, 3),        # 10 x 10
    (ring(10), 8.0, 4, 5),       # 210 x 252
    (chain(7), 3.0, 3, 2),       # 35 x 21, open chain
    (ring(6), 4.0, 0, 3),        # no up electrons: 1 x 20
    (ring(6), 4.0, 3, 0),        # no down electrons
    (cluster_2d(2, 3), 8.0, 3, 3),
]


def _to_dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV).to(dtype)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("lat,U,nu,nd", CASES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_plain_apply_two_pass_bit_identical(lat, U, nu, nd, dtype):
    B = hub.Basis(lat, U, nu, nd, device=0)
    try:
        x = _to_dev(random_state(B.dim, seed=41, nvec=1)[0], dtype)
        outs = []
        for path in (0, 1):
            hub.hub_set_apply_path(B.handle, path)
            y = torch.empty_like(x)
            hub.hub_apply_H(B.handle, [0.43], x, y)
            outs.append(y)
        assert torch.equal(outs[0], outs[1])
        if dtype == torch.complex128:
            ham = HubbardOracle(lat, U, nu, nd)
            xr = x.cpu().numpy()
            from oracle import from_canonical
            xi = from_canonical(xr, ham.states, lat.n_sites)
            ref = to_canonical(ham.apply(0.43, xi), ham.states, lat.n_sites)
            assert _rel(outs[1].cpu().numpy(), ref) < 1e-13
    finally:
        B.close()


def test_lanczos_two_pass_matches_one_pass_and_oracle():
    w = workloads()["ring8"]
    ham = HubbardOracle(w.lattice, w.U, 4, 4)
    E0, _, g = ground_state(ham, pulse_A(w.pulse, 0.0))
    B = hub.Basis(w.lattice, w.U, 4, 4, device=0)
    try:
        n = 100
        opts = hub.make_opts(tol=1e-13, m_max=30)
        res = {}
        for path in (0, 1):
            hub.hub_set_apply_path(B.handle, path)
            x = _to_dev(to_canonical(g, ham.states, 8))
            st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.0, w.dt, n, opts, x)
            res[path] = (x.cpu().numpy(), obs, log)
        assert _rel(res[1][0], res[0][0]) < 1e-12
        assert np.max(np.abs(res[1][1] - res[0][1])) < 1e-12
        # the fused path ends most steps from the row pass's early estimate
        # (y^(m), eps recorded there, |u_m| and the status by the column pass):
        # the same step logs as the one-pass decision
        lg0, lg1 = res[0][2], res[1][2]
        assert np.array_equal(lg1[:, :, 0], lg0[:, :, 0])  # m
        assert np.array_equal(lg1[:, :, 2:4], lg0[:, :, 2:4])  # converged, breakdown
        assert np.allclose(lg1[:, :, 4], lg0[:, :, 4], rtol=0.05, atol=1e-16)  # eps (a difference of nearby vectors)
        assert np.allclose(lg1[:, :, 5], lg0[:, :, 5], rtol=1e-10)  # beta of the last vector
        v = g.copy()
        for k in range(n):
            v = midpoint_step_exact(ham, v, k * w.dt, w.dt, w.pulse)
        ref = to_canonical(v, ham.states, 8)
        assert _rel(res[1][0], ref) < 1e-10
    finally:
        B.close()


def test_controller_bit_identical_on_two_pass():
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, 4, 4, device=0)
    try:
        hub.hub_set_apply_path(B.handle, 1)
        x0 = _to_dev(random_state(B.dim, seed=42)[0])
        opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
        outs = []
        for params in (None, ctl.constant_params(3), ctl.constant_params(10)):
            x = x0.clone()
            if params is not None:
                hub.hub_controller_load(B.handle, params)
                hub.hub_controller_enable(B.handle, True, 8, 0)
            try:
                st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.0, w.dt, 80, opts, x)
            finally:
                hub.hub_controller_enable(B.handle, False)
            outs.append((x, obs, log))
        for x, obs, log in outs[1:]:
            assert torch.equal(x, outs[0][0])
            assert np.array_equal(obs, outs[0][1]) and np.array_equal(log, outs[0][2])
    finally:
        B.close()


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-5)])
def test_cluster3x4_two_pass_steps(dtype, tol):
    w = workloads()["cluster3x4"]
    B = hub.Basis(w.lattice, w.U, 6, 6, device=0)
    try:
        x0 = _to_dev(random_state(B.dim, seed=43)[0], dtype)
        opts = hub.make_opts(tol=1e-10, m_max=30)
        res = {}
        for path in (0, -1):  # -1 picks the two-pass kernels at this size
            hub.hub_set_apply_path(B.handle, path)
            x = x0.clone()
            st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 2.3, w.dt, 5, opts, x)
            res[path] = (x.cpu().numpy().astype(np.complex128), obs)
        assert _rel(res[-1][0], res[0][0]) < tol
        assert np.max(np.abs(res[-1][1] - res[0][1])) < tol
        # plain apply at full size: bit-identical
        ys = []
        for path in (0, 1):
            hub.hub_set_apply_path(B.handle, path)
            y = torch.empty_like(x0)
            hub.hub_apply_H(B.handle, [0.5], x0, y)
            ys.append(y)
        assert torch.equal(ys[0], ys[1])
    finally:
        B.close()


@pytest.mark.parametrize("m_max", [2, 3, 5])
def test_two_pass_stops_at_m_max_like_one_pass(m_max):
    """The decision-only launch at j = m_max (fused from j = 2 on) stops the
    step exactly as the one-pass kernels do."""
    lat = ring(8)
    B = hub.Basis(lat, 8.0, 4, 4, device=0)
    try:
        x0 = _to_dev(random_state(B.dim, seed=44)[0])
        res = {}
        for path in (0, 1):
            hub.hub_set_apply_path(B.handle, path)
            x = x0.clone()
            st, info = hub.hub_krylov_expm_step(B.handle, [0.3], 0.2, hub.make_opts(tol=1e-15, m_max=m_max), x,
                                                allow_not_converged=True)
            res[path] = (st, info, x.cpu().numpy())
        assert res[0][0] == res[1][0] == hub.HUB_E_NOT_CONVERGED
        assert res[0][1][0, 0] == res[1][1][0, 0] == m_max
        assert _rel(res[1][2], res[0][2]) < 1e-12
    finally:
        B.close()

