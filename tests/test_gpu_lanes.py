"""Groups of vectors of one hub_propagate call run on concurrent lanes (each
with its own workspace and stream): results must equal propagating each
group on its own, bit for bit, and errors and counters must come back.

* 12-site cluster: single-vector groups (two-pass kernels), 4 and 5 members;
* 8-site ring: interleaved groups of 8 and 4 (12 members);
* complex64 and the fourth-order scheme;
* a lane that hits m_max reports HUB_E_NOT_CONVERGED.
"""
import numpy as np
import pytest
import torch

import paper_2005_13498_amd as hub
from synth import workloads, random_state, PulseParams

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _members(B, k, seed, dtype):
    x = np.stack(random_state(B.dim, seed=seed, nvec=k))
    return torch.from_numpy(x.reshape(-1)).to(DEV).to(dtype).contiguous()


def _pulses(k):
    return [PulseParams(0, 0.3 + 0.1 * i, 8.0, 0.05, 0.3) for i in range(k)]


def _check_split(B, pulses, x0, dt, n, opts, splits):
    """One call with all members vs one call per split (consecutive members)."""
    dim = B.dim
    xa = x0.clone()
    st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, dt, n, opts, xa)
    k = 0
    for size in splits:
        xb = x0[k * dim:(k + size) * dim].clone()
        st2, o2, l2 = hub.hub_propagate(B.handle, pulses[k:k + size], 0.0, dt, n, opts, xb)
        assert torch.equal(xa[k * dim:(k + size) * dim], xb)
        assert np.array_equal(obs[:, k:k + size], o2, equal_nan=True)
        assert np.array_equal(log[:, k:k + size], l2)
        k += size


@pytest.mark.parametrize("k", [4, 5])
def test_cluster3x4_single_vector_groups(k):
    w = workloads()["cluster3x4"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x0 = _members(B, k, 71, torch.complex128)
        hub.hub_controller_read_stats(B.handle)
        _check_split(B, _pulses(k), x0, w.dt, 12, hub.make_opts(tol=w.tol, m_max=w.m_max), [1] * k)
        assert hub.hub_controller_read_stats(B.handle)["chunks"] > 0
    finally:
        B.close()


@pytest.mark.parametrize("dtype,scheme", [(torch.complex128, 0), (torch.complex64, 0), (torch.complex128, 1)])
def test_ring8_interleaved_groups(dtype, scheme):
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x0 = _members(B, 12, 72, dtype)
        opts = hub.make_opts(tol=w.tol, m_max=w.m_max, scheme=scheme)
        _check_split(B, _pulses(12), x0, w.dt, 40, opts, [8, 4])
    finally:
        B.close()


def test_lane_not_converged_is_reported():
    w = workloads()["cluster3x4"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x0 = _members(B, 3, 73, torch.complex128)
        st, obs, log = hub.hub_propagate(B.handle, _pulses(3), 0.0, 0.05, 3, hub.make_opts(tol=1e-15, m_max=3), x0,
                                         allow_not_converged=True)
        assert st == hub.HUB_E_NOT_CONVERGED
        assert (log[0, :, 0] == 3).all()
    finally:
        B.close()
