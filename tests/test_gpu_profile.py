"""Kernel timing of the H*v launches (hub_profile_enable / hub_profile_read)
through the C ABI: every sampled launch is counted once, launches enqueued
past a step's Krylov decision are left out, and the event pool survives runs
longer than its size."""
import numpy as np
import pytest
import torch

import paper_2005_13498_amd as hub
from synth import workloads, random_state, ring

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _vec(B, seed):
    return torch.from_numpy(random_state(B.dim, seed=seed, nvec=1)[0]).to(DEV)


def test_plain_applies_are_all_timed():
    B = hub.Basis(ring(8), 8.0, 4, 4, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x = _vec(B, 61)
        y = torch.empty_like(x)
        hub.hub_profile_enable(B.handle, 1)
        hub.hub_profile_read(B.handle)
        for _ in range(1500):  # more samples than the pool holds: events are created on demand
            hub.hub_apply_H(B.handle, [0.2], x, y)
        n, ms, bpl = hub.hub_profile_read(B.handle)
        assert n == 1500 and ms > 0 and bpl == 2 * B.dim * 16
        n, ms, _ = hub.hub_profile_read(B.handle)
        assert n == 0 and ms == 0
        hub.hub_profile_enable(B.handle, 3)
        for _ in range(9):
            hub.hub_apply_H(B.handle, [0.2], x, y)
        assert hub.hub_profile_read(B.handle)[0] == 3
    finally:
        hub.hub_profile_enable(B.handle, 0)
        B.close()


@pytest.mark.parametrize("name,chunk", [("ring8", 16), ("ring8", 0), ("cluster3x4", 16), ("cluster3x4", 0)])
def test_propagation_counts_only_launches_that_work(name, chunk):
    """Every eligible launch sampled (period 1): iterations j = 1..m of each
    step (j = 0 records observables, another kernel), none of the speculative
    ones past the decision; on the fused two-pass path (12 sites) j = 1..m-1,
    since the column pass of j = m skips its apply."""
    w = workloads()[name]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x = _vec(B, 62)
        opts = hub.make_opts(tol=w.tol, m_max=w.m_max)
        hub.hub_set_schedule(B.handle, chunk, 1)
        hub.hub_profile_enable(B.handle, 1)
        hub.hub_profile_read(B.handle)
        hub.hub_controller_read_stats(B.handle)
        n_steps = 300
        st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.0, w.dt, n_steps, opts, x)
        n, ms, bpl = hub.hub_profile_read(B.handle)
        stats = hub.hub_controller_read_stats(B.handle)
        m = log[:, 0, 0].astype(int)
        assert stats["fallbacks"] == 0
        fused = name == "cluster3x4"
        assert n == int(m.sum()) - (n_steps if fused else 0), (n, int(m.sum()))
        if chunk:
            assert stats["lanczos_launches"] > n_steps + n  # speculative launches were enqueued
        assert ms > 0
    finally:
        hub.hub_profile_enable(B.handle, 0)
        hub.hub_set_schedule(B.handle, 32, 1)
        B.close()


def test_propagation_with_fallbacks():
    """Abandoned chunk steps: the launches after the device stopped are left
    out; those of the stopped step that ran before it are counted (they did
    the work, which the re-run repeats)."""
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, w.n_up, w.n_dn, device=0)
    hub.hub_set_propagate_path(B.handle, 0)  # the launch path's own mechanics
    try:
        x = _vec(B, 63)
        opts = hub.make_opts(tol=1e-14, m_max=40, m_hint=2)
        hub.hub_set_schedule(B.handle, 8, 0)
        hub.hub_profile_enable(B.handle, 1)
        hub.hub_profile_read(B.handle)
        hub.hub_controller_read_stats(B.handle)
        st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.0, 0.05, 60, opts, x)
        n, ms, _ = hub.hub_profile_read(B.handle)
        stats = hub.hub_controller_read_stats(B.handle)
        m = log[:, 0, 0].astype(int)
        assert stats["fallbacks"] >= 1
        # at most L - 1 <= m - 1 counted launches per abandoned attempt
        assert int(m.sum()) <= n <= int(m.sum()) + stats["fallbacks"] * int(m.max())
        assert n < stats["lanczos_launches"]
    finally:
        hub.hub_profile_enable(B.handle, 0)
        hub.hub_set_schedule(B.handle, 32, 1)
        B.close()
