"""Kernel plan tuning through the C ABI: hub_tune measures and installs a
plan, hub_get_plan reports it, hub_set_tuning installs a cached one or the
built-in rules; results under every plan match the oracle."""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import ring, workloads, random_state, PulseParams
from oracle import HubbardOracle, to_canonical, from_canonical, midpoint_step_exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", [hub.HUB_C128, hub.HUB_C64])
def test_tune_installs_a_measured_plan(prec):
    w = workloads()["cluster3x4"]
    B = hub.Basis(w.lattice, w.U, 6, 6)
    try:
        t = hub.hub_tune(B.handle, prec, 3)
        assert t["prop_group"] in (1, 2, 4, 8) and t["apply_group"] in (1, 2, 4, 8)
        assert t["single_two_pass"] in (0, 1)
        us = np.array(t["apply_us"])
        assert (us >= 0).all() and us[0, 0] > 0 and us[0, 1] > 0  # both single-vector paths fit at 12 sites
        assert np.array(t["step_us"])[0] > 0
        # 32 vectors fit at 12 sites for every feasible group size
        assert t["prop_group_large"] in (1, 2, 4, 8)
        assert t["step_us_large"][{1: 0, 2: 1, 4: 2, 8: 3}[t["prop_group_large"]]] > 0
        assert all((a > 0) == (b > 0) for a, b in zip(t["step_us"], t["step_us_large"]))
        # the installed plan is what the library reports
        plan = hub.hub_get_plan(B.handle, prec, 8, True)
        assert sum(g for g, _ in plan) == 8 and max(g for g, _ in plan) == t["prop_group"]
        plan_l = hub.hub_get_plan(B.handle, prec, 32, True)
        assert sum(g for g, _ in plan_l) == 32 and max(g for g, _ in plan_l) == t["prop_group_large"]
        plan_a = hub.hub_get_plan(B.handle, prec, 8, False)
        assert max(g for g, _ in plan_a) == t["apply_group"]
        # a cached table installs the same plan; None restores the built-in rules
        hub.hub_set_tuning(B.handle, prec, None)
        hub.hub_set_tuning(B.handle, prec, t)
        assert hub.hub_get_plan(B.handle, prec, 8, True) == plan
        with pytest.raises(hub.HubError):
            hub.hub_set_tuning(B.handle, prec, dict(t, prop_group=3))
        with pytest.raises(hub.HubError):
            hub.hub_set_tuning(B.handle, prec, dict(t, prop_group_large=6))
    finally:
        B.close()


def test_large_batches_take_their_own_group_size():
    """A plan's prop_group serves hub_propagate calls of up to 8 vectors,
    prop_group_large larger ones (the groups then fill the concurrent
    lanes); a plan without the large entry uses prop_group for both."""
    w = workloads()["ring8"]
    B = hub.Basis(w.lattice, w.U, 4, 4)
    try:
        plan = {"single_two_pass": 0, "block_two_pass": [0, 1, 1, 1], "apply_group": 8, "prop_group": 2,
                "prop_group_large": 8}
        hub.hub_set_tuning(B.handle, hub.HUB_C64, plan)
        assert [g for g, _ in hub.hub_get_plan(B.handle, hub.HUB_C64, 8, True)] == [2] * 4
        assert [g for g, _ in hub.hub_get_plan(B.handle, hub.HUB_C64, 9, True)] == [8, 1]
        assert [g for g, _ in hub.hub_get_plan(B.handle, hub.HUB_C64, 64, True)] == [8] * 8
        old = {k: v for k, v in plan.items() if k != "prop_group_large"}
        hub.hub_set_tuning(B.handle, hub.HUB_C64, old)
        assert [g for g, _ in hub.hub_get_plan(B.handle, hub.HUB_C64, 64, True)] == [2] * 32
    finally:
        B.close()


@pytest.mark.parametrize("group,block", [(1, 0), (1, 1), (2, 0), (2, 1), (4, 1), (8, 0), (8, 1)])
def test_every_plan_matches_oracle(group, block):
    """8-site ring, 8 members, 20 midpoint steps under each forced plan
    (group size, block kernels on or off): states within 1e-10 of the exact
    stepper."""
    w = workloads()["ring8"]
    ham = HubbardOracle(w.lattice, w.U, 4, 4)
    B = hub.Basis(w.lattice, w.U, 4, 4)
    hub.hub_set_propagate_path(B.handle, 0)  # plans are the launch path's (the resident stepper has none)
    try:
        plan = {"single_two_pass": 1, "block_two_pass": [0, block, block, block], "apply_group": group,
                "prop_group": group}
        hub.hub_set_tuning(B.handle, hub.HUB_C128, plan)
        got_plan = hub.hub_get_plan(B.handle, hub.HUB_C128, 8, True)
        assert all(g == group for g, _ in got_plan)
        if group > 1:
            assert all(k == (2 if block else 0) for _, k in got_plan)
        pulses = [PulseParams(0, 0.1 * (k + 1), 8.0, 0.1, 0.1) for k in range(8)]
        xs = random_state(ham.dim, seed=3, nvec=8)
        x = torch.from_numpy(np.concatenate([to_canonical(v, ham.states, 8) for v in xs])).to(DEV)
        n, dt = 20, 0.01
        hub.hub_propagate(B.handle, pulses, 0.0, dt, n, hub.make_opts(tol=1e-13, m_max=30), x, want_obs=False)
        got = x.cpu().numpy().reshape(8, -1)
        for k in (0, 5):
            v = xs[k]
            for s in range(n):
                v = midpoint_step_exact(ham, v, s * dt, dt, pulses[k])
            assert _rel(from_canonical(got[k], ham.states, 8), v) < 1e-10
    finally:
        B.close()


def test_tuned_group_shrinks_where_no_kernel_fits():
    """14 sites, complex64: a plan asking for groups of 8 gets groups of 4,
    the largest block whose tile row fits LDS (the one-pass kernel cannot
    stage 8 vectors of a 3,432-element row either); a block of 4 propagates
    with observables at every sample time, the last row taken one vector
    at a time."""
    from synth import ring
    B = hub.Basis(ring(14), 8.0, 7, 7)
    try:
        hub.hub_set_tuning(B.handle, hub.HUB_C64, {"single_two_pass": 1, "block_two_pass": [0, 1, 1, 1],
                                                   "apply_group": 8, "prop_group": 8})
        assert hub.hub_get_plan(B.handle, hub.HUB_C64, 8, True) == [(4, 2), (4, 2)]
        g = torch.Generator(device=DEV).manual_seed(7)
        v0 = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
        v0 /= torch.linalg.vector_norm(v0)
        x = v0.to(torch.complex64).repeat(4).contiguous()
        pulses = [PulseParams(0, a, 8.0, 0.01, 0.02) for a in (0.3, 0.6, 0.9, 1.2)]
        st, obs, log = hub.hub_propagate(B.handle, pulses, 0.0, 0.01, 2, hub.make_opts(tol=1e-8, m_max=30), x)
        o1, _ = hub.hub_observables(B.handle, [hub.hub_pulse_A(p, 0.02) for p in pulses], x)
        assert np.max(np.abs(obs[-1, :, 1:] - o1[:, 1:])) < 1e-6
        assert np.max(np.abs(obs[:, :, 1] - 1.0)) < 1e-5
    finally:
        B.close()
        torch.cuda.empty_cache()
