"""Learned Krylov controller, CPU side.

* the FP64 MLP oracle is pinned by closed forms (GELU values and symmetry,
  hand-built networks whose output is known), central finite differences of
  the loss, and the closed form of Adam's first step;
* the library's training-row builder (host code, no GPU) matches the
  oracle's features on a hand-made step log;
* the controller entry points reject bad arguments.
"""
import math

import numpy as np
import pytest

import paper_2005_13498_amd as hub
from oracle import mlp
from oracle.hamiltonian import pulse_A
from synth import PulseParams


def test_gelu_closed_forms():
    # gelu(z) = z Phi(z): Phi(0) = 1/2, Phi(1) = 0.8413447460685429 (normal table)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + (1.0 - 0.8413447460685429)) < 1e-15
    z = np.linspace(-6, 6, 49)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)   # Phi(z) + Phi(-z) = 1
    assert abs(mlp.gelu(40.0) - 40.0) < 1e-12 and abs(mlp.gelu(-40.0)) < 1e-12
    # derivative by central differences
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_prime(z), fd, atol=1e-8)


def test_forward_hand_built_networks():
    # all-zero weights: out = b3 whatever the input
    P = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    P["b3"] = np.array([2.5])
    X = np.random.default_rng(0).normal(size=(5, 8))
    out, _ = mlp.forward(mlp.pack(P), X)
    assert np.allclose(out, [[2.5]] * 5, atol=0)
    # two paths into the output: x[2] -> unit 5 (layer 1) -> unit 3 (layer 2) and
    # x[6] -> unit 7 -> unit 9
    P = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    P["W1"][5, 2] = 1.5
    P["W1"][7, 6] = -0.5
    P["b1"][5] = 0.25
    P["W2"][3, 5] = 2.0     # row = receiving unit, column = sending unit
    P["W2"][9, 7] = 1.0
    P["b2"][3] = -0.1
    P["W3"][0, 3] = 3.0
    P["W3"][0, 9] = -2.0
    P["b3"][:] = [0.5]
    x = np.zeros((1, 8))
    x[0, 2], x[0, 6] = 0.8, 1.2
    out, _ = mlp.forward(mlp.pack(P), x)
    h15 = mlp.gelu(1.5 * 0.8 + 0.25)
    h17 = mlp.gelu(-0.5 * 1.2)
    # units other than 5 and 7 carry gelu(0) = 0, so only the two paths contribute
    assert abs(out[0, 0] - (3.0 * mlp.gelu(2.0 * h15 - 0.1) - 2.0 * mlp.gelu(1.0 * h17) + 0.5)) < 1e-14


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = rng.normal(scale=0.3, size=mlp.N_PARAM)
    X = rng.normal(size=(7, 8))
    Y = rng.normal(size=(7, 1))
    L, g = mlp.loss_and_grad(theta, X, Y)
    assert abs(L - mlp.loss(theta, X, Y)) < 1e-14
    idx = np.concatenate([rng.choice(mlp.N_PARAM, 40, replace=False),
                          [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.N_PARAM)
        e[k] = h
        fd = (mlp.loss(theta + e, X, Y) - mlp.loss(theta - e, X, Y)) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * (1 + abs(fd)), (k, fd, g[k])


def test_adam_first_step_closed_form():
    # from m = v = 0 at t = 1 the bias-corrected step is -lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.ones(4), np.zeros(4), np.zeros(4), 1, 0.01, g)
    assert np.allclose(th, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the step at lr (bias corrections cancel the averages)
    th, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, t, 0.1, np.array([4.0]))
    assert abs(th[0] + 0.5) < 1e-8


def test_pulse_derivative():
    for p in (PulseParams(0, 0.7, 8.0, 2.5, 0.5), PulseParams(1, 0.4, 6.0, 1.0, 0.3, math.cos(0.2))):
        for t in (0.3, 1.1, 2.4, 2.9):
            h = 1e-6
            fd = (pulse_A(p, t + h) - pulse_A(p, t - h)) / (2 * h)
            assert abs(mlp.pulse_dA(p, t) - fd) < 1e-6 * (1 + abs(fd))


def _hand_log(n):
    m = [5, 6, 6, 7, 6, 5, 8, 6, 6, 7][:n]
    e = [3e-11, 1e-12, 4e-11, 0.0, 2e-13, 7e-11, 5e-12, 1e-11, 9e-12, 3e-14][:n]
    return m, e


def test_feature_rows_by_hand():
    p = PulseParams(0, 0.9, 8.0, 2.5, 0.5)
    m, e = _hand_log(10)
    X, Y = mlp.features(p, 0.25, 0.005, 88.0, 1e-10, 0, 1, m, e, chunk=4)
    # row 6: chunk [4, 8) planned after step 3 -> history h = 3, 2, 1, 0
    assert abs(X[6, 3] - math.log10(1e-40) / 10) < 1e-15          # eps_3 = 0 is floored
    assert abs(X[6, 4] - math.log10(4e-11) / 10) < 1e-15
    assert abs(X[6, 6] - math.log10(3e-11) / 10) < 1e-15
    assert abs(X[6, 7] - 0.7) < 1e-15 and abs(Y[6, 0] - 3.0) < 1e-15
    # row 1: planned before step 0 -> tol and the default 8
    assert np.allclose(X[1, 3:7], -1.0) and abs(X[1, 7] - 0.8) < 1e-15
    # row 2 of chunk 2 sees history 3.. only through h = 3
    assert abs(X[5, 7] - 0.7) < 1e-15
    assert abs(X[0, 2] - 0.44) < 1e-15


def test_library_feature_rows_match_oracle():
    p = PulseParams(0, 0.9, 8.0, 2.5, 0.5)
    m, e = _hand_log(10)
    log = np.zeros((10, 6))
    log[:, 0] = m
    log[:, 1] = 1
    log[:, 2] = 1
    log[:, 4] = e
    for chunk, m_hint in ((4, 0), (3, 5), (1, 0)):
        opts = hub.make_opts(tol=1e-10, m_max=30, m_hint=m_hint)
        F, T = hub.hub_controller_features(p, 0.25, 0.005, 88.0, opts, log, chunk)
        X, Y = mlp.features(p, 0.25, 0.005, 88.0, 1e-10, m_hint, 1, m, e, chunk)
        assert np.allclose(F, X.astype(np.float32), rtol=1e-6, atol=1e-7)
        assert np.allclose(T, Y.astype(np.float32), atol=1e-7)


def test_controller_argument_checks():
    from synth import ring
    h = hub.hub_basis_create(ring(4), 4.0, 2, 2, device=-1)
    try:
        with pytest.raises(hub.HubError) as e:
            hub.hub_controller_enable(h, True, 16, 1)        # nothing loaded
        assert e.value.status == hub.HUB_E_INVALID
        with pytest.raises(hub.HubError) as e:
            hub.hub_controller_load(h, np.zeros(hub.MLP_NPARAM))  # host-only handle
        assert e.value.status == hub.HUB_E_DEVICE
        with pytest.raises(hub.HubError):
            hub.hub_controller_load(h, np.zeros(10))
        hub.hub_controller_enable(h, False)
        assert hub.hub_controller_read_stats(h)["steps"] == 0
    finally:
        hub.hub_basis_destroy(h)
    assert hub.hub_mlp_workspace_bytes(1000) > 0
    assert hub.MLP_NPARAM == mlp.N_PARAM == 4801
