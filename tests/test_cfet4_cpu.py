"""Fourth-order commutator-free exponential integrator (NEXT-2), oracle pins:
* without a field both factors are exp(-i dt/2 H), so a step is exp(-i dt H);
* with a strong pulse the global error falls as dt^4 (the midpoint rule's as
  dt^2), against a converged fine-step reference."""
import math

import numpy as np

from oracle import HubbardOracle
from oracle.stepper import cfet4_step_exact, midpoint_step_exact, expm_apply
from synth import chain, ring, random_state, PulseParams


def test_no_field_is_the_exact_exponential():
    h = HubbardOracle(ring(6), 4.0, 3, 3)
    v = random_state(h.dim, seed=3)[0]
    p = PulseParams(0, 0.0, 5.0, 1.0, 0.3)
    got = cfet4_step_exact(h, v, 0.3, 0.2, p)
    ref = expm_apply(h.H(0.0), v, 0.2)
    assert np.linalg.norm(got - ref) < 1e-13


def _run(step, h, v, t0, T, n, p):
    dt = T / n
    x = v.copy()
    for k in range(n):
        x = step(h, x, t0 + k * dt, dt, p)
    return x


def test_fourth_order_convergence_under_a_pulse():
    h = HubbardOracle(chain(5), 4.0, 2, 2)
    v = random_state(h.dim, seed=4)[0]
    p = PulseParams(0, 1.2, 6.0, 0.6, 0.3)
    t0, T = 0.2, 0.8
    ref = _run(cfet4_step_exact, h, v, t0, T, 256, p)
    e = [np.linalg.norm(_run(cfet4_step_exact, h, v, t0, T, n, p) - ref) for n in (8, 16)]
    slope = math.log2(e[0] / e[1])
    assert 3.5 < slope < 4.6, (e, slope)
    m = [np.linalg.norm(_run(midpoint_step_exact, h, v, t0, T, n, p) - ref) for n in (8, 16)]
    assert 1.7 < math.log2(m[0] / m[1]) < 2.4
    assert e[1] < m[1] / 10
