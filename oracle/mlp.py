"""FP64 reference of the learned Krylov controller (not in the paper).

TEST INFRASTRUCTURE ONLY (see the package header).

The controller is a plain multilayer perceptron 8 -> 64 -> 64 -> 1 with the
exact (erf) GELU on both hidden layers and a linear output, trained by Adam
on the mean squared error.  Written from the textbook definitions:

    h1 = gelu(W1 x + b1),  h2 = gelu(W2 h1 + b2),  out = W3 h2 + b3
    gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
    L = (1/N) sum_r |out_r - y_r|^2
    Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
        theta <- theta - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Parameters are one flat vector: W1[64][8], b1[64], W2[64][64], b2[64],
W3[1][64], b3[1] (row-major, output unit first).  The output is log2 of the
Krylov dimension of a step.

Features of a step n whose history ends at step h (the last finished step
when n was planned): the vector potential at the step's midpoint and its time
derivative / 10, tau |H|_inf, log10 of the a-posteriori estimates of steps
h, h-1, h-2, h-3 over 10 (floored at 1e-40; log10(tol)/10 before step 0),
and m_h / 10 (m_hint / 10, or 0.8, before step 0).  For training rows the
planning points are the multiples of the chunk length: h = n - 1 - (n mod chunk).
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID, N_OUT = 8, 64, 1
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)

_erf = np.vectorize(math.erf, otypes=[float])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAM
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[k:k + n].reshape(shp)
        k += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X):
    """X [N, 8] -> out [N, 2] (and the intermediate values)."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    out = h2 @ P["W3"].T + P["b3"]
    return out, (X, z1, h1, z2, h2)


def loss(theta, X, Y) -> float:
    out, _ = forward(theta, X)
    return float(np.sum((out - np.asarray(Y, dtype=np.float64)) ** 2) / len(X))


def loss_and_grad(theta, X, Y):
    """L and dL/dtheta (same flat layout) by backpropagation."""
    P = unpack(theta)
    out, (X, z1, h1, z2, h2) = forward(theta, X)
    N = len(X)
    d_out = 2.0 * (out - np.asarray(Y, dtype=np.float64)) / N      # [N, 2]
    g = {"W3": d_out.T @ h2, "b3": d_out.sum(axis=0)}
    d_z2 = (d_out @ P["W3"]) * gelu_prime(z2)                      # [N, 64]
    g["W2"] = d_z2.T @ h1
    g["b2"] = d_z2.sum(axis=0)
    d_z1 = (d_z2 @ P["W2"]) * gelu_prime(z1)
    g["W1"] = d_z1.T @ X
    g["b1"] = d_z1.sum(axis=0)
    L = float(np.sum((out - Y) ** 2) / N)
    return L, pack(g)


def adam_step(theta, m, v, t: int, lr: float, grad, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def pulse_dA(pulse, t: float) -> float:
    """Time derivative of oracle.hamiltonian.pulse_A (analytic)."""
    kind, A0, omega, t0, sigma, b = pulse.as_tuple() if hasattr(pulse, "as_tuple") else pulse
    s = t - t0
    env = math.exp(-s * s / (2.0 * sigma * sigma))
    denv = -s / (sigma * sigma) * env
    if int(kind) == 0:
        return A0 * (denv * math.sin(omega * s) + env * omega * math.cos(omega * s))
    return A0 * (denv * (math.cos(omega * s) - b) - env * omega * math.sin(omega * s))


def features(pulse, t_start: float, dt: float, norm_inf: float, tol: float, m_hint: int, substeps: int,
             m_used, err_est, chunk: int):
    """Training rows (X [n, 8], Y [n, 1]) of one vector's finished run."""
    from .hamiltonian import pulse_A
    n_steps = len(m_used)
    X = np.zeros((n_steps, N_IN))
    Y = np.zeros((n_steps, N_OUT))
    for n in range(n_steps):
        h = n - 1 - (n % chunk)
        tm = t_start + (n + 0.5) * dt
        X[n, 0] = pulse_A(pulse, tm)
        X[n, 1] = pulse_dA(pulse, tm) / 10.0
        X[n, 2] = dt / substeps * norm_inf
        for q in range(4):
            e = err_est[h - q] if h - q >= 0 else None
            X[n, 3 + q] = (math.log10(tol) if e is None else math.log10(max(e, 1e-40))) / 10.0
        X[n, 7] = (m_used[h] if h >= 0 else (m_hint if m_hint > 0 else 8)) / 10.0
        Y[n, 0] = math.log2(max(1, m_used[n]))
    return X, Y
