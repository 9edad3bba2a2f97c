"""Training driver of the learned Krylov controller (argument marshalling and
the Adam loop; every forward, gradient and update runs in libhub's kernels).

    rows = collect_rows(basis, pulses, ...)        # adaptive runs -> (X, Y)
    params, losses = train(X, Y, steps=600)        # hub_mlp_train_step loop
    hub_controller_load(basis.handle, params); hub_controller_enable(basis.handle, True)
"""
from __future__ import annotations

import numpy as np

from . import (MLP_HID, MLP_IN, MLP_NPARAM, MLP_OUT, hub_basis_classes, hub_controller_features,
               hub_mlp_train_step, hub_mlp_workspace_bytes, hub_propagate, make_opts)


def init_params(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters: weights N(0, 1/fan_in), zero biases, output
    bias log2 8 so an untrained controller predicts m = 8."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, 1 / np.sqrt(MLP_IN), MLP_HID * MLP_IN), np.zeros(MLP_HID),
             rng.normal(0, 1 / np.sqrt(MLP_HID), MLP_HID * MLP_HID), np.zeros(MLP_HID),
             rng.normal(0, 1 / np.sqrt(MLP_HID), MLP_OUT * MLP_HID), np.array([3.0])]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_NPARAM
    return p


def collect_rows(basis, v0, pulses, t_start: float, dt: float, n_steps: int, opts, chunk: int):
    """Propagate v0 (device tensor, left unchanged) under each pulse with the
    adaptive schedule and return the stacked training rows."""
    _, _, norm_inf = hub_basis_classes(basis.handle)
    X, Y = [], []
    for p in pulses:
        v = v0.clone()
        _, _, log = hub_propagate(basis.handle, [p], t_start, dt, n_steps, opts, v, want_obs=False)
        f, t = hub_controller_features(p, t_start, dt, norm_inf, opts, log[:, 0, :], chunk)
        X.append(f)
        Y.append(t)
    return np.concatenate(X), np.concatenate(Y)


def train(X: np.ndarray, Y: np.ndarray, steps: int = 600, lr: float = 3e-3, seed: int = 0, device: int = 0,
          params: np.ndarray | None = None, report_every: int = 50):
    """Full-batch Adam on the rows; returns (params, [(step, loss), ...])."""
    import torch

    dev = f"cuda:{device}"
    P = torch.tensor(init_params(seed) if params is None else np.asarray(params, np.float32), device=dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xd = torch.tensor(np.ascontiguousarray(X, np.float32), device=dev)
    Yd = torch.tensor(np.ascontiguousarray(Y, np.float32), device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(max(1, hub_mlp_workspace_bytes(len(X)) // 4), dtype=torch.float32, device=dev)
    hist = []
    for t in range(1, steps + 1):
        hub_mlp_train_step(P, m, v, t, lr, Xd, Yd, loss, ws)
        if t == 1 or t % report_every == 0 or t == steps:
            hist.append((t, float(loss.item())))
    return P.cpu().numpy(), hist


def constant_params(m: float) -> np.ndarray:
    """Parameters of a controller that always predicts Krylov dimension m."""
    p = np.zeros(MLP_NPARAM, dtype=np.float32)
    p[-1] = np.log2(m)
    return p


def group_runs(hub_mod, lattice, n_up: int, n_dn: int, groups, t0: float, sigma: float, dt: float, n_steps: int,
               tol: float, chunk: int, device: int = 0):
    """Adaptive runs of every (U, members) group from the ground state of
    H(A = 0) at that U: one hub_propagate call per group, the members'
    pulses A0 sin(omega (t - t0)) exp(-(t - t0)^2 / 2 sigma^2).  Returns the
    training rows (X, Y) of every member and step."""
    import torch

    X, Y = [], []
    opts = make_opts(tol=tol, m_max=30)
    for U, mem in groups:
        B = hub_mod.Basis(lattice, U, n_up, n_dn, device=device)
        try:
            g = torch.empty(B.dim, dtype=torch.complex128, device=f"cuda:{device}")
            hub_mod.hub_ground_state(B.handle, 0.0, g, make_opts(tol=1e-10, m_max=60), allow_degenerate=True)
            pulses = [(0, a0, om, t0, sigma, 0.0) for a0, om in mem]
            v = g.repeat(len(pulses)).contiguous()
            _, _, log = hub_propagate(B.handle, pulses, 0.0, dt, n_steps, opts, v, want_obs=False)
            _, _, norm_inf = hub_basis_classes(B.handle)
            for k, p in enumerate(pulses):
                f, t = hub_controller_features(p, 0.0, dt, norm_inf, opts, log[:, k, :], chunk)
                X.append(f)
                Y.append(t)
            del v, g
        finally:
            B.close()
    return np.concatenate(X), np.concatenate(Y)
