"""Krylov-subspace time step with the a-posteriori stopping rule (Alg. 6).

Sec. 3.4: exp(-i tau H) v is approximated by beta V exp(-i tau h) e_1, where
V is an orthonormal (Lanczos) basis of the Krylov space K_m(H, v), h = V^dag H V
is tridiagonal, and beta = |v|.  The dimension m grows until the estimate of
Hochbruck-Lubich-Selhofer (cited as [posteriori]) built from two consecutive
small-exponential vectors y^(j-1), y^(j) falls below tol, or the new
off-diagonal element falls below |H| tol (an invariant subspace was found).

Readings (the printed algorithm leaves these open):
  * |H| is the maximum absolute row sum, which the Peierls phases leave
    unchanged over time;
  * when the loop reaches N_max without meeting the stopping rule the result
    built from N_max vectors is returned, flagged as not converged;
  * no reorthogonalisation (none is printed);
  * y^(j-1) is padded with a zero to length j for the difference.

The small exponential is scipy.linalg.expm of the j x j matrix, a library
stand-in for Expokit.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def tridiag_expm_e1(alpha, beta, tau: float) -> np.ndarray:
    """exp(-i tau T) e_1 for the symmetric tridiagonal T = tridiag(beta, alpha, beta)."""
    alpha = np.asarray(alpha)
    beta = np.asarray(beta)
    j = len(alpha)
    T = np.diag(alpha.astype(np.complex128))
    if j > 1:
        T = T + np.diag(beta[: j - 1], 1) + np.diag(np.conj(beta[: j - 1]), -1)
    return sla.expm(-1j * tau * T)[:, 0]


def krylov_step_alg6(apply_H, v: np.ndarray, tau: float, n_max: int, tol: float,
                     h_norm: float):
    """One step of Alg. 6.  Returns (result, info) with info = dict(m, eps,
    converged, breakdown, alphas, betas)."""
    beta0 = np.linalg.norm(v)
    n = v.shape[0]
    V = np.zeros((n, n_max + 1), dtype=np.complex128)
    h = np.zeros((n_max + 1, n_max + 1), dtype=np.complex128)
    V[:, 0] = v / beta0
    y_prev = np.zeros(0, dtype=np.complex128)
    eps = np.inf
    for j in range(1, n_max + 1):
        w = apply_H(V[:, j - 1])
        if j > 1:
            w = w - h[j - 2, j - 1] * V[:, j - 2]
        h[j - 1, j - 1] = np.vdot(V[:, j - 1], w)
        w = w - h[j - 1, j - 1] * V[:, j - 1]
        h[j, j - 1] = np.linalg.norm(w)
        h[j - 1, j] = np.conj(h[j, j - 1])
        if h[j, j - 1] != 0:
            V[:, j] = w / h[j, j - 1]
        y = sla.expm(-1j * tau * h[:j, :j])[:, 0]
        diff = y.copy()
        diff[: j - 1] -= y_prev
        ny = np.linalg.norm(y)
        delta = np.linalg.norm(diff) / ny
        if delta < 1:
            eps = min(1 + ny, delta / (1 - delta) * ny)
        else:
            eps = 1 + ny
        breakdown = abs(h[j, j - 1]) < h_norm * tol
        if eps < tol or breakdown:
            return beta0 * (V[:, :j] @ y), dict(
                m=j, eps=eps, converged=True, breakdown=bool(breakdown),
                alphas=np.real(np.diag(h)[:j]).copy(),
                betas=np.real(np.diag(h, -1)[:j]).copy())
        y_prev = y
    j = n_max
    return beta0 * (V[:, :j] @ y), dict(
        m=j, eps=eps, converged=False, breakdown=False,
        alphas=np.real(np.diag(h)[:j]).copy(), betas=np.real(np.diag(h, -1)[:j]).copy())
