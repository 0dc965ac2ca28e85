"""Lanczos tridiagonalisation and the extreme-eigenvalue estimate (oracle).

Appendix B.2: a few Lanczos steps from a random start give T_J; the extreme
eigenvalues of T_J estimate lambda_min / lambda_max of K, and Alg. S2 uses
them (slightly widened) to place the quadrature.

Reading of the unspecified widening (the paper only says "slightly larger
and smaller values"):
* upper: lambda_max_est = theta_max + beta_{J+1} |y_J| (the Ritz residual of
  the top Ritz pair, y the unit eigenvector of T_J);
* lower: lambda_min_est = min(theta_min, sigma^2) when sigma^2 > 0 (the
  kernel part is positive semi-definite, so sigma^2 <= lambda_min), otherwise
  theta_min / 2.
"""
from __future__ import annotations

import numpy as np


def lanczos(mvm, v0: np.ndarray, steps: int, reorth: bool = False, pinv=None):
    """Three-term Lanczos on K from v0 (Appendix B.2).

    Returns (alpha[0:J], beta[0:J]) where alpha is the diagonal of T_J and
    beta[j] = beta_{j+2} couples q_{j+1} and q_{j+2} (beta[J-1] is the
    residual norm ||r_J||). Stops early on an exact breakdown.

    With ``pinv`` (x -> P^{-1} x): Lanczos on A = P^{-1/2} K P^{-1/2} from
    P^{-1/2} v0, carried in the vectors z = P^{1/2} qt and p = P^{-1} z
    (the preconditioned form of the msMINRES oracle; no reorthogonalisation).
    """
    v0 = np.asarray(v0, dtype=np.float64)
    if pinv is not None:
        pv = pinv(v0)
        b0 = float(np.sqrt(v0 @ pv))
        z, p = v0 / b0, pv / b0
        z_prev = np.zeros_like(z)
        beta_prev = 0.0
        alpha, beta = [], []
        for _ in range(steps):
            v = mvm(p) - beta_prev * z_prev
            a = float(p @ v)
            v = v - a * z
            pv = pinv(v)
            b = float(np.sqrt(max(v @ pv, 0.0)))
            alpha.append(a)
            beta.append(b)
            if b == 0.0:
                break
            z_prev, z, p = z, v / b, pv / b
            beta_prev = b
        return np.array(alpha), np.array(beta)
    q = v0 / np.linalg.norm(v0)
    q_prev = np.zeros_like(q)
    beta_prev = 0.0
    basis = [q]
    alpha, beta = [], []
    for _ in range(steps):
        v = mvm(q) - beta_prev * q_prev
        a = float(q @ v)
        v = v - a * q
        if reorth:
            for u in basis:
                v = v - (u @ v) * u
        b = float(np.linalg.norm(v))
        alpha.append(a)
        beta.append(b)
        if b == 0.0:
            break
        q_prev, q = q, v / b
        beta_prev = b
        basis.append(q)
    return np.array(alpha), np.array(beta)


def tridiag(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    J = alpha.size
    T = np.diag(alpha)
    if J > 1:
        T += np.diag(beta[: J - 1], 1) + np.diag(beta[: J - 1], -1)
    return T


def eig_bounds(mvm, v0: np.ndarray, steps: int, noise: float, pinv=None):
    """(lambda_min_est, lambda_max_est, theta_min, theta_max) per the reading above.
    ``noise`` is the known floor of the spectrum (sigma^2 for K; 1 for the
    preconditioned operator, whose Lanczos run ``pinv`` selects)."""
    alpha, beta = lanczos(mvm, v0, steps, pinv=pinv)
    theta, y = np.linalg.eigh(tridiag(alpha, beta))
    theta_min, theta_max = float(theta[0]), float(theta[-1])
    hi = theta_max + float(beta[-1]) * abs(float(y[-1, -1]))
    lo = min(theta_min, noise) if noise > 0 else 0.5 * theta_min
    return lo, hi, theta_min, theta_max
