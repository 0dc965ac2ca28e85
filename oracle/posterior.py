"""Gaussian-process posterior covariance at a candidate set (oracle, FP64).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Sec. 5.2 (Thompson sampling): a posterior sample at T candidate points X*
given observations at N points X is mean + Sigma^{1/2} eps, with

    Sigma = Kss + jitter I - Ksx (Kxx + sigma_obs^2 I)^{-1} Kxs,

Kss = o^2 k(X*, X*), Ksx = o^2 k(X*, X) = Kxs^T, Kxx = o^2 k(X, X), and the
small diagonal jitter the paper adds for conditioning. CIQ needs only
products Sigma v; the sample's quadratic part is Sigma^{1/2} eps.

Readings where the paper is silent: the jitter sits on the candidate block
(it keeps Sigma >= jitter I, the floor the eigenvalue bounds use); the solve
with Kxx + sigma_obs^2 I is done exactly (the paper's experiments use CG);
both leave Sigma itself unchanged up to the solve's accuracy.
"""
from __future__ import annotations

import numpy as np

from . import kernels as _k


def cross_kernel(kind, x1, x2, lengthscale, outputscale) -> np.ndarray:
    """o^2 k(x1, x2) (rows x1, columns x2), FP64."""
    return outputscale * _k.unit_kernel(kind, _k.scaled_sqdist(x1, x2, lengthscale))


def posterior_covariance(kind, xs, xo, lengthscale, outputscale, jitter, obs_noise) -> np.ndarray:
    """Dense Sigma (T x T) by the definition above (small T)."""
    Kss = cross_kernel(kind, xs, xs, lengthscale, outputscale)
    Ksx = cross_kernel(kind, xs, xo, lengthscale, outputscale)
    Kxx = cross_kernel(kind, xo, xo, lengthscale, outputscale) + obs_noise * np.eye(len(xo))
    S = Kss + jitter * np.eye(len(xs)) - Ksx @ np.linalg.solve(Kxx, Ksx.T)
    return 0.5 * (S + S.T)


def posterior_mvm(kind, xs, xo, lengthscale, outputscale, jitter, obs_noise):
    """v -> Sigma v without forming Sigma (blocked candidate product plus the
    observation correction through one solve per call)."""
    Ksx = cross_kernel(kind, xs, xo, lengthscale, outputscale)
    Kxx = cross_kernel(kind, xo, xo, lengthscale, outputscale) + obs_noise * np.eye(len(xo))

    def mvm(v):
        v = np.asarray(v, dtype=np.float64)
        out = _k.kernel_mvm_blocked(kind, xs, lengthscale, outputscale, jitter, v)
        return out - Ksx @ np.linalg.solve(Kxx, Ksx.T @ v)
    return mvm
