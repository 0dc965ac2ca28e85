"""CIQ-whitened SVGP predictive distribution in natural parameters
(oracle, FP64).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Sec. 5.1 and Appendix E. With inducing points Z (M), whitened variational
distribution q(u') = N(m', S') stored by its natural parameters
theta = S'^{-1} m', Theta = -S'^{-1} / 2, and a_x = Kzz^{-1/2} k_Zx (CIQ),

    c_x     = (-2 Theta)^{-1} a_x          (= S' a_x)
    mu(x)   = c_x^T theta                  (= a_x^T m')
    var(x)  = k(x, x) - a_x^T a_x + a_x^T c_x

and the derivatives the O(M^2) natural-gradient step needs are a_x (of mu
with respect to the expectation parameter eta = m'), -2 mu(x) a_x (of var)
and a_x a_x^T (of var with respect to H = m' m'^T + S').

Reading: Kzz carries its jitter on the diagonal (the inducing-point
problem's noise); the solve with -2 Theta is exact here (the paper uses
Jacobi-preconditioned CG, which the GPU path runs to a tolerance).
"""
from __future__ import annotations

import numpy as np

from . import ciq as _ciq
from . import posterior as _post


def natural_from_standard(m: np.ndarray, S: np.ndarray):
    """(theta, Theta) of N(m, S)."""
    Si = np.linalg.inv(S)
    return Si @ m, -0.5 * Si


def predictive(kind, z, x, lengthscale, outputscale, jitter, theta, Theta, a=None):
    """(mu, var, a, c) for the columns x, with a = Kzz^{-1/2} K_Zx by the
    symmetric root (eigendecomposition) unless given."""
    Kzx = _post.cross_kernel(kind, z, x, lengthscale, outputscale)
    if a is None:
        Kzz = _post.cross_kernel(kind, z, z, lengthscale, outputscale) + jitter * np.eye(len(z))
        a = _ciq.exact_power(Kzz, Kzx, -0.5)
    c = np.linalg.solve(-2.0 * Theta, a)
    mu = c.T @ theta
    kxx = np.full(x.shape[0], float(outputscale))           # k(x, x) = o^2 for both kernels
    var = kxx - np.sum(a * a, axis=0) + np.sum(a * c, axis=0)
    return mu, var, a, c
