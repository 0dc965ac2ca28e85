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

The natural-gradient step of App. E: the expected log likelihood of a point
depends on the variational parameters only through mu(x) and var(x), so
with c_mean = d ELL / d mu and c_var = d ELL / d var (the likelihood's
constants; closed form for a Gaussian likelihood) the chain rule gives

    d ELL / d eta = (c_mean - 2 c_var mu) a,     d ELL / d H = c_var a a^T,

and the whitened KL term has d KL / d eta = theta, d KL / d H = I/2 + Theta.
The step moves the natural parameters by `step` times the ELBO gradient in
the expectation parameters (the minibatch sum scaled by N / B). Reading: the
paper prints the update with a minus sign on the ELBO gradient; the ELBO is
maximised, so the step here ascends it (equivalently, descends -ELBO). At
step 1 with a Gaussian likelihood it lands on the minibatch's optimal q(u'),
which the tests check in closed form.
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


def elbo_grads(theta, Theta, a, mu, c_mean, c_var, scale):
    """(d ELBO / d eta, d ELBO / d H) for the minibatch with columns a (M x B),
    predictive means mu (B) and likelihood constants c_mean, c_var (B)."""
    M = a.shape[0]
    g_eta = scale * (a @ (c_mean - 2.0 * c_var * mu)) - theta
    g_H = scale * ((a * c_var) @ a.T) - (0.5 * np.eye(M) + Theta)
    return g_eta, g_H


def ngd_step(theta, Theta, a, mu, c_mean, c_var, scale, step):
    """One natural-gradient step: natural parameters += step * ELBO gradient in
    the expectation parameters."""
    g_eta, g_H = elbo_grads(theta, Theta, a, mu, c_mean, c_var, scale)
    return theta + step * g_eta, Theta + step * g_H


def gaussian_ell_constants(y, mu, noise):
    """c_mean, c_var of E_q log N(y | f, noise) = -log(2 pi noise)/2 - ((y - mu)^2 + var) / (2 noise)."""
    return (y - mu) / noise, np.full(np.shape(mu), -0.5 / noise)


def elbo_gaussian(eta, H, a, kxx, y, noise, scale):
    """The ELBO with a Gaussian likelihood as a function of the expectation
    parameters (eta, H): scale * sum_b E_q log N(y_b | f_b, noise) - KL(q(u') || N(0, I)),
    mu_b = a_b^T eta, var_b = kxx - a_b^T a_b + a_b^T (H - eta eta^T) a_b."""
    S = H - np.outer(eta, eta)
    mu = a.T @ eta
    var = kxx - np.sum(a * a, axis=0) + np.einsum("ib,ij,jb->b", a, S, a)
    ell = np.sum(-0.5 * np.log(2.0 * np.pi * noise) - ((y - mu) ** 2 + var) / (2.0 * noise))
    sign, logdet = np.linalg.slogdet(S)
    kl = 0.5 * (np.trace(H) - logdet - len(eta))
    return scale * ell - kl
