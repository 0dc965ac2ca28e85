"""Pins of the posterior-covariance oracle (Sec. 5.2) against the joint
Gaussian it conditions: the block of the inverse joint covariance, positive
semi-definiteness above the jitter, zero posterior variance at noise-free
observations, and CIQ on it against the eigendecomposition."""
import numpy as np
import pytest

from oracle import ciq as oc
from oracle import kernels as ok
from oracle import posterior as opost
from oracle import quadrature as oq


def _pts(seed, t, n, d):
    rng = np.random.default_rng(seed)
    return rng.random((t, d)), rng.random((n, d))


@pytest.mark.parametrize("kind,t,n,d", [("rbf", 120, 30, 3), ("matern52", 90, 45, 6)])
def test_posterior_is_the_conditional_of_the_joint(kind, t, n, d):
    """Sigma^{-1} is the candidate block of the inverse joint covariance of
    (f(X*) + jitter noise, y(X)): an independent route through one dense
    kernel matrix of the stacked points."""
    xs, xo = _pts(t + n, t, n, d)
    ls, o2, jit, s2 = [0.4], 1.7, 1e-3, 2e-2
    S = opost.posterior_covariance(kind, xs, xo, ls, o2, jit, s2)
    J = ok.kernel_matrix(kind, np.vstack([xs, xo]), ls, o2, 0.0)
    J[:t, :t] += jit * np.eye(t)
    J[t:, t:] += s2 * np.eye(n)
    Jinv = np.linalg.inv(J)
    ref = np.linalg.inv(Jinv[:t, :t])
    assert np.abs(S - ref).max() <= 1e-8 * np.abs(ref).max()


def test_posterior_floor_and_interpolation():
    xs, xo = _pts(3, 80, 20, 2)
    xs[:20] = xo                      # candidates that coincide with observations
    ls, o2, jit = [0.3], 1.0, 1e-4
    S = opost.posterior_covariance("matern52", xs, xo, ls, o2, jit, 1e-10)
    lam = np.linalg.eigvalsh(S)
    assert lam[0] >= jit * (1 - 1e-6)
    # noise-free observations pin the posterior: variance = jitter there
    assert np.allclose(np.diag(S)[:20], jit, rtol=0, atol=1e-8)
    assert np.all(np.diag(S)[20:] > jit)
    # more noise, less information: the covariance grows (Loewner order)
    S2 = opost.posterior_covariance("matern52", xs, xo, ls, o2, jit, 1e-1)
    assert np.linalg.eigvalsh(S2 - S)[0] > -1e-10


def test_posterior_mvm_matches_dense():
    xs, xo = _pts(5, 300, 40, 4)
    args = ("rbf", xs, xo, [0.35], 1.2, 1e-3, 1e-2)
    S = opost.posterior_covariance(*args)
    V = np.random.default_rng(1).standard_normal((300, 3))
    assert np.allclose(opost.posterior_mvm(*args)(V), S @ V, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode,p", [("invsqrt", -0.5), ("sqrt", 0.5)])
def test_ciq_on_posterior_against_eigendecomposition(mode, p):
    xs, xo = _pts(9, 250, 30, 3)
    args = ("matern52", xs, xo, [0.3], 1.0, 1e-3, 1e-4)
    S = opost.posterior_covariance(*args)
    lam = np.linalg.eigvalsh(S)
    B = np.random.default_rng(2).standard_normal((250, 4))
    q = 15
    out, info = oc.ciq(opost.posterior_mvm(*args), B, lam[0], lam[-1], q, 1500, 1e-12, mode)
    assert info.converged.all()
    ex = oc.exact_power(S, B, p)
    err = np.linalg.norm(out - ex, axis=0) / np.linalg.norm(ex, axis=0)
    # per eigencomponent both forms err by |sqrt(lam) r_Q(lam) - 1| (the quadrature bound)
    assert err.max() <= 2 * oq.max_rel_error(lam[0], lam[-1], q) + 1e-9
