"""Pins of the SVGP predictive oracle (Sec. 5.1, App. E): the natural-parameter
forms equal the standard whitened forms and the unwhitened textbook
predictive distribution of q(u) = N(Kzz^{1/2} m', Kzz^{1/2} S' Kzz^{1/2});
the App. E derivatives against central finite differences."""
import numpy as np

from oracle import kernels as ok
from oracle import svgp as osv


def _setup(M=60, B=9, d=3, seed=0):
    rng = np.random.default_rng(seed)
    z, x = rng.random((M, d)), rng.random((B, d))
    m = rng.standard_normal(M) * 0.5
    G = rng.standard_normal((M, M)) / np.sqrt(M)
    S = G @ G.T * 0.3 + 0.2 * np.eye(M)
    return z, x, m, S


def test_natural_forms_equal_standard_and_unwhitened():
    z, x, m, S = _setup()
    kind, ls, o2, jit = "matern52", [0.4], 1.3, 1e-4
    theta, Theta = osv.natural_from_standard(m, S)
    mu, var, a, c = osv.predictive(kind, z, x, ls, o2, jit, theta, Theta)
    assert np.allclose(c, S @ a, rtol=1e-10, atol=1e-12)
    assert np.allclose(mu, a.T @ m, rtol=1e-10, atol=1e-12)
    std_var = o2 - np.einsum("ib,ij,jb->b", a, np.eye(len(z)) - S, a)
    assert np.allclose(var, std_var, rtol=1e-10, atol=1e-12)
    # unwhitened: q(u) = N(Kzz^{1/2} m, Kzz^{1/2} S Kzz^{1/2}); the usual SVGP predictive
    Kzz = ok.kernel_matrix(kind, z, ls, o2, jit)
    lam, U = np.linalg.eigh(Kzz)
    R = (U * np.sqrt(lam)) @ U.T
    mu_u, S_u = R @ m, R @ S @ R
    Kzx = o2 * ok.unit_kernel(kind, ok.scaled_sqdist(z, x, ls))
    A = np.linalg.solve(Kzz, Kzx)
    assert np.allclose(mu, A.T @ mu_u, rtol=1e-8, atol=1e-10)
    v_ref = o2 - np.sum(Kzx * A, axis=0) + np.einsum("ib,ij,jb->b", A, S_u, A)
    assert np.allclose(var, v_ref, rtol=1e-7, atol=1e-9)


def test_expectation_parameter_derivatives():
    """d mu / d eta = a, d var / d eta = -2 mu a, d var / d H = a a^T, with
    eta = m', H = m' m'^T + S' (finite differences through the standard
    parameters m' = eta, S' = H - eta eta^T)."""
    z, x, m, S = _setup(M=25, B=3)
    kind, ls, o2, jit = "rbf", [0.5], 1.0, 1e-4
    eta, H = m.copy(), np.outer(m, m) + S

    def f(eta_, H_):
        th, Th = osv.natural_from_standard(eta_, H_ - np.outer(eta_, eta_))
        return osv.predictive(kind, z, x, ls, o2, jit, th, Th)

    mu, var, a, c = f(eta, H)
    h = 1e-6
    for k in (0, 7, 19):
        e = np.zeros_like(eta)
        e[k] = h
        mp, vp, *_ = f(eta + e, H)
        mm, vm, *_ = f(eta - e, H)
        assert np.allclose((mp - mm) / (2 * h), a[k], rtol=1e-6, atol=1e-8)
        assert np.allclose((vp - vm) / (2 * h), -2 * mu * a[k], rtol=1e-5, atol=1e-7)
    for (i, j) in ((0, 0), (3, 11)):
        E = np.zeros_like(H)
        E[i, j] += h / 2
        E[j, i] += h / 2
        _, vp, *_ = f(eta, H + E)
        _, vm, *_ = f(eta, H - E)
        assert np.allclose((vp - vm) / (2 * h), a[i] * a[j], rtol=1e-5, atol=1e-8)
