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


def _ngd_case(M=30, B=7, seed=3):
    rng = np.random.default_rng(seed)
    z, x, m, S = _setup(M=M, B=B, seed=seed)
    kind, ls, o2, jit = "rbf", [0.45], 1.2, 1e-4
    theta, Theta = osv.natural_from_standard(m, S)
    mu, var, a, c = osv.predictive(kind, z, x, ls, o2, jit, theta, Theta)
    y = rng.standard_normal(B)
    return theta, Theta, a, mu, y, m, S, o2


def test_elbo_gradients_match_finite_differences():
    """d ELBO / d eta and d ELBO / d H (App. E decomposition: c_mean, c_var of
    a Gaussian likelihood, the KL derivatives theta and I/2 + Theta) against
    central differences of the ELBO written out in expectation parameters."""
    theta, Theta, a, mu, y, m, S, o2 = _ngd_case()
    noise, scale = 0.3, 5.0
    cm, cv = osv.gaussian_ell_constants(y, mu, noise)
    g_eta, g_H = osv.elbo_grads(theta, Theta, a, mu, cm, cv, scale)
    eta, H = m.copy(), np.outer(m, m) + S
    f = lambda e, h: osv.elbo_gaussian(e, h, a, o2, y, noise, scale)
    h = 1e-6
    for k in (0, 11, 29):
        e = np.zeros_like(eta)
        e[k] = h
        fd = (f(eta + e, H) - f(eta - e, H)) / (2 * h)
        assert np.isclose(fd, g_eta[k], rtol=1e-6, atol=1e-7), (k, fd, g_eta[k])
    for (k, l) in ((0, 0), (4, 17), (29, 3)):
        E = np.zeros_like(H)
        E[k, l] += h
        E[l, k] += h                      # symmetric perturbation
        fd = (f(eta, H + E) - f(eta, H - E)) / (2 * h)
        want = g_H[k, l] + g_H[l, k] if k != l else 2 * g_H[k, k]
        assert np.isclose(fd, want, rtol=1e-6, atol=1e-7), (k, l, fd, want)


def test_unit_step_reaches_gaussian_optimum():
    """With a Gaussian likelihood a unit natural-gradient step from any q(u')
    lands on the minibatch's optimal whitened posterior: S* = (I + scale A A^T / noise)^{-1},
    m* = S* scale A y / noise (the ascent direction; a sign slip moves away)."""
    theta, Theta, a, mu, y, m, S, o2 = _ngd_case(M=24, B=10, seed=5)
    noise, scale = 0.2, 3.0
    cm, cv = osv.gaussian_ell_constants(y, mu, noise)
    th1, Th1 = osv.ngd_step(theta, Theta, a, mu, cm, cv, scale, 1.0)
    M = len(theta)
    S_opt = np.linalg.inv(np.eye(M) + scale * a @ a.T / noise)
    m_opt = S_opt @ (scale * a @ y / noise)
    th_opt, Th_opt = osv.natural_from_standard(m_opt, S_opt)
    assert np.allclose(Th1, Th_opt, rtol=1e-10, atol=1e-10)
    assert np.allclose(th1, th_opt, rtol=1e-9, atol=1e-10)
    # a small step increases the ELBO
    eta, H = m.copy(), np.outer(m, m) + S
    th2, Th2 = osv.ngd_step(theta, Theta, a, mu, cm, cv, scale, 0.05)
    S2 = np.linalg.inv(-2.0 * Th2)
    m2 = S2 @ th2
    before = osv.elbo_gaussian(eta, H, a, o2, y, noise, scale)
    after = osv.elbo_gaussian(m2, np.outer(m2, m2) + S2, a, o2, y, noise, scale)
    assert after > before
