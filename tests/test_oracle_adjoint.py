"""Pins of the oracle's backward pass (Sec. 3.3) against the Daleckii-Krein
divided-difference formula and central finite differences."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import ciq
from oracle import kernels as kk
from oracle import quadrature as qd


def _problem(kind="rbf", n=64, d=3, seed=0, ard=True):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    ls = np.exp(rng.uniform(np.log(0.2), np.log(0.8), d)) if ard else np.array([0.35])
    return x, ls, 1.3, 0.05, rng


@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_matches_daleckii_krein_of_rational(mode):
    x, ls, o2, s2, rng = _problem()
    K = kk.kernel_matrix("rbf", x, ls, o2, s2)
    lam = np.linalg.eigvalsh(K)
    B = rng.standard_normal((64, 3))
    G = rng.standard_normal((64, 3))
    mvm = lambda v: K @ v
    _, _, t, w, A = ciq.ciq(mvm, B, lam[0], lam[-1], 10, 64, 1e-14, mode, return_solves=True)
    dB, dK = adj.ciq_vjp(mvm, A, G, t, w, 64, 1e-14, mode)
    if mode == "invsqrt":
        ddf = adj.dd_rational(t, w)
        fB = ciq.exact_rational(K, G, t, w, "invsqrt")
    else:
        base = adj.dd_rational(t, w)
        ddf = lambda li, lj: np.sum([wq * tq / ((tq + li) * (tq + lj)) for tq, wq in zip(t, w)], axis=0)
        fB = ciq.exact_rational(K, G, t, w, "sqrt")
        del base
    ref = adj.daleckii_krein_vjp(K, B, G, ddf)
    assert np.linalg.norm(dK - ref) <= 1e-8 * np.linalg.norm(ref)
    np.testing.assert_allclose(dB, fB, rtol=1e-8, atol=1e-10)


def test_matches_true_derivative_within_quadrature_error():
    x, ls, o2, s2, rng = _problem(seed=1)
    K = kk.kernel_matrix("rbf", x, ls, o2, s2)
    lam = np.linalg.eigvalsh(K)
    B = rng.standard_normal((64, 2))
    G = rng.standard_normal((64, 2))
    mvm = lambda v: K @ v
    _, _, t, w, A = ciq.ciq(mvm, B, lam[0], lam[-1], 20, 64, 1e-14, "invsqrt", return_solves=True)
    _, dK = adj.ciq_vjp(mvm, A, G, t, w, 64, 1e-14)
    ref = adj.daleckii_krein_vjp(K, B, G, adj.dd_invsqrt)
    assert np.linalg.norm(dK - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["rbf", "matern52"])
@pytest.mark.parametrize("ard", [True, False])
def test_hyperparameter_grads_vs_finite_differences(kind, ard):
    x, ls, o2, s2, rng = _problem(kind, n=40, d=3, seed=2, ard=ard)
    B = rng.standard_normal((40, 2))
    G = rng.standard_normal((40, 2))
    K = kk.kernel_matrix(kind, x, ls, o2, s2)
    lam = np.linalg.eigvalsh(K)
    lo, hi = 0.5 * lam[0], 2.0 * lam[-1]
    t, w = qd.hht_quadrature(lo, hi, 12)

    def loss(ls_, o2_, s2_, B_=B):
        Kp = kk.kernel_matrix(kind, x, ls_, o2_, s2_)
        return float(np.sum(G * ciq.exact_rational(Kp, B_, t, w)))

    mvm = lambda v: K @ v
    _, _, _, _, A = ciq.ciq(mvm, B, lo, hi, 12, 400, 1e-13, return_solves=True)
    dB, dK = adj.ciq_vjp(mvm, A, G, t, w, 400, 1e-13)
    g_ls, g_o2, g_s2 = adj.hyper_grads(kind, x, ls, o2, dK)
    h = 1e-6
    for d in range(ls.size):
        e = np.zeros(ls.size); e[d] = h * ls[d]
        fd = (loss(ls + e, o2, s2) - loss(ls - e, o2, s2)) / (2 * e[d])
        assert abs(g_ls[d] - fd) <= 1e-6 * (abs(fd) + 1e-3)
    fd = (loss(ls, o2 * (1 + h), s2) - loss(ls, o2 * (1 - h), s2)) / (2 * h * o2)
    assert abs(g_o2 - fd) <= 1e-6 * (abs(fd) + 1e-3)
    fd = (loss(ls, o2, s2 * (1 + h)) - loss(ls, o2, s2 * (1 - h))) / (2 * h * s2)
    assert abs(g_s2 - fd) <= 1e-6 * (abs(fd) + 1e-3)
    i, j = 5, 1
    E = np.zeros_like(B); E[i, j] = 1e-6
    fd = (loss(ls, o2, s2, B + E) - loss(ls, o2, s2, B - E)) / 2e-6
    assert abs(dB[i, j] - fd) <= 1e-7 * (abs(fd) + 1e-3)
