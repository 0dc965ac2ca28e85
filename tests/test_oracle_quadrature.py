"""Pins of the oracle's quadrature (Appendix B, Alg. S2) against things other
than itself: a closed form, a literal high-precision evaluation of the
paper's complex-argument formula, the paper's stated bounds and rates."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as qd

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))
CLAIMS = {c["id"]: c for c in GOLDEN["claims"]}


@pytest.mark.parametrize("Q", [1, 2, 3, 5, 8, 15])
@pytest.mark.parametrize("lam", [1e-3, 1.0, 37.5])
def test_kappa_one_closed_form(Q, lam):
    # k = 1: K'(1) = K(0) = pi/2, sn = sin, cn = cos, dn = 1, so
    # t_q = lam tan^2(theta_q), w_q = sqrt(lam) / (Q cos^2 theta_q),
    # theta_q = pi (q - 1/2) / (2Q), and sum_q w_q/(t_q + lam) = lam^{-1/2} exactly.
    t, w = qd.hht_quadrature(lam, lam, Q)
    th = np.pi * (np.arange(1, Q + 1) - 0.5) / (2 * Q)
    np.testing.assert_allclose(t, lam * np.tan(th) ** 2, rtol=1e-13)
    np.testing.assert_allclose(w, math.sqrt(lam) / (Q * np.cos(th) ** 2), rtol=1e-13)
    assert abs(np.sum(w / (t + lam)) * math.sqrt(lam) - 1.0) < 1e-14


def _literal_mpmath(lmin, lmax, Q):
    """The Appendix B formula evaluated literally with complex arguments:
    sigma_q^2 = lmin sn(i u_q K'(k) | k)^2, w~_q = -2 sqrt(lmin)/(pi Q) K' cn dn,
    then t = -sigma^2, w = -w~ (must come out real and positive)."""
    mp.mp.dps = 40
    lmin_m, lmax_m = mp.mpf(lmin), mp.mpf(lmax)
    m = lmin_m / lmax_m                        # parameter k^2
    Kp = mp.ellipk(1 - m)                      # K'(k) = K(k'), k'^2 = 1 - k^2
    ts, ws = [], []
    for q in range(1, Q + 1):
        z = 1j * (mp.mpf(q) - mp.mpf(1) / 2) / Q * Kp
        sn = mp.ellipfun("sn", z, m)
        cn = mp.ellipfun("cn", z, m)
        dn = mp.ellipfun("dn", z, m)
        sig2 = lmin_m * sn ** 2
        wt = -2 * mp.sqrt(lmin_m) / (mp.pi * Q) * Kp * cn * dn
        assert abs(mp.im(sig2)) < mp.mpf(10) ** -30 * (1 + abs(sig2))
        assert abs(mp.im(wt)) < mp.mpf(10) ** -30 * (1 + abs(wt))
        ts.append(float(-mp.re(sig2)))
        ws.append(float(-mp.re(wt)))
    return np.array(ts), np.array(ws)


@pytest.mark.parametrize("lmin,lmax,Q", [(1e-2, 87.0, 8), (1e-3, 2.5e3, 15), (0.3, 0.9, 4),
                                         (1e-4, 1e2, 12), (1.0, 1e8, 20)])
def test_matches_literal_complex_formula(lmin, lmax, Q):
    t, w = qd.hht_quadrature(lmin, lmax, Q)
    tr, wr = _literal_mpmath(lmin, lmax, Q)
    assert np.all(tr > 0) and np.all(wr > 0)
    kappa = lmax / lmin
    # scipy's ellipj takes the parameter m = 1 - k^2 rounded in double, which
    # costs about eps * kappa relative accuracy as kappa grows.
    rtol = 1e-13 + 4e-16 * kappa
    np.testing.assert_allclose(t, tr, rtol=rtol)
    np.testing.assert_allclose(w, wr, rtol=rtol)


def test_positive_ascending_and_scale_law():
    t, w = qd.hht_quadrature(1e-3, 50.0, 15)
    assert np.all(t > 0) and np.all(w > 0) and np.all(np.diff(t) > 0)
    t2, w2 = qd.hht_quadrature(1e-3 * 7.0, 50.0 * 7.0, 15)
    np.testing.assert_allclose(t2, 7.0 * t, rtol=1e-12)
    np.testing.assert_allclose(w2, math.sqrt(7.0) * w, rtol=1e-12)


def test_hale_rate():
    # error <= C exp(-2 Q pi^2 / (log kappa + 3)) with a moderate constant, and
    # strictly decaying in Q until double-precision round-off
    for kappa in [1e2, 1e4, 1e6, 1e8]:
        prev = None
        for Q in [2, 4, 6, 8, 10, 12, 15]:
            err = qd.max_rel_error(1.0, kappa, Q)
            bound = math.exp(-2 * Q * math.pi ** 2 / (math.log(kappa) + 3))
            assert err <= 20.0 * bound + 1e-14, (kappa, Q, err, bound)
            if prev is not None and prev > 1e-13:
                assert err < prev
            prev = err


def test_paper_claims_q8_and_q20():
    c8 = CLAIMS["q8_kappa_1e4"]
    assert qd.max_rel_error(1.0, c8["kappa"], c8["q"]) < c8["max_rel_err"]
    c20 = CLAIMS["q20_machine_precision"]
    assert qd.max_rel_error(1.0, c20["kappa"], c20["q"]) < c20["max_rel_err"]


@pytest.mark.parametrize("kappa", [1.5, 1e2, 1e4, 1e7])
@pytest.mark.parametrize("Q", [3, 8, 15])
def test_weight_shift_ratio_lemma(kappa, Q):
    lmin = 0.37
    t, w = qd.hht_quadrature(lmin, lmin * kappa, Q)
    lhs = np.sum(w / t)
    rhs = 4 * Q * math.log(5 * math.sqrt(kappa)) / (math.pi * math.sqrt(lmin))
    assert lhs < rhs


@pytest.mark.parametrize("Q", [1, 2, 7, 15, 40])
def test_trig_identity(Q):
    th = np.pi * (np.arange(1, Q + 1) - 0.5) / (2 * Q)
    assert abs(np.sum(1.0 / (Q * np.sin(th) ** 2)) - 2 * Q) < 1e-10 * Q


def test_rejects_bad_bounds():
    for args in [(0.0, 1.0, 4), (2.0, 1.0, 4), (1.0, 2.0, 0), (-1.0, 1.0, 3), (1.0, float("inf"), 3)]:
        with pytest.raises(ValueError):
            qd.hht_quadrature(*args)


def test_planted_sign_mistake_is_caught():
    # the listing's literal return values (negative w~, sigma^2) must fail the
    # exactness pin: this guards the reading of the sign convention.
    t, w = qd.hht_quadrature(2.0, 2.0, 5)
    assert not abs(np.sum((-w) / ((-t) + 2.0)) * math.sqrt(2.0) - 1.0) < 1e-3
