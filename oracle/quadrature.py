"""Hale-Higham-Trefethen quadrature for K^{-1/2} (oracle, FP64).

Follows Appendix B (the nodes/weights formula for f(z) = z^{-1/2} and its
real-valued restatement with t_q = -sigma_q^2, w_q = -w~_q) and Alg. S2,
which evaluates the Jacobi functions at the imaginary argument i u K'(k)
through Jacobi's imaginary transformation and SciPy's ``ellipj``.

Readings of the printed algorithm (each checked numerically in the tests):
* The squared complementary modulus is k'^2 = 1 - k^2 (the listing's comment
  assigns sqrt(1 - k^2) to it). K'(k) = K(k') is evaluated with
  ``ellipkm1(k^2)`` = K(m = 1 - k^2), so 1 - k^2 is never rounded for K'.
* The listing returns w_q and t_q with the signs of w~_q and sigma_q^2
  (both negative); the rule actually used, per the real restatement in
  Appendix B, is the positive pair t_q = -sigma_q^2, w_q = -w~_q.
* The extra 1/(pi i) prefactor of the contour sum is already inside w~_q
  and is not applied again.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def hht_quadrature(lambda_min: float, lambda_max: float, q: int):
    """Shifts t (ascending, > 0) and weights w (> 0) such that
    K^{-1/2} ~= sum_q w_q (t_q I + K)^{-1} for spec(K) in [lambda_min, lambda_max].
    """
    if not (0.0 < lambda_min <= lambda_max) or not np.isfinite(lambda_max) or q < 1:
        raise ValueError("need 0 < lambda_min <= lambda_max < inf and q >= 1")
    k2 = lambda_min / lambda_max                 # squared modulus k^2
    kp = special.ellipkm1(k2)                     # K'(k) = K(k'), parameter 1 - k^2
    u = (np.arange(1, q + 1) - 0.5) / q           # u_q = (q - 1/2) / Q
    # sn, cn, dn of (u_q K'(k) | k'), parameter m = k'^2 = 1 - k^2
    snb, cnb, dnb, _ = special.ellipj(u * kp, 1.0 - k2)
    # Jacobi imaginary transformation: sn(iu|k) = i snb/cnb, cn(iu|k) = 1/cnb,
    # dn(iu|k) = dnb/cnb, so sn^2 = -(snb/cnb)^2 is real and negative.
    sn_sq = -(snb / cnb) ** 2
    cn = 1.0 / cnb
    dn = dnb / cnb
    sigma_sq = lambda_min * sn_sq                                   # < 0
    w_tilde = -2.0 * np.sqrt(lambda_min) / (np.pi * q) * kp * cn * dn  # < 0
    return -sigma_sq, -w_tilde


def rational(t: np.ndarray, w: np.ndarray, lam) -> np.ndarray:
    """r_Q(lambda) = sum_q w_q / (t_q + lambda), the scalar CIQ approximant of
    lambda^{-1/2} (Sec. 3, rational approximation)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.sum(w[:, None] / (t[:, None] + lam.reshape(1, -1)), axis=0).reshape(lam.shape)


def max_rel_error(lambda_min: float, lambda_max: float, q: int, n_grid: int = 4001) -> float:
    """max over a log grid of [lambda_min, lambda_max] of |sqrt(lam) r_Q(lam) - 1|."""
    t, w = hht_quadrature(lambda_min, lambda_max, q)
    lam = np.geomspace(lambda_min, lambda_max, n_grid)
    return float(np.max(np.abs(np.sqrt(lam) * rational(t, w, lam) - 1.0)))
