"""Pins of the oracle's CIQ composition (Sec. 3, Alg. S1) against the plain
eigendecomposition definition, closed forms and invariants."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ciq
from oracle import kernels as kk
from oracle import lanczos as lz
from oracle import quadrature as qd

CLAIMS = {c["id"]: c for c in json.load(open(os.path.join(
    os.path.dirname(__file__), "golden", "paper_claims.json")))["claims"]}


def test_diagonal_matrix_exact():
    d = np.geomspace(0.01, 30.0, 9).repeat(3)
    K = np.diag(d)
    b = np.random.default_rng(1).standard_normal((27, 2))
    t, w = qd.hht_quadrature(d.min(), d.max(), 20)
    d4 = np.array([0.2, 1.0, 3.0, 6.0]).repeat(5)
    b4 = b[:20]
    for mode, p in [("invsqrt", -0.5), ("sqrt", 0.5)]:
        # 4 distinct eigenvalues: the Krylov space is exhausted after 4 products
        out, info = ciq.ciq(lambda v: d4[:, None] * v, b4, 0.2, 6.0, 20, 4, 0.0, mode)
        assert info.iters == 4
        np.testing.assert_allclose(out, (d4 ** p)[:, None] * b4, rtol=1e-11)
        # many distinct eigenvalues: converges to the exact root elementwise
        out, info = ciq.ciq(lambda v: K @ v, b, d.min(), d.max(), 20, 100, 1e-13, mode)
        np.testing.assert_allclose(out, (d ** p)[:, None] * b, rtol=1e-11)


def test_equals_exact_rational_at_convergence():
    rng = np.random.default_rng(2)
    x = rng.random((24, 2))
    K = kk.kernel_matrix("matern52", x, [0.4], 1.3, 0.05)
    lam = np.linalg.eigvalsh(K)
    b = rng.standard_normal((24, 3))
    for mode in ["invsqrt", "sqrt"]:
        out, info, t, w, _ = ciq.ciq(lambda v: K @ v, b, lam[0], lam[-1], 7, 300, 1e-13, mode,
                                      return_solves=True)
        ref = ciq.exact_rational(K, b, t, w, mode)
        assert np.max(ciq.rel_err(out, ref)) < 1e-10


@pytest.mark.parametrize("family", ["isqrt", "inv2"])
def test_paper_claim_q8_families(family):
    # Fig. 1: Q = 8 gives < 1e-4 for spectra t^{-1/2} and t^{-2} (exact bounds, exact solves)
    c = CLAIMS["q8_below_1e-4"]
    rng = np.random.default_rng(3)
    N = 200
    U, _ = np.linalg.qr(rng.standard_normal((N, N)))
    tt = np.arange(1, N + 1.0)
    lam = tt ** -0.5 if family == "isqrt" else tt ** -2.0
    K = (U * lam) @ U.T
    K = 0.5 * (K + K.T)
    b = rng.standard_normal(N)
    t, w = qd.hht_quadrature(lam.min(), lam.max(), c["q"])
    err = ciq.rel_err(ciq.exact_rational(K, b, t, w, "sqrt"), ciq.exact_power(K, b, 0.5))[0]
    assert err < c["max_rel_err"]


def test_invariants_and_theorem_bound():
    rng = np.random.default_rng(4)
    x = rng.random((300, 3))
    K = kk.kernel_matrix("rbf", x, [0.25], 1.0, 1e-2)
    lam = np.linalg.eigvalsh(K)
    kappa = lam[-1] / lam[0]
    b = rng.standard_normal(300)
    mvm = lambda v: K @ v
    s, i1 = ciq.ciq(mvm, b, lam[0], lam[-1], 15, 400, 1e-10, "sqrt")
    a, i2 = ciq.ciq(mvm, b, lam[0], lam[-1], 15, 400, 1e-10, "invsqrt")
    ss, _ = ciq.ciq(mvm, s, lam[0], lam[-1], 15, 400, 1e-10, "sqrt")
    back, _ = ciq.ciq(mvm, s, lam[0], lam[-1], 15, 400, 1e-10, "invsqrt")
    assert np.linalg.norm(ss - K @ b) / np.linalg.norm(K @ b) < 1e-6
    assert np.linalg.norm(back - b) / np.linalg.norm(b) < 1e-6
    assert np.linalg.norm(K @ a - s) / np.linalg.norm(s) < 1e-12   # sqrt = K * invsqrt
    # Theorem 1: ||a_J - K^{1/2} b|| <= quad term + msMINRES term (loose; check at small J)
    for J in [5, 20, 60]:
        sJ, _ = ciq.ciq(mvm, b, lam[0], lam[-1], 15, J, 0.0, "sqrt")
        err = np.linalg.norm(sJ - ciq.exact_power(K, b, 0.5))
        rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
        ms_term = 2 * 15 * math.log(5 * math.sqrt(kappa)) * kappa * math.sqrt(lam[0]) / math.pi \
            * rho ** (J - 1) * np.linalg.norm(b)
        quad = qd.max_rel_error(lam[0], lam[-1], 15) * np.linalg.norm(ciq.exact_power(K, b, 0.5))
        assert err <= ms_term + 2 * quad + 1e-12


def test_error_decays_in_q_then_plateaus_at_solver_tol():
    rng = np.random.default_rng(5)
    x = rng.random((400, 2))
    K = kk.kernel_matrix("matern52", x, [0.3], 1.0, 1e-3)
    lam = np.linalg.eigvalsh(K)
    b = rng.standard_normal(400)
    ex = ciq.exact_power(K, b, -0.5)
    errs = []
    for Q in [2, 4, 8, 12]:
        t, w = qd.hht_quadrature(lam[0], lam[-1], Q)
        errs.append(ciq.rel_err(ciq.exact_rational(K, b, t, w), ex)[0])
    assert errs[0] > errs[1] > errs[2] > errs[3]
    out, info = ciq.ciq(lambda v: K @ v, b, lam[0], lam[-1], 12, 2000, 1e-4)
    e = ciq.rel_err(out, ex)[0]
    assert 1e-7 < e < 1e-3            # at the msMINRES tolerance, not the quadrature's


def test_lanczos_bounds_interlace_and_converge():
    rng = np.random.default_rng(6)
    x = rng.random((500, 3))
    K = kk.kernel_matrix("rbf", x, [0.2], 1.0, 1e-2)
    lam = np.linalg.eigvalsh(K)
    v0 = rng.standard_normal(500)
    for J in [5, 10, 20]:
        a, bt = lz.lanczos(lambda v: K @ v, v0, J, reorth=True)
        th = np.linalg.eigvalsh(lz.tridiag(a, bt))
        assert th[0] >= lam[0] - 1e-10 and th[-1] <= lam[-1] + 1e-10
    a, bt = lz.lanczos(lambda v: K @ v, v0, 60, reorth=True)
    th = np.linalg.eigvalsh(lz.tridiag(a, bt))
    assert abs(th[-1] - lam[-1]) < 1e-8 * lam[-1]
    lo, hi, tmin, tmax = lz.eig_bounds(lambda v: K @ v, v0, 20, 1e-2)
    assert lo <= lam[0] + 1e-12 and hi >= tmax and abs(hi - lam[-1]) < 0.05 * lam[-1]
