"""Host checks of the FP64 device math used for kernel entries (mvm_mfma.h):
the exp polynomial's coefficients as compiled, its error over the range the
kernels use, and the square-root iteration. FMAs are emulated in extended
precision; the hardware reciprocal square root is modelled by 1/sqrt(x)
perturbed by a relative error of 2^-22 (far worse than the instruction's)."""
import pathlib
import re

import numpy as np
import pytest

SRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2006_11267_amd" / "csrc" / "mvm_mfma.h"


def _exp_coefficients():
    s = SRC.read_text()
    body = s[s.index("double exp_neg(double y)"):]
    body = body[:body.index("return ldexp")]
    lead = float(re.search(r"double p = ([0-9.eE+-]+);", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fma\(p, g, ([0-9.eE+-]+)\);", body)]
    return [lead] + rest          # highest degree first


def _fma(a, b, c):
    return (np.longdouble(a) * np.longdouble(b) + np.longdouble(c)).astype(np.float64)


def _exp_neg(y, coef):
    nf = np.rint(-y * 1.4426950408889634074)
    g = _fma(-nf, 6.93147180559945286227e-01, -y)
    g = _fma(-nf, 2.31904681384629955842e-17, g)
    p = np.full_like(g, coef[0])
    for c in coef[1:]:
        p = _fma(p, g, c)
    return np.ldexp(p, np.maximum(nf, -1100).astype(int))


def test_exp_polynomial_degree_and_leading_terms():
    coef = _exp_coefficients()
    assert len(coef) == 12
    assert coef[-1] == 1.0 and coef[-2] == 1.0 and abs(coef[-3] - 0.5) < 1e-14


def test_exp_neg_relative_error():
    coef = _exp_coefficients()
    y = np.concatenate([np.linspace(0.0, 60.0, 600_001), np.linspace(60.0, 700.0, 100_001)])
    ref = np.exp(-y.astype(np.longdouble))
    rel = np.abs(_exp_neg(y, coef) / ref - 1.0).astype(np.float64)
    assert rel.max() < 2.5e-16, rel.max()


def test_exp_neg_underflows_to_zero():
    coef = _exp_coefficients()
    assert _exp_neg(np.array([800.0, 5000.0]), coef).max() == 0.0


def _sqrt64(x, rsq_rel_err):
    x = np.maximum(x, 1e-200)
    y = (1.0 / np.sqrt(x.astype(np.longdouble))).astype(np.float64) * (1.0 + rsq_rel_err)
    g = x * y
    h = 0.5 * y
    r = _fma(-g, h, 0.5)
    g = _fma(g, r, g)
    h = _fma(h, r, h)
    d = _fma(-g, g, x)
    g = _fma(d, h, g)
    d = _fma(-g, g, x)
    return _fma(d, h, g)


@pytest.mark.parametrize("pert", [0.0, 2.0 ** -22, -(2.0 ** -22)])
def test_sqrt64_within_one_ulp(pert):
    rng = np.random.default_rng(3)
    x = np.concatenate([10.0 ** rng.uniform(-12, 4, 200_000), np.array([1.0, 4.0, 5.0, 1e-300, 0.0])])
    got = _sqrt64(x, pert)
    ref = np.sqrt(np.maximum(x, 1e-200).astype(np.longdouble))
    ulp = np.spacing(ref.astype(np.float64))
    assert (np.abs(got - ref).astype(np.float64) <= ulp).all()


def test_matern_entry_at_zero_distance_is_one():
    coef = _exp_coefficients()
    rho = _sqrt64(np.array([0.0]), 0.0)
    k = (1.0 + 0.0 / 3.0 + rho) * _exp_neg(rho, coef)
    assert k[0] == 1.0
