"""Pins of the preconditioned oracle (Sec. 3.4, Appendix D) against things
other than itself: LAPACK's pivoted Cholesky, dense linear algebra, the
unpreconditioned msMINRES run on an explicitly formed A = P^{-1/2} K P^{-1/2},
and the identities R' R'^T = K^{-1}, R R^T = K, R'^T K R' = I."""
import numpy as np
import pytest
from scipy.linalg import eigh as geigh
from scipy.linalg import lapack

from oracle import ciq as oc
from oracle import kernels as ok
from oracle import msminres as om
from oracle import precond as op
from oracle import quadrature as oq


def _points(n, d, seed):
    return np.random.default_rng(seed).random((n, d))


def _ktil(kind, x, ls, o2):
    return ok.kernel_matrix(kind, x, ls, o2, 0.0)


@pytest.mark.parametrize("kind,n,d,ls,rank", [("rbf", 120, 3, 0.4, 25), ("matern52", 150, 5, 0.3, 40),
                                             ("rbf", 60, 2, 0.2, 60)])
def test_pivoted_cholesky_matches_lapack(kind, n, d, ls, rank):
    """The first R columns of LAPACK's complete-pivoting Cholesky (dpstrf,
    the same largest-diagonal rule) are the rank-R partial factor."""
    x = _points(n, d, n + rank)
    Kt = _ktil(kind, x, [ls], 1.3)
    L, piv, dres = op.pivoted_cholesky(kind, x, [ls], 1.3, rank)
    c, lpiv, lrank, info = lapack.dpstrf(Kt.copy(), lower=1, tol=-1.0)
    assert info >= 0
    m = min(rank, lrank, len(piv))
    lp = np.asarray(lpiv[:m]) - 1
    assert np.array_equal(piv[:m], lp)
    Lf = np.tril(c)
    Lp = np.zeros((n, m))
    Lp[np.asarray(lpiv) - 1, :] = Lf[:, :m]
    assert np.allclose(L[:, :m], Lp, atol=1e-12, rtol=0)


def test_pivoted_cholesky_structure():
    kind, n, d, ls, o2, rank = "matern52", 200, 6, 0.3, 1.0, 50
    x = _points(n, d, 7)
    Kt = _ktil(kind, x, [ls], o2)
    L, piv, dres = op.pivoted_cholesky(kind, x, [ls], o2, rank)
    assert len(piv) == rank and len(set(piv.tolist())) == rank
    res = Kt - L @ L.T
    assert np.allclose(np.diag(res), dres, atol=1e-12)
    # residual is a Schur complement: PSD, zero on the pivot rows/columns
    assert np.linalg.eigvalsh(res).min() > -1e-12
    assert np.abs(res[piv, :]).max() < 1e-12
    # lower triangular in pivot order, positive diagonal
    Lp = L[piv, :]
    assert np.allclose(np.triu(Lp, 1), 0.0)
    assert (np.diag(Lp) > 0).all()
    # the trace of the residual never grows with the rank
    t = [op.pivoted_cholesky(kind, x, [ls], o2, r)[2].sum() for r in (5, 10, 20, 50)]
    assert all(a >= b for a, b in zip(t, t[1:]))
    assert np.isclose(t[-1], np.trace(res))


def test_pivoted_cholesky_full_rank_and_stop_rule():
    x = _points(150, 2, 3)
    Kt = _ktil("rbf", x, [0.5], 1.0)
    L, piv, dres = op.pivoted_cholesky("rbf", x, [0.5], 1.0, 150)
    # numerically low rank: the rule stops before 150 columns, the rest stay zero
    assert len(piv) < 150 and np.all(L[:, len(piv):] == 0.0)
    assert dres.max() <= op.STOP_RTOL
    assert np.abs(Kt - L @ L.T).max() < 1e-9
    # duplicated points: the factor never takes a duplicate as a pivot
    xd = np.vstack([x[:10], x[:10]])
    L2, piv2, _ = op.pivoted_cholesky("rbf", xd, [0.5], 1.0, 20)
    assert len(piv2) <= 10


def test_preconditioner_inverse_and_root():
    x = _points(90, 4, 11)
    L, _, _ = op.pivoted_cholesky("matern52", x, [0.35], 1.0, 15)
    pre = op.Preconditioner(L, 1e-2)
    P = pre.dense()
    X = np.random.default_rng(1).standard_normal((90, 5))
    assert np.allclose(pre.inv(X), np.linalg.solve(P, X), rtol=1e-10, atol=1e-10)
    lp, Up = np.linalg.eigh(P)
    Ph = (Up * np.sqrt(lp)) @ Up.T
    assert np.allclose(pre.sqrt(X), Ph @ X, rtol=1e-11, atol=1e-11)
    assert np.allclose(pre.sqrt(pre.sqrt(X)), P @ X, rtol=1e-10, atol=1e-10)
    with pytest.raises(ValueError):
        op.Preconditioner(L, 0.0)


def _setup(kind="matern52", n=160, d=5, ls=0.3, o2=1.0, s2=1e-3, rank=20, s=3, seed=5):
    x = _points(n, d, seed)
    K = ok.kernel_matrix(kind, x, [ls], o2, s2)
    L, _, _ = op.pivoted_cholesky(kind, x, [ls], o2, rank)
    pre = op.Preconditioner(L, s2)
    B = np.random.default_rng(seed + 1).standard_normal((n, s))
    return x, K, pre, B


def test_preconditioned_spectrum_floor():
    """A = P^{-1/2} K P^{-1/2} >= I (the pivoted-Cholesky residual is PSD).
    When N exceeds the kernel's numerical rank (lambda_min(K) ~ sigma^2, as
    at the large workloads) kappa(A) is far below kappa(K); when K's smallest
    eigenvalue is well above sigma^2 the floor 1 of A makes kappa larger
    (300 points in 5 dimensions), a property of this preconditioner."""
    x, K, pre, _ = _setup(n=400, d=3, rank=60)
    g = geigh(K, pre.dense(), eigvals_only=True)
    assert g[0] > 1 - 1e-9
    assert np.isclose(g[0], 1.0, atol=1e-8)          # residual rank < N: eigenvalue 1 exists
    ek = np.linalg.eigvalsh(K)
    assert 20 * g[-1] / g[0] < ek[-1] / ek[0]
    x, K, pre, _ = _setup(n=300, d=5, rank=40)
    g = geigh(K, pre.dense(), eigvals_only=True)
    ek = np.linalg.eigvalsh(K)
    assert g[0] > 1 - 1e-9 and g[-1] / g[0] > ek[-1] / ek[0]


@pytest.mark.parametrize("j,bar", [(1, 1e-9), (2, 1e-9), (5, 1e-9), (12, 1e-9), (30, 1e-5)])
def test_preconditioned_msminres_equals_transformed_system(j, bar):
    """Iterate j of the P^{-1} recurrence = P^{-1/2} times the plain msMINRES
    iterate j on the explicit A with right-hand side P^{-1/2} c. The two
    runs round differently; once the Lanczos vectors lose orthogonality
    (j = 30 here) their iterates drift apart by more than rounding, hence
    the looser bar there."""
    x, K, pre, B = _setup()
    t = np.array([1e-3, 0.1, 10.0])
    X, info = om.msminres(lambda v: K @ v, B, t, j, 0.0, pinv=pre.inv)
    lp, Up = np.linalg.eigh(pre.dense())
    Pmh = (Up / np.sqrt(lp)) @ Up.T
    A = Pmh @ K @ Pmh
    A = 0.5 * (A + A.T)
    Y, info2 = om.msminres(lambda v: A @ v, Pmh @ B, t, j, 0.0)
    ref = np.einsum("ij,qjs->qis", Pmh, Y)
    scale = np.abs(ref).max()
    assert np.abs(X - ref).max() <= bar * scale
    assert np.allclose(info.rel_residual, info2.rel_residual, rtol=max(1e-7, 100 * bar), atol=1e-12)
    # |phibar| is the residual of the transformed system
    u = Pmh @ B
    Ph = (Up * np.sqrt(lp)) @ Up.T
    for qi, tq in enumerate(t):
        yq = Ph @ X[qi]
        r = np.linalg.norm((A + tq * np.eye(len(A))) @ yq - u, axis=0) / np.linalg.norm(u, axis=0)
        assert np.allclose(r, info.rel_residual[qi], rtol=1e-6, atol=1e-12)


def test_preconditioned_msminres_fewer_iterations():
    x, K, pre, B = _setup(n=400, d=3, rank=60, s=2)
    t = np.array([1e-3])
    _, i_pc = om.msminres(lambda v: K @ v, pre.sqrt(B), t, 2000, 1e-6, pinv=pre.inv)
    _, i_pl = om.msminres(lambda v: K @ v, B, t, 2000, 1e-6)
    assert i_pc.converged.all() and i_pl.converged.all()
    assert 2 * i_pc.iters < i_pl.iters


def test_preconditioned_bounds_interlace():
    x, K, pre, _ = _setup(n=250, rank=30)
    g = geigh(K, pre.dense(), eigvals_only=True)
    v0 = np.random.default_rng(2).standard_normal(250)
    lo, hi, tmin, tmax = op.eig_bounds(lambda v: K @ v, pre, v0, 20)
    assert g[0] - 1e-9 <= tmin <= tmax <= g[-1] * (1 + 1e-9)
    assert lo <= 1.0 and hi >= tmax
    assert hi >= 0.98 * g[-1]


@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_pc_ciq_rotation_equivalence(mode):
    """With B = I and a tight tolerance, the outputs form R' (R): R' R'^T =
    K^{-1}, R'^T K R' = I, R R^T = K (to the quadrature error at Q = 20)."""
    kind, n = "rbf", 120
    x = _points(n, 3, 21)
    s2 = 1e-2
    K = ok.kernel_matrix(kind, x, [0.4], 1.0, s2)
    L, _, _ = op.pivoted_cholesky(kind, x, [0.4], 1.0, 12)
    pre = op.Preconditioner(L, s2)
    g = geigh(K, pre.dense(), eigvals_only=True)
    out, info = op.ciq_pc(lambda v: K @ v, pre, np.eye(n), g[0], g[-1], 20, 400, 1e-12, mode=mode)
    assert info.converged.all()
    if mode == "invsqrt":
        assert np.abs(out @ out.T - np.linalg.inv(K)).max() <= 1e-7 * np.abs(np.linalg.inv(K)).max()
        assert np.abs(out.T @ K @ out - np.eye(n)).max() <= 1e-7
    else:
        assert np.abs(out @ out.T - K).max() <= 1e-7 * np.abs(K).max()
    # not the symmetric root itself (a genuine rotation)
    ref = oc.exact_power(K, np.eye(n), -0.5 if mode == "invsqrt" else 0.5)
    assert np.abs(out - ref).max() > 1e-4 * np.abs(ref).max()


def test_pc_ciq_equals_rational_of_a():
    """With exact shifted solves, the output is P^{-1/2} r_Q(A) B (r_Q the
    quadrature rational) to rounding; against A^{-1/2} to the quadrature error."""
    x, K, pre, B = _setup(n=150, rank=25)
    g = geigh(K, pre.dense(), eigvals_only=True)
    q = 10
    t, w = oq.hht_quadrature(g[0], g[-1], q)
    out, info = op.ciq_pc(lambda v: K @ v, pre, B, g[0], g[-1], q, 600, 1e-13)
    assert info.converged.all()
    rq = lambda la: oq.rational(t, w, la)
    ref = op.dense_reference(K, pre, B, rq)
    assert np.abs(out - ref).max() <= 1e-9 * np.abs(ref).max()
    ex = op.dense_reference(K, pre, B, lambda la: la ** -0.5)
    err = np.linalg.norm(out - ex) / np.linalg.norm(ex)
    assert err <= 2 * oq.max_rel_error(g[0], g[-1], q) + 1e-10
