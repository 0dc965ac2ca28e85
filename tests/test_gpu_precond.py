"""The pivoted-Cholesky preconditioned path (Sec. 3.4, Appendix D) through the
C ABI: the factor against the oracle (pivots bit-exact), preconditioned CIQ
against the oracle at fixed small J and at convergence, the rotation
identities R'^T K R' = I and (R B)^T (R' B) = B^T B at sizes without a dense
reference, fewer iterations than plain CIQ, and the graph loop."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import kernels as okern
from oracle import precond as opc
from scipy.linalg import eigh as geigh

pytestmark = pytest.mark.gpu


def _inputs(n, d, s, seed, dtype=np.float64, ard=False):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(dtype)
    b = rng.standard_normal((n, s)).astype(dtype)
    ls = list(np.exp(rng.uniform(np.log(0.2), np.log(0.6), d))) if ard else [0.3]
    return x, b, ls


@pytest.mark.parametrize("kind,n,d,rank,ard,xdt", [("rbf", 1000, 3, 50, False, np.float64),
                                                   ("matern52", 777, 5, 100, True, np.float64),
                                                   ("matern52", 4100, 6, 200, False, np.float32),
                                                   ("rbf", 300, 2, 300, False, np.float64)])
def test_pivoted_cholesky_parity(kind, n, d, rank, ard, xdt):
    """Pivots equal the oracle's exactly (both take the first largest
    residual diagonal; the FP64 entries differ by ~1 ulp, far below the gaps
    between candidates for these seeded points), each column to 1e-12 of the
    outputscale times its conditioning, the residual trace to 1e-9 relative.
    The last case stops at the numerical rank before 300 columns."""
    torch = torch_cuda()
    ciq = ciq_module()
    x, _, ls = _inputs(n, d, 1, n + rank, xdt, ard)
    o2 = 1.3
    announce(f"pivoted cholesky {kind} n={n} d={d} rank={rank} ard={ard}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, o2, 1e-3)
    L, piv, tr = ciq.ciq_pivoted_cholesky(prob, rank)
    torch.cuda.synchronize()
    Lo, pivo, dres = opc.pivoted_cholesky(kind, x.astype(np.float64), ls, o2, rank)
    m = len(pivo)
    assert np.array_equal(piv[:m], pivo)
    assert np.all(piv[m:] == -1)
    # column m divides by sqrt(d_p): rounding in its numerator grows by
    # sqrt(o2 / d_p), large once the factor nears the numerical rank
    Lg = L.cpu().numpy()
    for k in range(m):
        amp = max(1.0, np.sqrt(o2) / Lo[pivo[k], k])
        assert np.abs(Lg[:, k] - Lo[:, k]).max() <= 1e-12 * o2 * amp, k
    assert np.all(Lg[:, m:] == 0.0)
    assert abs(tr - dres.sum()) <= 1e-9 * max(dres.sum(), 1e-3 * o2)
    if kind == "rbf" and rank == 300:
        assert m < rank


def _oracle_setup(kind, x, ls, noise, rank):
    L, _, _ = opc.pivoted_cholesky(kind, x.astype(np.float64), ls, 1.0, rank)
    pre = opc.Preconditioner(L, noise)
    K = okern.kernel_matrix(kind, x.astype(np.float64), ls, 1.0, noise)
    return K, pre


class _Rounded:
    """The oracle's preconditioner built from a Gram matrix Lbar^T Lbar
    perturbed at its rounding scale (entry (r, c) by eps sqrt(G_rr G_cc), the
    size of sum_i |L_ir L_ic|). P^{-1} and P^{1/2} pass through that R x R
    matrix, whose condition number (with sigma^2 added) is ~||G|| / sigma^2,
    so any FP64 evaluation moves them by ~eps ||G|| / (lam + sigma^2)
    relative along the small eigenvalues."""

    def __init__(self, pre, rng):
        G = pre.gram
        E = rng.standard_normal(G.shape)
        E = (E + E.T) / np.sqrt(2.0)
        dg = np.sqrt(np.outer(np.diag(G), np.diag(G)))
        self.p = opc.Preconditioner(pre.L, pre.s2)
        self.p.gram = G + 2.2e-16 * dg * E
        self.p.lam, self.p.V = np.linalg.eigh(self.p.gram)
        self.p.lam = np.maximum(self.p.lam, 0.0)

    def sqrt(self, X):
        return self.p.sqrt(X)

    def inv(self, X):
        return self.p.inv(X)


@pytest.mark.parametrize("cache", ["on", "off"])
@pytest.mark.parametrize("J", [1, 3, 10])
@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_precond_small_j_parity_fp64(mode, J, cache):
    """FP64, fixed J before the Lanczos vectors lose orthogonality, the same
    bounds on both sides: GPU and oracle agree to rounding (the factors,
    the Gram eigendecompositions and the products round differently). The
    bar is 10x the oracle's own move under one-ulp perturbations of the
    entries of K and of the Gram matrix behind P (see _Rounded), and at
    least eps kappa(P) (the rounding scale of any evaluation of P^{-1} x)."""
    torch = torch_cuda()
    ciq = ciq_module()
    kind, n, d, s, rank, noise = "matern52", 2100, 4, 33, 100, 1e-3
    x, b, ls = _inputs(n, d, s, 7)
    K, pre = _oracle_setup(kind, x, ls, noise, rank)
    # the spectrum of A = P^{-1/2} K P^{-1/2} (a loose upper bound such as
    # lambda_max(K) / sigma^2 would put kappa ~ 5e5 into the shifts, where the
    # oracle's SciPy shifts carry ~eps kappa relative error of their own)
    gev = geigh(K, pre.dense(), eigvals_only=True)
    bounds = (gev[0], gev[-1])
    announce(f"precond small-J parity {mode} J={J} cache={cache}")
    fn = ciq.ciq_invsqrt_mvm if mode == "invsqrt" else ciq.ciq_sqrt_mvm
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.0, noise)
    out, info, solves = fn(prob, torch.from_numpy(b).cuda(), q=10, max_iter=J, tol=0.0, bounds=bounds,
                           keep_solves=True, kernel_cache=cache, precond_rank=rank)
    assert info["precond_rank"] == rank and info["iters"] == J
    ref, oinfo, t, w, X = opc.ciq_pc(lambda v: K @ v, pre, b, bounds[0], bounds[1], 10, J, 0.0, mode,
                                     return_solves=True)
    # the scale of rounding differences: how far the oracle's own result moves
    # when every entry of K is perturbed by one ulp (independently per entry)
    spread, spread_x = 0.0, 0.0
    for seed in range(2):
        rng = np.random.default_rng(100 + seed)
        E = rng.standard_normal(K.shape)
        Kp = K * (1.0 + 2.2e-16 * (E + E.T) / np.sqrt(2.0))
        alt, _, _, _, altX = opc.ciq_pc(lambda v: Kp @ v, _Rounded(pre, rng), b, bounds[0], bounds[1], 10, J, 0.0,
                                        mode, return_solves=True)
        spread = max(spread, colwise_rel(alt, ref).max())
        spread_x = max(spread_x, max(colwise_rel(altX[qi], X[qi]).max() for qi in range(10)))
    # floor: P^{-1} x is x / sigma^2 minus a low-rank correction, so any FP64
    # evaluation carries absolute errors ~eps |x| / sigma^2, i.e. relative
    # eps kappa(P) along the leading eigenvectors of P
    kappa_p = (pre.lam.max() + noise) / noise
    floor = max(2.2e-16 * kappa_p, 1e-11)
    bar, bar_x = max(10.0 * spread, floor), max(10.0 * spread_x, floor)
    gap = colwise_rel(out.cpu().numpy(), ref).max()
    sv = solves.cpu().numpy()
    gap_x = max(colwise_rel(sv[:, qi, :], X[qi]).max() for qi in range(10))
    print(f"gap {gap:.2e} bar {bar:.2e}; solves gap {gap_x:.2e} bar {bar_x:.2e}", flush=True)
    assert gap < bar, (gap, bar)
    assert gap_x < bar_x, (gap_x, bar_x)
    np.testing.assert_allclose(info["max_rel_residual"], oinfo.rel_residual.max(), rtol=1e-8)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,n,d,s,rank", [("rbf", 1500, 3, 8, 64), ("matern52", 3001, 5, 20, 151)])
def test_precond_converged_parity(kind, n, d, s, rank, prec):
    """At convergence (bounds from the library's own preconditioned Lanczos
    estimate): FP64 (sigma^2 = 1e-3, tol 1e-10) to 1e-7. FP32 products
    (sigma^2 = 1e-2, tol 1e-7) to 2e-4: FP32 entries with FP32 sums over
    64-column chunks give 4e-5 on these inputs in a CPU simulation, for plain
    and preconditioned CIQ alike (the error follows kappa(K), not kappa(A))."""
    torch = torch_cuda()
    ciq = ciq_module()
    noise = 1e-3 if prec == "f64" else 1e-2
    dt = np.float64 if prec == "f64" else np.float32
    x, b, ls = _inputs(n, d, s, n, dt)
    K, pre = _oracle_setup(kind, x, ls, noise, rank)
    announce(f"precond converged parity {kind} n={n} s={s} rank={rank} {prec}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.0, noise)
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, _ = fn(prob, torch.from_numpy(b).cuda(), q=15, max_iter=2000, tol=1e-10 if prec == "f64" else 1e-7,
                          precond_rank=rank)
        assert info["converged"], info["max_rel_residual"]
        gev = geigh(K, pre.dense(), eigvals_only=True)
        assert info["lambda_min"] <= gev[0] * (1 + 1e-9) and info["lambda_max"] >= 0.9 * gev[-1]
        ref, _ = opc.ciq_pc(lambda v: K @ v, pre, b.astype(np.float64), info["lambda_min"], info["lambda_max"], 15,
                            2000, 1e-12, mode)
        err = colwise_rel(out.cpu().numpy(), ref).max()
        print(f"{prec} {mode}: rel err {err:.3e}, iters {info['iters']}", flush=True)
        assert err < (1e-7 if prec == "f64" else 2e-4), (mode, err)


def test_precond_rotation_identities_and_fewer_iterations():
    """N = 8000 Matern-5/2 (d = 6, l = 0.3, sigma^2 = 1e-3, the large
    workload's kernel): A = R'B satisfies A^T K A = B^T B and
    (R B)^T A = B^T B (K applied by the FP64 product), and the preconditioned
    run (rank 200) needs fewer iterations than plain CIQ at the same tol."""
    torch = torch_cuda()
    ciq = ciq_module()
    kind, n, d, s, rank, noise = "matern52", 8000, 6, 16, 200, 1e-3
    x, b, ls = _inputs(n, d, s, 8000)
    announce(f"precond identities n={n} rank={rank}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.0, noise)
    bt = torch.from_numpy(b).cuda()
    kw = dict(q=15, max_iter=4000, tol=1e-9)
    a, ia, _ = ciq.ciq_invsqrt_mvm(prob, bt, precond_rank=rank, **kw)
    rb, ir, _ = ciq.ciq_sqrt_mvm(prob, bt, precond_rank=rank, **kw)
    plain, ip, _ = ciq.ciq_invsqrt_mvm(prob, bt, **kw)
    ka = ciq.ciq_kernel_mvm(prob, a)
    torch.cuda.synchronize()
    A, KA, RB = a.cpu().numpy(), ka.cpu().numpy(), rb.cpu().numpy()
    BtB = b.T @ b
    e1 = np.abs(A.T @ KA - BtB).max() / np.abs(BtB).max()
    e2 = np.abs(RB.T @ A - BtB).max() / np.abs(BtB).max()
    print(f"iters precond {ia['iters']} plain {ip['iters']}; identity errors {e1:.2e} {e2:.2e}", flush=True)
    assert ia["converged"] and ir["converged"] and ip["converged"]
    assert e1 < 1e-6 and e2 < 1e-6
    assert ia["iters"] < ip["iters"]
    # a genuine rotation: R'B is not K^{-1/2}B
    assert colwise_rel(A, plain.cpu().numpy()).max() > 1e-3


def test_precond_graph_equals_eager():
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, ls = _inputs(1200, 4, 8, 3, np.float32)
    announce("precond graph vs eager")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", ls, 1.0, 1e-2)
    kw = dict(q=8, max_iter=81, tol=1e-7, bounds=(1.0, 400.0), precond_rank=40, keep_solves=True)
    e_out, e_info, e_sol = ciq.ciq_invsqrt_mvm(prob, torch.from_numpy(b).cuda(), **kw)
    g_out, g_info, g_sol = ciq.ciq_invsqrt_mvm(prob, torch.from_numpy(b).cuda(), graph=True, **kw)
    torch.cuda.synchronize()
    assert g_info["iters"] == e_info["iters"]
    assert torch.equal(g_out, e_out) and torch.equal(g_sol, e_sol)


def test_precond_zero_and_ragged_columns():
    """A zero column stays zero; a column that stops early does not disturb
    the others (each column's result equals its single-column solve to the
    convergence tolerance: the products of different widths round
    differently)."""
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, ls = _inputs(999, 3, 5, 11)
    b[:, 2] = 0.0
    b[:, 4] *= 1e-3
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", ls, 1.0, 1e-2)
    announce("precond zero / ragged columns")
    kw = dict(q=10, max_iter=500, tol=1e-8, bounds=(1.0, 3e3), precond_rank=30, kernel_cache="off")
    out, info, _ = ciq.ciq_sqrt_mvm(prob, torch.from_numpy(b).cuda(), **kw)
    o = out.cpu().numpy()
    assert np.all(o[:, 2] == 0.0)
    for c in (0, 4):
        one, _, _ = ciq.ciq_sqrt_mvm(prob, torch.from_numpy(np.ascontiguousarray(b[:, c:c + 1])).cuda(), **kw)
        assert colwise_rel(o[:, c:c + 1], one.cpu().numpy()).max() < 1e-6


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3", "f32"])
def test_precond_other_products_and_rank_clamp(prec):
    """The preconditioned step is independent of the product's precision form:
    split BF16/FP16 products and the on-the-fly FP32 product (cache off) give
    results satisfying A^T K A = B^T B to their product accuracy; a rank above
    n is clamped to n (the factor then stops at the numerical rank)."""
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, ls = _inputs(1800, 5, 8, 31, np.float32)
    announce(f"precond product form {prec}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "matern52", ls, 1.0, 1e-2)
    bt = torch.from_numpy(b).cuda()
    a, info, _ = ciq.ciq_invsqrt_mvm(prob, bt, q=12, max_iter=2000, tol=1e-7, precond_rank=60,
                                     precision=prec, kernel_cache="off")
    assert info["converged"] and info["precond_rank"] == 60
    p64 = ciq.Problem(prob.x.double().contiguous(), "matern52", ls, 1.0, 1e-2)
    ka = ciq.ciq_kernel_mvm(p64, a.double().contiguous())
    torch.cuda.synchronize()
    A, KA = a.double().cpu().numpy(), ka.cpu().numpy()
    BtB = b.astype(np.float64).T @ b.astype(np.float64)
    err = np.abs(A.T @ KA - BtB).max() / np.abs(BtB).max()
    print(f"{prec}: identity error {err:.2e}, iters {info['iters']}", flush=True)
    assert err < {"f32": 1e-4, "f16x3": 1e-3, "bf16x3": 5e-3}[prec]
    if prec == "f32":
        xs, bs, _ = _inputs(90, 2, 3, 5, np.float64)
        ps = ciq.Problem(torch.from_numpy(xs).cuda(), "rbf", [0.5], 1.0, 1e-2)
        out, inf2, _ = ciq.ciq_invsqrt_mvm(ps, torch.from_numpy(bs).cuda(), q=10, max_iter=300, tol=1e-10,
                                           precond_rank=500)
        assert inf2["converged"] and 0 < inf2["precond_rank"] <= 90
        Ks = okern.kernel_matrix("rbf", xs, [0.5], 1.0, 1e-2)
        O = out.cpu().numpy()
        assert np.abs(O.T @ Ks @ O - bs.T @ bs).max() <= 1e-7 * np.abs(bs.T @ bs).max()
