"""ciq_svgp_predict (Sec. 5.1, App. E) against the oracle: the whitened
features a = Kzz^{-1/2} k_Zx (symmetric root), and the predictive mean and
variance from natural parameters."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import svgp as osv

pytestmark = pytest.mark.gpu


def _setup(M, nb, d, seed, dtype):
    rng = np.random.default_rng(seed)
    z = rng.random((M, d)).astype(dtype)
    x = rng.random((nb, d)).astype(dtype)
    m = rng.standard_normal(M) * 0.5
    G = rng.standard_normal((M, M)) / np.sqrt(M)
    S = G @ G.T * 0.3 + 0.2 * np.eye(M)
    theta, Theta = osv.natural_from_standard(m, S)
    return z, x, theta, Theta


@pytest.mark.parametrize("prec,M,nb,kind", [("f64", 700, 24, "matern52"), ("f32", 1100, 40, "rbf")])
def test_svgp_predict_against_oracle(prec, M, nb, kind):
    """FP64: CIQ at tol 1e-10 and the dense solve at 1e-12 give a, mean and
    var to 1e-7; FP32 products (CIQ at tol 1e-7): 1e-4 on a and the mean, the
    variance's absolute error 1e-4 of the outputscale."""
    torch = torch_cuda()
    ciq = ciq_module()
    dt = np.float64 if prec == "f64" else np.float32
    z, x, theta, Theta = _setup(M, nb, 3, M, dt)
    ls, o2, jit = [0.4], 1.2, 1e-3
    announce(f"svgp predict {prec} M={M} nb={nb} {kind}")
    prob = ciq.Problem(torch.from_numpy(z).cuda(), kind, ls, o2, jit)
    mean, var, a, info, info_s = ciq.ciq_svgp_predict(
        prob, torch.from_numpy(x).cuda(), torch.from_numpy(theta).cuda(), torch.from_numpy(Theta).cuda(), q=15,
        max_iter=3000, tol=1e-10 if prec == "f64" else 1e-7, solve_max_iter=2000, solve_tol=1e-12, want_a=True)
    torch.cuda.synchronize()
    mu_o, var_o, a_o, c_o = osv.predictive(kind, z.astype(np.float64), x.astype(np.float64), ls, o2, jit, theta,
                                           Theta)
    ea = colwise_rel(a.cpu().numpy(), a_o).max()
    em = np.abs(mean.cpu().numpy() - mu_o).max() / np.abs(mu_o).max()
    ev = np.abs(var.cpu().numpy() - var_o).max()
    print(f"{prec}: a {ea:.2e} mean {em:.2e} var(abs) {ev:.2e}; iters {info['iters']} solve {info_s['iters']}",
          flush=True)
    assert info["converged"] and info_s["converged"]
    bar = 1e-7 if prec == "f64" else 1e-4
    assert ea < bar and em < bar and ev < bar * o2


@pytest.mark.parametrize("M,nb", [(700, 24), (1001, 37), (64, 1)])
def test_ngd_step_against_oracle(M, nb):
    """ciq_svgp_ngd_step against the oracle's App. E step (FP64; the rank-nb
    Theta update on MFMA sums in another order: 1e-12 of the largest entry)."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(M + nb)
    _, _, theta, Theta = _setup(M, 2, 3, M + 1, np.float64)
    a = rng.standard_normal((M, nb)) / np.sqrt(M)
    mean = rng.standard_normal(nb)
    cm, cv = rng.standard_normal(nb), -np.abs(rng.standard_normal(nb))
    scale, step = 37.0, 0.3
    announce(f"svgp ngd step M={M} nb={nb}")
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    th, Th = dev(theta), dev(Theta)
    ciq.ciq_svgp_ngd_step(dev(a), dev(mean), dev(cm), dev(cv), th, Th, scale, step)
    th_o, Th_o = osv.ngd_step(theta, Theta, a, mean, cm, cv, scale, step)
    assert np.abs(Th.cpu().numpy() - Th_o).max() <= 1e-12 * np.abs(Th_o).max()
    assert np.abs(th.cpu().numpy() - th_o).max() <= 1e-12 * np.abs(th_o).max()


def test_svgp_predict_m10000_subset():
    """The SVGP measurement workload's size (M = 10,000 inducing points in
    [0,1]^10, RBF-ARD, jitter 1e-4) on 4 test points: GPU FP64 path with the
    oracle's own Lanczos bounds, CIQ to 1e-10, against the oracle's
    msMINRES-CIQ on the dense FP64 Kzz (same bounds and tolerance) and its
    exact solve with -2 Theta (1e-7)."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    from oracle import ciq as ociq
    from oracle import kernels as okern
    from oracle import lanczos as olz
    from oracle import posterior as opost
    p = workloads.workload(5).problems[0]
    M, nb = 10000, 4
    rng = np.random.default_rng(8001)
    z = rng.random((M, p.d))
    x = rng.random((nb, p.d))
    H = rng.standard_normal((M, 16))
    Theta = -0.5 * (np.eye(M) + H @ H.T / 16)
    theta = rng.standard_normal(M)
    Kzz = okern.kernel_matrix(p.kernel, z, p.lengthscale, p.outputscale, p.noise)
    lo, hi, _, _ = olz.eig_bounds(lambda v: Kzz @ v, workloads.start_vector(M, 5004, np.float64), 20, p.noise)
    Kzx = opost.cross_kernel(p.kernel, z, x, p.lengthscale, p.outputscale)
    a_o, _ = ociq.ciq(lambda v: Kzz @ v, Kzx, lo, hi, 15, 3000, 1e-10, "invsqrt")
    mu_o, var_o, _, _ = osv.predictive(p.kernel, z, x, p.lengthscale, p.outputscale, p.noise, theta, Theta, a=a_o)
    announce("svgp predict f64 M=10000 nb=4 vs oracle")
    prob = ciq.Problem(torch.from_numpy(z).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
    mean, var, a, info, info_s = ciq.ciq_svgp_predict(
        prob, torch.from_numpy(x).cuda(), torch.from_numpy(theta).cuda(), torch.from_numpy(Theta).cuda(), q=15,
        max_iter=3000, tol=1e-10, bounds=(lo, hi), solve_max_iter=3000, solve_tol=1e-12, want_a=True)
    ea = colwise_rel(a.cpu().numpy(), a_o).max()
    em = np.abs(mean.cpu().numpy() - mu_o).max() / np.abs(mu_o).max()
    ev = np.abs(var.cpu().numpy() - var_o).max()
    print(f"M=10000: a {ea:.2e} mean {em:.2e} var(abs) {ev:.2e}; iters {info['iters']} solve {info_s['iters']}",
          flush=True)
    assert info["converged"] and info_s["converged"]
    assert ea < 1e-7 and em < 1e-7 and ev < 1e-7 * p.outputscale


def test_whitening_workload_forward_parity():
    """K^{-1/2} B of the SVGP whitening workload (M = 5,000 inducing points in
    [0,1]^10, RBF-ARD, jitter 1e-4), first 8 of its 256 columns: the FP64 path
    against the oracle's msMINRES-CIQ (same bounds, tol 1e-10; 1e-8), and the
    FP32 path at the workload's tol 1e-3 against the exact root (the
    method's error at that tolerance, bounded by 1e-2)."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    from oracle import ciq as ociq
    from oracle import kernels as okern
    from oracle import lanczos as olz
    wl = workloads.workload(5)
    p = wl.problems[0]
    k = 8
    x64, b64 = p.x.astype(np.float64), p.b[:, :k].astype(np.float64)
    K = okern.kernel_matrix(p.kernel, x64, p.lengthscale, p.outputscale, p.noise)
    lo, hi, _, _ = olz.eig_bounds(lambda v: K @ v, workloads.start_vector(p.n, 5004, np.float64), 20, p.noise)
    ref, _ = ociq.ciq(lambda v: K @ v, b64, lo, hi, wl.q, 5000, 1e-10, "invsqrt")
    announce("whitening workload forward parity M=5000")
    prob64 = ciq.Problem(torch.from_numpy(x64).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
    out, info, _ = ciq.ciq_invsqrt_mvm(prob64, torch.from_numpy(b64).cuda(), q=wl.q, max_iter=5000, tol=1e-10,
                                       bounds=(lo, hi))
    gap = colwise_rel(out.cpu().numpy(), ref).max()
    exact = ociq.exact_power(K, b64, -0.5)
    prob32 = ciq.Problem(torch.from_numpy(p.x).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
    out32, info32, _ = ciq.ciq_invsqrt_mvm(prob32, torch.from_numpy(p.b).cuda(), q=wl.q, max_iter=wl.max_iter,
                                           tol=wl.tol)
    err32 = colwise_rel(out32[:, :k].cpu().numpy(), exact).max()
    print(f"M=5000: FP64 vs oracle {gap:.2e} ({info['iters']} it); FP32 tol {wl.tol:g} vs exact {err32:.2e} "
          f"({info32['iters']} it)", flush=True)
    assert info["converged"] and gap < 1e-8
    assert err32 < 1e-2
