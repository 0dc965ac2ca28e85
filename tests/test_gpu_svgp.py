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
