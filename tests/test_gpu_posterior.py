"""Posterior-covariance roots (Sec. 5.2, Thompson sampling) through
ciq_posterior_mvm against the oracle: fixed small J and converged runs, on
resident and on-the-fly candidate products, and a full-size round trip."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import ciq as oc
from oracle import posterior as opost

pytestmark = pytest.mark.gpu


def _inputs(t, n, d, s, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    xs = rng.random((t, d)).astype(dtype)
    xo = rng.random((n, d)).astype(dtype)
    b = rng.standard_normal((t, s)).astype(dtype)
    return xs, xo, b


@pytest.mark.parametrize("cache", ["on", "off"])
@pytest.mark.parametrize("J", [1, 5])
@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_posterior_small_j_parity_fp64(mode, J, cache):
    """FP64, same bounds, fixed J: agreement to rounding. The bar is 10x the
    oracle's own move when the entries of Sigma are perturbed at their
    rounding scale (eps times |Kss| + |W W^T|, the two terms Sigma is the
    difference of)."""
    torch = torch_cuda()
    ciq = ciq_module()
    t, n, d, s = 1500, 121, 4, 7                     # odd n: odd leading dimension of W
    kind, ls, o2, jit, s2 = "matern52", [0.35], 1.0, 1e-3, 1e-3
    xs, xo, b = _inputs(t, n, d, s, 11)
    S = opost.posterior_covariance(kind, xs, xo, ls, o2, jit, s2)
    Kss = opost.cross_kernel(kind, xs, xs, ls, o2)
    lam = np.linalg.eigvalsh(S)
    bounds = (lam[0], lam[-1])
    announce(f"posterior small-J parity {mode} J={J} cache={cache}")
    prob = ciq.Problem(torch.from_numpy(xs).cuda(), kind, ls, o2, jit)
    out, info = ciq.ciq_posterior_mvm(prob, torch.from_numpy(xo).cuda(), s2, torch.from_numpy(b).cuda(), mode=mode,
                                      q=10, max_iter=J, tol=0.0, bounds=bounds, kernel_cache=cache)
    ref, oinfo = oc.ciq(lambda v: S @ v, b, bounds[0], bounds[1], 10, J, 0.0, mode)
    assert info["iters"] == J and info["kernel_cached"] == (cache == "on")
    mag = np.abs(Kss) + np.abs(Kss + jit * np.eye(t) - S)
    spread = 0.0
    for seed in range(2):
        E = np.random.default_rng(50 + seed).standard_normal(S.shape)
        Sp = S + 2.2e-16 * mag * (E + E.T) / np.sqrt(2.0)
        alt, _ = oc.ciq(lambda v: Sp @ v, b, bounds[0], bounds[1], 10, J, 0.0, mode)
        spread = max(spread, colwise_rel(alt, ref).max())
    bar = max(10.0 * spread, 1e-11)
    gap = colwise_rel(out.cpu().numpy(), ref).max()
    print(f"gap {gap:.2e} bar {bar:.2e}", flush=True)
    assert gap < bar


@pytest.mark.parametrize("n_obs", [1, 63, 64, 65, 130, 257])
def test_posterior_observation_counts(n_obs):
    """The device factors of the observation block (64-column panels, the
    block padded with the identity) at counts below, at, just above and
    across panel boundaries: converged FP64 K^{1/2}-root against the oracle's
    CIQ on the dense Sigma (the textbook posterior covariance) with the same
    bounds, to 1e-8."""
    torch = torch_cuda()
    ciq = ciq_module()
    t, d, s = 700, 3, 5
    kind, ls, o2, jit, s2 = "rbf", [0.3], 1.1, 1e-2, 1e-3
    xs, xo, b = _inputs(t, n_obs, d, s, 100 + n_obs)
    S = opost.posterior_covariance(kind, xs, xo, ls, o2, jit, s2)
    lam = np.linalg.eigvalsh(S)
    bounds = (lam[0], lam[-1])
    announce(f"posterior observation count n_obs={n_obs}")
    prob = ciq.Problem(torch.from_numpy(xs).cuda(), kind, ls, o2, jit)
    out, info = ciq.ciq_posterior_mvm(prob, torch.from_numpy(xo).cuda(), s2, torch.from_numpy(b).cuda(),
                                      mode="sqrt", q=12, max_iter=2000, tol=1e-11, bounds=bounds)
    assert info["converged"] and info["setup_ms"] > 0.0
    ref, _ = oc.ciq(lambda v: S @ v, b, bounds[0], bounds[1], 12, 2000, 1e-12, "sqrt")
    err = colwise_rel(out.cpu().numpy(), ref).max()
    print(f"n_obs={n_obs}: rel err {err:.2e}, iters {info['iters']}, set-up {info['setup_ms']:.1f} ms", flush=True)
    assert err < 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_posterior_converged_parity(prec):
    """Converged (library bounds), FP64 to 1e-7, FP32 products to 2e-4, both
    modes, against the oracle's CIQ on the dense Sigma with the same bounds."""
    torch = torch_cuda()
    ciq = ciq_module()
    t, n, d, s = 2500, 200, 5, 6
    kind, ls, o2, jit, s2 = "rbf", [0.3], 1.3, 1e-2, 1e-3
    dt = np.float64 if prec == "f64" else np.float32
    xs, xo, b = _inputs(t, n, d, s, 12, dt)
    S = opost.posterior_covariance(kind, xs.astype(np.float64), xo.astype(np.float64), ls, o2, jit, s2)
    announce(f"posterior converged parity {prec}")
    prob = ciq.Problem(torch.from_numpy(xs).cuda(), kind, ls, o2, jit)
    for mode in ("invsqrt", "sqrt"):
        out, info = ciq.ciq_posterior_mvm(prob, torch.from_numpy(xo).cuda(), s2, torch.from_numpy(b).cuda(),
                                          mode=mode, q=15, max_iter=3000,
                                          tol=1e-10 if prec == "f64" else 1e-7)
        assert info["converged"]
        lam = np.linalg.eigvalsh(S)
        assert info["lambda_min"] <= lam[0] * (1 + 1e-6) and info["lambda_max"] >= 0.9 * lam[-1]
        ref, _ = oc.ciq(lambda v: S @ v, b.astype(np.float64), info["lambda_min"], info["lambda_max"], 15, 3000,
                        1e-12, mode)
        err = colwise_rel(out.cpu().numpy(), ref).max()
        print(f"{prec} {mode}: rel err {err:.2e}, iters {info['iters']}", flush=True)
        assert err < (1e-7 if prec == "f64" else 2e-4)


def test_posterior_full_size_round_trip():
    """T = 50,000 candidates (the large workload's points and kernel, jitter
    1e-3), 1,000 observations, FP64 resident products: Sigma^{-1/2}
    (Sigma^{1/2} b) = b to 1e-4 (a property of any size). Sigma is a
    difference Kss - W W^T whose smallest eigenvalues (the jitter) sit far
    below the size of its terms, so its FP32 products carry ~1e-4 relative
    error there; the FP32 path's error against this FP64 one is measured by
    the benchmark's posterior workload."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(2, s=4)
    p = wl.problems[0]
    xo = np.random.default_rng(2007).random((1000, p.d))
    announce("posterior full size round trip f64 T=50000 n_obs=1000 s=4")
    prob = ciq.Problem(torch.from_numpy(p.x.astype(np.float64)).cuda(), p.kernel, p.lengthscale, p.outputscale,
                       p.noise)
    xo_t = torch.from_numpy(xo).cuda()
    b = torch.from_numpy(p.b.astype(np.float64)).cuda()
    kw = dict(q=15, max_iter=6000, tol=5e-6, seed=4001)
    half, i1 = ciq.ciq_posterior_mvm(prob, xo_t, 1e-3, b, mode="sqrt", **kw)
    back, i2 = ciq.ciq_posterior_mvm(prob, xo_t, 1e-3, half, mode="invsqrt", **kw)
    err = colwise_rel(back.cpu().numpy(), b.cpu().numpy()).max()
    print(f"round trip rel err {err:.2e} iters {i1['iters']} {i2['iters']} bounds {i1['lambda_min']:.3g} "
          f"{i1['lambda_max']:.4g}", flush=True)
    assert i1["converged"] and i2["converged"] and i1["kernel_cached"]
    assert err < 1e-4
