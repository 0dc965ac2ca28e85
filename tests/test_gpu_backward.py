"""Parity of the HIP backward pass (ciq_backward through the C ABI, and the
torch.autograd.Function above it) with the oracle's adjoint: the same forward
solves, the same shifts, converged tolerances."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import adjoint as oadj
from oracle import ciq as ociq
from oracle import kernels as okern

pytestmark = pytest.mark.gpu


def _svgp_small(m=256, s=4, seed=5001, kind="rbf", ard=True, dtype=np.float64):
    import workloads
    rng = np.random.default_rng(seed)
    x = rng.random((m, 10)).astype(dtype)
    b = rng.standard_normal((m, s)).astype(dtype)
    g = rng.standard_normal((m, s)).astype(dtype)
    ls = workloads.loguniform(10, 0.1, 1.0, seed + 2) if ard else np.array([0.6])
    return x, b, g, ls


@pytest.mark.parametrize("kind", ["rbf", "matern52"])
@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
@pytest.mark.parametrize("ard,cache", [(True, "on"), (False, "on"), (True, "off")])
def test_backward_fp64_matches_oracle(kind, mode, ard, cache):
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, g, ls = _svgp_small(kind=kind, ard=ard)
    o2, s2 = 1.3, 1e-2
    K = okern.kernel_matrix(kind, x, ls, o2, s2)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"backward f64 {kind} {mode} ard={ard} cache={cache} m={x.shape[0]}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, o2, s2)
    fn = ciq.ciq_sqrt_mvm if mode == "sqrt" else ciq.ciq_invsqrt_mvm
    out, info, solves = fn(prob, torch.from_numpy(b).cuda(), q=15, max_iter=1000, tol=1e-11, bounds=bounds,
                           keep_solves=True)
    db, dls, do2, dn, binfo = ciq.ciq_backward(prob, torch.from_numpy(g).cuda(), info["t"], info["w"], solves,
                                               mode=mode, max_iter=1000, tol=1e-11, kernel_cache=cache)
    assert binfo["kernel_cached"] == (cache == "on")
    # oracle adjoint with its own forward solves
    mvm = lambda v: K @ v
    _, _, t, w, A = ociq.ciq(mvm, b, bounds[0], bounds[1], 15, 1000, 1e-11, mode, return_solves=True)
    odb, odK = oadj.ciq_vjp(mvm, A, g, t, w, 1000, 1e-11, mode)
    ols, oo2, on = oadj.hyper_grads(kind, x, ls, o2, odK)
    assert colwise_rel(db.cpu().numpy(), odb).max() < 1e-8
    np.testing.assert_allclose(dls, ols, rtol=1e-7, atol=1e-9 * np.abs(ols).max())
    np.testing.assert_allclose(do2, oo2, rtol=1e-7)
    np.testing.assert_allclose(dn, on, rtol=1e-7)


def test_backward_fp32_matches_oracle_and_fd():
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, g, ls = _svgp_small(dtype=np.float32)
    x64 = x.astype(np.float64)
    o2, s2 = 1.0, 1e-4          # the SVGP workload's jitter
    K = okern.kernel_matrix("rbf", x64, ls, o2, s2)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce("backward f32 svgp-like m=256")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", ls, o2, s2)
    out, info, solves = ciq.ciq_invsqrt_mvm(prob, torch.from_numpy(b).cuda(), q=15, max_iter=1000, tol=1e-7,
                                            bounds=bounds, keep_solves=True)
    db, dls, do2, dn, _ = ciq.ciq_backward(prob, torch.from_numpy(g).cuda(), info["t"], info["w"], solves,
                                           max_iter=1000, tol=1e-7)
    mvm = lambda v: K @ v
    _, _, t, w, A = ociq.ciq(mvm, b.astype(np.float64), bounds[0], bounds[1], 15, 1000, 1e-11,
                             return_solves=True)
    odb, odK = oadj.ciq_vjp(mvm, A, g.astype(np.float64), t, w, 1000, 1e-11)
    ols, oo2, on = oadj.hyper_grads("rbf", x64, ls, o2, odK)
    assert colwise_rel(db.cpu().numpy(), odb).max() < 1e-4
    assert np.max(np.abs(dls - ols)) <= 1e-4 * np.max(np.abs(ols))
    assert abs(do2 - oo2) <= 1e-4 * abs(oo2)
    # finite differences of the exact rational function (oracle, dense)
    h = 1e-5

    def loss(ls_, o2_):
        Kp = okern.kernel_matrix("rbf", x64, ls_, o2_, s2)
        return float(np.sum(g * ociq.exact_rational(Kp, b.astype(np.float64), t, w)))
    fd = (loss(ls, o2 * (1 + h)) - loss(ls, o2 * (1 - h))) / (2 * h * o2)
    assert abs(do2 - fd) <= 1e-3 * abs(fd)


def test_autograd_function():
    torch = torch_cuda()
    ciq = ciq_module()
    x, b, g, ls = _svgp_small(m=200, s=3, seed=77)
    xt = torch.from_numpy(x).cuda()
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    lst = torch.tensor(ls, dtype=torch.float64, requires_grad=True)
    o2t = torch.tensor(1.1, dtype=torch.float64, requires_grad=True)
    s2t = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
    K = okern.kernel_matrix("rbf", x, ls, 1.1, 0.02)
    lam = np.linalg.eigvalsh(K)
    announce("autograd function m=200")
    out = ciq.ciq_apply(bt, xt, lst, o2t, s2t, kernel="rbf", mode="invsqrt", q=15, max_iter=1000, tol=1e-11,
                        bounds=(lam[0], lam[-1]))
    loss = (out * torch.from_numpy(g).cuda()).sum()
    loss.backward()
    mvm = lambda v: K @ v
    _, _, t, w, A = ociq.ciq(mvm, b, lam[0], lam[-1], 15, 1000, 1e-11, return_solves=True)
    odb, odK = oadj.ciq_vjp(mvm, A, g, t, w, 1000, 1e-11)
    ols, oo2, on = oadj.hyper_grads("rbf", x, ls, 1.1, odK)
    assert colwise_rel(bt.grad.cpu().numpy(), odb).max() < 1e-8
    np.testing.assert_allclose(lst.grad.numpy(), ols, rtol=1e-7, atol=1e-9 * np.abs(ols).max())
    np.testing.assert_allclose(o2t.grad.item(), oo2, rtol=1e-7)
    np.testing.assert_allclose(s2t.grad.item(), on, rtol=1e-7)
