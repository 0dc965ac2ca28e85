"""Full-size (N = 50,000, Matern-5/2, d = 6) accuracy of the FP32 path at the
benchmark's settings. The oracle cannot run msMINRES at this size, so the
checks are (i) a property that holds at any size, K^{-1/2} (K^{1/2} b) = b,
and (ii) the FP32 result against the library's FP64 path run to a much
tighter tolerance (the FP64 path is held to the oracle at smaller sizes)."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda

pytestmark = pytest.mark.gpu


def _problem(ciq, torch, dtype, s):
    import workloads
    wl = workloads.workload(2, s=s)
    p = wl.problems[0]
    x = torch.from_numpy(p.x.astype(dtype)).cuda()
    b = torch.from_numpy(p.b.astype(dtype)).cuda()
    return wl, ciq.Problem(x, p.kernel, p.lengthscale, p.outputscale, p.noise), b


def test_round_trip_full_size():
    torch = torch_cuda()
    ciq = ciq_module()
    wl, prob, b = _problem(ciq, torch, np.float32, 4)
    announce("full-size round trip f32 n=50000 s=4")
    half, i1, _ = ciq.ciq_sqrt_mvm(prob, b, q=15, max_iter=4000, tol=1e-5, seed=4001)
    back, i2, _ = ciq.ciq_invsqrt_mvm(prob, half, q=15, max_iter=4000, tol=1e-5, seed=4001)
    err = colwise_rel(back.cpu().numpy(), b.cpu().numpy()).max()
    print(f"round trip rel err {err:.3e} iters {i1['iters']} {i2['iters']}", flush=True)
    assert i1["converged"] and i2["converged"]
    assert err < 1e-4


def test_fp32_at_bench_settings_vs_fp64_full_size():
    torch = torch_cuda()
    ciq = ciq_module()
    wl, p32, b32 = _problem(ciq, torch, np.float32, 4)
    _, p64, b64 = _problem(ciq, torch, np.float64, 4)
    announce("full-size f32 (tol 1e-4) vs f64 (tol 1e-9) n=50000 s=4")
    bounds = None
    out32, i32, _ = ciq.ciq_invsqrt_mvm(p32, b32, q=15, max_iter=4000, tol=wl.tol, seed=4001)
    bounds = (i32["lambda_min"], i32["lambda_max"])
    out64, i64, _ = ciq.ciq_invsqrt_mvm(p64, b64, q=15, max_iter=6000, tol=1e-9, bounds=bounds)
    err = colwise_rel(out32.cpu().numpy(), out64.cpu().numpy()).max()
    print(f"f32 vs f64 rel err {err:.3e} iters {i32['iters']} vs {i64['iters']}", flush=True)
    assert i32["converged"] and i64["converged"]
    assert err < 1e-4
