"""ciq_kernel_mvm_noalloc through the C ABI: the allocation-free kernel product
(static device scratch) gives exactly ciq_kernel_mvm's result -- same kernels,
same launch configuration -- on consecutive calls of decreasing size, and
rejects a request larger than its scratch before any device work."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import kernels as okern

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64", "f16x3"])
def test_noalloc_matches_kernel_mvm_twice(prec):
    torch = torch_cuda()
    ciq = ciq_module()
    dt = np.float64 if prec == "f64" else np.float32
    tdt = torch.float64 if prec == "f64" else torch.float32
    # second call smaller than the first: the scratch keeps the first call's
    # contents, which must not leak into the second result
    for n, d, s, kind in [(5000, 6, 20, "matern52"), (777, 3, 5, "rbf")]:
        rng = np.random.default_rng(n + s)
        x = rng.random((n, d)).astype(dt)
        v = rng.standard_normal((n, s)).astype(dt)
        announce(f"noalloc mvm {prec} {kind} n={n} d={d} s={s}")
        prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, [0.35], 1.3, 0.02)
        vt = torch.from_numpy(v).cuda()
        ref = ciq.ciq_kernel_mvm(prob, vt, precision=prec)
        y = torch.full((n, s), float("nan"), dtype=tdt, device="cuda")
        ciq.ciq_kernel_mvm_noalloc(prob, vt, y, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (prec, n, s)
        K = okern.kernel_matrix(kind, x.astype(np.float64), [0.35], 1.3, 0.02)
        err = colwise_rel(y.cpu().numpy(), K @ v.astype(np.float64)).max()
        assert err < {"f64": 1e-12, "f32": 1e-6, "f16x3": 2e-5}[prec], err


def test_noalloc_rejects_oversize():
    torch = torch_cuda()
    ciq = ciq_module()
    import paper_2006_11267_amd._lib as L
    n, s = 50_000, 64           # FP64 partials alone exceed the 64 MiB scratch
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.random((n, 6)).astype(np.float32)).cuda()
    v = torch.ones((n, s), dtype=torch.float32, device="cuda")
    y = torch.zeros((n, s), dtype=torch.float32, device="cuda")
    announce("noalloc mvm oversize n=50000 s=64")
    prob = ciq.Problem(x, "matern52", [0.3], 1.0, 1e-3)
    with pytest.raises(L.CIQError) as ei:
        ciq.ciq_kernel_mvm_noalloc(prob, v, y)
    assert ei.value.status == L.CIQ_EINVAL
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0
