"""Parity of the HIP kernel product Y = K V (ciq_kernel_mvm, through the C ABI)
with the oracle's FP64 K V, over tile-spanning ragged shapes and, at full
size, on sampled rows."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import kernels as okern

pytestmark = pytest.mark.gpu


# relative error bars per precision form: FP64 rounding; FP32 entry rounding;
# split forms: 2^-16 (BF16 hi + lo); FP16 hi + lo keeps ~22 bits for entries
# in its normal range but fewer below 6.1e-5 (its subnormals), which many
# entries of high-dimensional Matern rows are
MVM_TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 5e-5, "f16x3": 2e-5}


def _case(n, d, s, kind, ls, seed, dtype):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(dtype)
    v = rng.standard_normal((n, s)).astype(dtype)
    return x, v


@pytest.mark.parametrize("kind", ["rbf", "matern52"])
@pytest.mark.parametrize("n,d,s", [(1, 1, 1), (17, 3, 1), (100, 6, 5), (257, 8, 16), (1000, 10, 33),
                                   (700, 16, 64), (300, 2, 100), (130, 5, 300)])
@pytest.mark.parametrize("prec", ["f32", "f64", "bf16x3", "f16x3"])
def test_mvm_matches_oracle(kind, n, d, s, prec):
    torch = torch_cuda()
    ciq = ciq_module()
    dt = np.float64 if prec == "f64" else np.float32
    x, v = _case(n, d, s, kind, 0.3, n * 7 + d, dt)
    ls = np.linspace(0.2, 0.9, d) if d > 1 else np.array([0.4])
    announce(f"mvm {prec} {kind} n={n} d={d} s={s}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.7, 0.05)
    y = ciq.ciq_kernel_mvm(prob, torch.from_numpy(v).cuda(), precision=prec).cpu().numpy()
    torch.cuda.synchronize()
    K = okern.kernel_matrix(kind, x.astype(np.float64), ls, 1.7, 0.05)
    ref = K @ v.astype(np.float64)
    err = colwise_rel(y, ref).max()
    assert err < MVM_TOL[prec], err


def test_mvm_isotropic_and_ldv():
    torch = torch_cuda()
    ciq = ciq_module()
    x, v = _case(333, 4, 24, "rbf", 0.3, 5, np.float32)
    announce("mvm strided ld n=333 s=20 of 24")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", [0.25], 0.8, 1e-3)
    vt = torch.from_numpy(v).cuda()
    y = ciq.ciq_kernel_mvm(prob, vt[:, :20]).cpu().numpy()   # ldv = 24 > s = 20
    K = okern.kernel_matrix("rbf", x.astype(np.float64), [0.25], 0.8, 1e-3)
    assert colwise_rel(y, K @ v[:, :20].astype(np.float64)).max() < 2e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("kind,n,d,s", [("matern52", 50_000, 6, 64), ("rbf", 100_000, 8, 256)])
def test_mvm_full_size_sampled_rows(kind, n, d, s, prec):
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    c = 2 if kind == "matern52" else 3
    wl = workloads.workload(c)
    p = wl.problems[0]
    dt = np.float64 if prec == "f64" else np.float32
    announce(f"mvm full size {prec} {kind} n={n} s={s}")
    prob = ciq.Problem(torch.from_numpy(p.x.astype(dt)).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
    b = torch.from_numpy(p.b.astype(dt)).cuda()
    y = ciq.ciq_kernel_mvm(prob, b).cpu().numpy()
    rows = np.random.default_rng(1).choice(n, 48, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    Kr = okern.kernel_rows(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise, rows)
    ref = Kr @ p.b.astype(np.float64)
    rel = np.linalg.norm(y[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert rel.max() < (1e-12 if prec == "f64" else 1e-5), rel.max()
