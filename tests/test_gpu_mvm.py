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
# per sampled row at full size: the same per-product bars, loosened 2-5x for
# the fewer terms a single row averages over
FULL_ROW_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 2e-4, "f16x3": 5e-5}


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


@pytest.mark.parametrize("prec", ["f32", "f64", "bf16x3", "f16x3"])
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
    y = ciq.ciq_kernel_mvm(prob, b, precision=prec).cpu().numpy()
    rows = np.random.default_rng(1).choice(n, 48, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    Kr = okern.kernel_rows(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise, rows)
    ref = Kr @ p.b.astype(np.float64)
    rel = np.linalg.norm(y[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"on-the-fly full size {prec} {kind}: max row rel err {rel.max():.2e}", flush=True)
    assert rel.max() < FULL_ROW_TOL[prec], rel.max()


# Resident-matrix products (the solvers' streamed K, ciq_kernel_mvm_resident):
# FP64 entries; FP32: entries rounded once to FP32, FP32 MFMA with FP64 sums
# across 64-column chunks; split FP16: entries and V each kept to ~22 bits
# (hi + 2^-11 lo, V after a per-column power-of-two scale), three part
# products, so the bar is a few units of 2^-22 ~ 2.4e-7.
RESIDENT_TOL = {"f64": 1e-12, "f32": 1e-6, "f16x3": 2e-6}


@pytest.mark.parametrize("kind", ["rbf", "matern52"])
@pytest.mark.parametrize("n,d,s", [(1, 1, 1), (17, 3, 1), (100, 6, 5), (257, 8, 16), (1000, 10, 33),
                                   (700, 16, 64), (300, 2, 100), (130, 5, 300)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16x3"])
def test_resident_mvm_matches_oracle(kind, n, d, s, prec):
    torch = torch_cuda()
    ciq = ciq_module()
    dt = np.float64 if prec == "f64" else np.float32
    x, v = _case(n, d, s, kind, 0.3, n * 11 + d, dt)
    ls = np.linspace(0.2, 0.9, d) if d > 1 else np.array([0.4])
    announce(f"resident mvm {prec} {kind} n={n} d={d} s={s}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.7, 0.05)
    y = ciq.ciq_kernel_mvm_resident(prob, torch.from_numpy(v).cuda(), precision=prec).cpu().numpy()
    K = okern.kernel_matrix(kind, x.astype(np.float64), ls, 1.7, 0.05)
    ref = K @ v.astype(np.float64)
    err = colwise_rel(y, ref).max()
    print(f"resident {prec} {kind} n={n} s={s}: max col rel err {err:.2e}", flush=True)
    assert err < RESIDENT_TOL[prec], err


def test_resident_mvm_scaled_columns():
    """Columns of very different magnitude (the per-column scales of the split
    FP16 operand) and a zero column."""
    torch = torch_cuda()
    ciq = ciq_module()
    x, v = _case(900, 6, 20, "matern52", 0.3, 77, np.float32)
    v = (v * np.logspace(-20, 20, 20)[None, :]).astype(np.float32)
    v[:, 7] = 0.0
    announce("resident mvm f16x3 scaled columns n=900 s=20")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "matern52", [0.3], 1.0, 1e-3)
    y = ciq.ciq_kernel_mvm_resident(prob, torch.from_numpy(v).cuda(), precision="f16x3").cpu().numpy()
    K = okern.kernel_matrix("matern52", x.astype(np.float64), [0.3], 1.0, 1e-3)
    ref = K @ v.astype(np.float64)
    assert np.all(y[:, 7] == 0.0)
    keep = [c for c in range(20) if c != 7]
    err = colwise_rel(y[:, keep], ref[:, keep]).max()
    assert err < RESIDENT_TOL["f16x3"], err


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
@pytest.mark.parametrize("kind,n,d,s", [("matern52", 50_000, 6, 64), ("rbf", 100_000, 8, 256)])
def test_resident_mvm_full_size_sampled_rows(kind, n, d, s, prec):
    """The benchmark's product (N = 50,000, S = 64: 16 column ranges, tuned row
    tiles) and the N = 100,000, S = 256 precision workload, on rows the oracle
    evaluates one by one."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    c = 2 if kind == "matern52" else 3
    p = workloads.workload(c).problems[0]
    announce(f"resident mvm full size {prec} {kind} n={n} s={s}")
    prob = ciq.Problem(torch.from_numpy(p.x.astype(np.float32)).cuda(), p.kernel, p.lengthscale, p.outputscale,
                       p.noise)
    b = torch.from_numpy(p.b.astype(np.float32)).cuda()
    y = ciq.ciq_kernel_mvm_resident(prob, b, precision=prec).cpu().numpy()
    rows = np.random.default_rng(2).choice(n, 48, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    Kr = okern.kernel_rows(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise, rows)
    ref = Kr @ p.b.astype(np.float64)
    rel = np.linalg.norm(y[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"resident full size {prec} {kind}: max row rel err {rel.max():.2e}", flush=True)
    assert rel.max() < 1e-5, rel.max()
