"""Full-size (N = 50,000, Matern-5/2, d = 6, kappa ~ 2.5e6) accuracy at the
benchmark's settings. The checks are (i) the benchmark's path and the FP64
path against the CPU FP64 oracle's K^{+-1/2}B for the first 8 columns
(msMINRES-CIQ to relative residual 1e-10 on the dense FP64 kernel matrix,
written once by tests/golden/make_matern52_n50000_reference.py), (ii) a
property that holds at any size, K^{-1/2} (K^{1/2} b) = b, and (iii) the
result against the library's FP64 path run to tol 1e-9.

At this conditioning a MINRES stopping tolerance of 1e-4 leaves ~1.5e-4
(K^{-1/2}B) and ~4e-4 (K^{1/2}B) relative error; the benchmark stops at 5e-6,
which these tests hold to 1e-4."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda

pytestmark = pytest.mark.gpu

BENCH_TOL = 5e-6     # the benchmark's stopping tolerance


def _problem(ciq, torch, dtype, s):
    import workloads
    wl = workloads.workload(2, s=s)
    p = wl.problems[0]
    x = torch.from_numpy(p.x.astype(dtype)).cuda()
    b = torch.from_numpy(p.b.astype(dtype)).cuda()
    return wl, ciq.Problem(x, p.kernel, p.lengthscale, p.outputscale, p.noise), b


def test_round_trip_full_size_fp64():
    torch = torch_cuda()
    ciq = ciq_module()
    wl, prob, b = _problem(ciq, torch, np.float64, 4)
    announce("full-size round trip f64 n=50000 s=4")
    half, i1, _ = ciq.ciq_sqrt_mvm(prob, b, q=15, max_iter=6000, tol=BENCH_TOL, seed=4001)
    back, i2, _ = ciq.ciq_invsqrt_mvm(prob, half, q=15, max_iter=6000, tol=BENCH_TOL, seed=4001)
    err = colwise_rel(back.cpu().numpy(), b.cpu().numpy()).max()
    print(f"round trip rel err {err:.3e} iters {i1['iters']} {i2['iters']}", flush=True)
    assert i1["converged"] and i2["converged"]
    assert err < 1e-4


@pytest.fixture(scope="module")
def tight_fp64():
    """K^{-1/2} B and K^{1/2} B at tol 1e-9 on the FP64 path, with the bounds
    the default path estimates."""
    torch = torch_cuda()
    ciq = ciq_module()
    wl, p64, b64 = _problem(ciq, torch, np.float64, 4)
    announce("full-size f64 reference tol 1e-9 n=50000 s=4")
    lo, hi = ciq.ciq_eig_bounds(p64, steps=20, seed=0)
    bounds = (lo, hi)
    inv, ii, _ = ciq.ciq_invsqrt_mvm(p64, b64, q=15, max_iter=8000, tol=1e-9, bounds=bounds)
    sq, isq, _ = ciq.ciq_sqrt_mvm(p64, b64, q=15, max_iter=8000, tol=1e-9, bounds=bounds)
    assert ii["converged"] and isq["converged"]
    return bounds, inv.cpu().numpy(), sq.cpu().numpy()


@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_fp64_at_bench_settings_full_size(tight_fp64, mode):
    """The benchmark's path (FP64 product, tol 5e-6) meets 1e-4 relative error."""
    torch = torch_cuda()
    ciq = ciq_module()
    bounds, inv, sq = tight_fp64
    wl, p64, b64 = _problem(ciq, torch, np.float64, 4)
    announce(f"full-size f64 tol {BENCH_TOL} {mode} n=50000 s=4")
    fn = ciq.ciq_invsqrt_mvm if mode == "invsqrt" else ciq.ciq_sqrt_mvm
    out, info, _ = fn(p64, b64, q=15, max_iter=6000, tol=BENCH_TOL, bounds=bounds)
    err = colwise_rel(out.cpu().numpy(), inv if mode == "invsqrt" else sq).max()
    print(f"f64 {mode} rel err {err:.3e} iters {info['iters']}", flush=True)
    assert info["converged"]
    assert err < 1e-4


@pytest.mark.parametrize("cache", ["on", "off"])
def test_fp32_full_size(tight_fp64, cache):
    """The FP32 products (resident: FP64 entries rounded once; on the fly:
    FP32 entries) at the benchmark's tolerance meet 1e-4 for K^{1/2}B, the
    benchmark's output."""
    torch = torch_cuda()
    ciq = ciq_module()
    bounds, inv, sq = tight_fp64
    wl, p32, b32 = _problem(ciq, torch, np.float32, 4)
    announce(f"full-size f32 tol {BENCH_TOL} cache={cache} n=50000 s=4")
    out, info, _ = ciq.ciq_sqrt_mvm(p32, b32, q=15, max_iter=6000, tol=BENCH_TOL, bounds=bounds,
                                    kernel_cache=cache)
    err = colwise_rel(out.cpu().numpy(), sq).max()
    print(f"f32 cache={cache} sqrt rel err {err:.3e} iters {info['iters']}", flush=True)
    assert info["converged"] and info["kernel_cached"] == (cache == "on")
    assert err < 1e-4


def test_preconditioned_full_size_rotation_identities():
    """The bench's preconditioned form (rank 800, FP32 resident products,
    tol 5e-6) at full size, S = 16: A = R'B and RB satisfy A^T K A = B^T B and
    (RB)^T A = B^T B (properties of any size; K applied by the FP64
    on-the-fly product), to 1e-4 relative, with 4-5x fewer iterations than
    plain CIQ needs at this tolerance (~2977)."""
    torch = torch_cuda()
    ciq = ciq_module()
    wl, prob, b = _problem(ciq, torch, np.float32, 16)
    announce("full-size preconditioned identities f32 rank 800 n=50000 s=16")
    kw = dict(q=15, max_iter=6000, tol=BENCH_TOL, seed=4001, precond_rank=800)
    a, ia, _ = ciq.ciq_invsqrt_mvm(prob, b, **kw)
    rb, ir, _ = ciq.ciq_sqrt_mvm(prob, b, **kw)
    p64 = ciq.Problem(prob.x.double().contiguous(), prob.kernel, prob.lengthscale, prob.outputscale, prob.noise)
    ka = ciq.ciq_kernel_mvm(p64, a.double().contiguous())
    torch.cuda.synchronize()
    A, KA, RB, B = (t.double().cpu().numpy() for t in (a, ka, rb, b))
    BtB = B.T @ B
    e1 = np.abs(A.T @ KA - BtB).max() / np.abs(BtB).max()
    e2 = np.abs(RB.T @ A - BtB).max() / np.abs(BtB).max()
    print(f"identity errors {e1:.2e} {e2:.2e}; iters {ia['iters']} {ir['iters']}; rank {ia['precond_rank']}",
          flush=True)
    assert ia["converged"] and ir["converged"] and ia["precond_rank"] == 800
    assert ia["iters"] < 1000
    assert e1 < 1e-4 and e2 < 1e-4


def _oracle_reference():
    import json
    import os
    g = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    meta_path = os.path.join(g, "matern52_n50000_s8_reference.json")
    if not os.path.exists(meta_path):
        pytest.skip("oracle reference not written (tests/golden/make_matern52_n50000_reference.py)")
    meta = json.load(open(meta_path))
    ref = {m: np.load(os.path.join(g, f"matern52_n50000_s8_{m}.npy"), allow_pickle=False) for m in ("sqrt", "invsqrt")}
    return meta, ref


@pytest.mark.parametrize("prec", ["f32", "f16x3"])
@pytest.mark.parametrize("mode", ["sqrt", "invsqrt"])
def test_benchmark_path_against_oracle(prec, mode):
    """The benchmark's solve (all 64 columns, so its launch configuration:
    resident matrix, 16 column ranges, estimated bounds, tol 5e-6) against
    the CPU FP64 oracle's K^{+-1/2}B for the first 8 columns (msMINRES-CIQ to
    relative residual 1e-10, written by an oracle-only script): the metric's
    1e-4 per column."""
    meta, ref = _oracle_reference()
    torch = torch_cuda()
    ciq = ciq_module()
    wl, prob, b = _problem(ciq, torch, np.float32, 64)
    announce(f"benchmark path {prec} {mode} vs oracle reference n=50000 s=64")
    fn = ciq.ciq_sqrt_mvm if mode == "sqrt" else ciq.ciq_invsqrt_mvm
    out, info, _ = fn(prob, b, q=15, max_iter=6000, tol=BENCH_TOL, seed=4001, precision=prec)
    assert info["converged"] and info["kernel_cached"]
    k = ref[mode].shape[1]
    err = colwise_rel(out[:, :k].cpu().numpy(), ref[mode])
    print(f"benchmark path {prec} {mode}: per-column rel err vs oracle max {err.max():.2e} median "
          f"{np.median(err):.2e} ({info['iters']} iterations)", flush=True)
    assert err.max() < 1e-4, err


@pytest.mark.parametrize("mode", ["sqrt", "invsqrt"])
def test_fp64_path_against_oracle(mode):
    """The FP64 path on the oracle's own bounds, run to the oracle's relative
    residual 1e-10: both sides then carry only Krylov and rounding error, and
    they agree to 1e-6 per column (100x below the metric's bar)."""
    meta, ref = _oracle_reference()
    torch = torch_cuda()
    ciq = ciq_module()
    wl, prob, b = _problem(ciq, torch, np.float64, 64)
    b = b[:, :ref[mode].shape[1]].contiguous()      # the reference's right-hand sides: B's first columns
    announce(f"fp64 path {mode} vs oracle reference n=50000 s=8 tol 1e-10")
    fn = ciq.ciq_sqrt_mvm if mode == "sqrt" else ciq.ciq_invsqrt_mvm
    out, info, _ = fn(prob, b, q=meta["q"], max_iter=20000, tol=meta["tol"],
                      bounds=(meta["lambda_min"], meta["lambda_max"]))
    assert info["converged"]
    err = colwise_rel(out.cpu().numpy(), ref[mode])
    print(f"fp64 path {mode}: per-column rel err vs oracle max {err.max():.2e} ({info['iters']} iterations, "
          f"oracle {meta['iters']})", flush=True)
    assert err.max() < 1e-6, err
