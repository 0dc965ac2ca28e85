"""Parity of the HIP msMINRES-CIQ path (ciq_invsqrt_mvm / ciq_sqrt_mvm /
ciq_eig_bounds through the C ABI) with the oracle on the same seeded inputs
and the same eigenvalue bounds."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import ciq as ociq
from oracle import kernels as okern
from oracle import lanczos as olz
from oracle import msminres as oms
from oracle import quadrature as oqd

pytestmark = pytest.mark.gpu


def _dense(p):
    return okern.kernel_matrix(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise)


def _oracle_spread(K, b, bounds, q, J, tol, mode, ref, seeds=2):
    """How far the oracle's own result moves when every entry of K is
    perturbed by one ulp (2.2e-16 relative, independent per entry): the scale
    of the rounding differences between two correct FP64 kernel products
    (entry evaluation and summation order) at this (K, J)."""
    spread = 0.0
    for seed in range(seeds):
        rng = np.random.default_rng(100 + seed)
        E = rng.standard_normal(K.shape)
        Kp = K * (1.0 + 2.2e-16 * (E + E.T) / np.sqrt(2.0))
        alt, _ = ociq.ciq(lambda v: Kp @ v, b, bounds[0], bounds[1], q, J, tol, mode)
        spread = max(spread, colwise_rel(alt, ref).max())
    return spread


def _gpu_problem(ciq, torch, p):
    return ciq.Problem(torch.from_numpy(np.ascontiguousarray(p.x)).cuda(), p.kernel, p.lengthscale,
                       p.outputscale, p.noise)


@pytest.mark.parametrize("cache", ["on", "off"])
@pytest.mark.parametrize("J", [1, 2, 5, 10])
@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_fp64_recurrence_parity_small_j(mode, J, cache):
    """Before Lanczos loses orthogonality the finite-precision iterates are
    stable, so GPU and oracle must agree to rounding: RBF N=1024 d=3 (first
    workload's inputs), Q=8, fixed J, no early stop; with the resident kernel
    matrix and with entries evaluated in every product."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(1, s=3)
    p = wl.problems[0]
    K = _dense(p)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f64 small-J parity {mode} J={J} cache={cache}")
    fn = ciq.ciq_invsqrt_mvm if mode == "invsqrt" else ciq.ciq_sqrt_mvm
    out, info, solves = fn(_gpu_problem(ciq, torch, p), torch.from_numpy(p.b).cuda(), q=8, max_iter=J,
                           tol=0.0, bounds=bounds, keep_solves=True, kernel_cache=cache)
    assert info["kernel_cached"] == (cache == "on")
    ref, oinfo, t, w, X = ociq.ciq(lambda v: K @ v, p.b, bounds[0], bounds[1], 8, J, 0.0, mode,
                                   return_solves=True)
    assert info["iters"] == oinfo.iters == J
    assert colwise_rel(out.cpu().numpy(), ref).max() < 1e-11
    sv = solves.cpu().numpy()
    for qi in range(8):
        assert colwise_rel(sv[:, qi, :], X[qi]).max() < 1e-11
    np.testing.assert_allclose(info["max_rel_residual"], oinfo.rel_residual.max(), rtol=1e-9)


@pytest.mark.parametrize("mode", ["invsqrt", "sqrt"])
def test_fp64_workload1(mode):
    """The first workload as stated (RBF N=1024, S=1, Q=8, J=100, tol 1e-4,
    FP64). J=100 is past the loss of orthogonality and short of convergence:
    there two correct finite-precision runs differ chaotically. The bar is
    calibrated on the oracle itself: its own iterate moves when every product
    is perturbed by 1e-16 relative (three seeds); the GPU-oracle gap must be
    within 3x the largest such move, with the same iteration count."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(1)
    p = wl.problems[0]
    K = _dense(p)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f64 workload1 {mode} n={p.n}")
    fn = ciq.ciq_invsqrt_mvm if mode == "invsqrt" else ciq.ciq_sqrt_mvm
    out, info, _ = fn(_gpu_problem(ciq, torch, p), torch.from_numpy(p.b).cuda(), q=wl.q, max_iter=wl.max_iter,
                      tol=wl.tol, bounds=bounds)
    out = out.cpu().numpy()
    ref, oinfo = ociq.ciq(lambda v: K @ v, p.b, bounds[0], bounds[1], wl.q, wl.max_iter, wl.tol, mode)
    spread = 0.0
    for seed in range(3):
        rng = np.random.default_rng(seed)
        pert = lambda v: (K @ v) * (1.0 + 1e-16 * rng.standard_normal(v.shape))
        alt, _ = ociq.ciq(pert, p.b, bounds[0], bounds[1], wl.q, wl.max_iter, wl.tol, mode)
        spread = max(spread, colwise_rel(alt, ref).max())
    exact = ociq.exact_power(K, p.b, 0.5 if mode == "sqrt" else -0.5)
    assert info["iters"] == oinfo.iters
    gap = colwise_rel(out, ref).max()
    assert gap <= 3.0 * spread + 1e-12, (gap, spread)
    own = colwise_rel(ref, exact).max()
    assert colwise_rel(out, exact).max() < 1.2 * own


@pytest.mark.parametrize("cache", ["on", "off"])
@pytest.mark.parametrize("n,s,kind,q", [(777, 5, "matern52", 6), (64, 3, "rbf", 15), (1, 2, "rbf", 4),
                                        (200, 17, "rbf", 8)])
def test_fp64_ragged_shapes(n, s, kind, q, cache):
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(n + s)
    x = rng.random((n, 3))
    b = rng.standard_normal((n, s))
    b[:, 0] *= 1e-3
    if s > 2:
        b[:, 2] = 0.0                      # zero column -> zero output
    K = okern.kernel_matrix(kind, x, [0.3], 1.2, 0.02)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f64 ragged n={n} s={s} {kind} q={q} cache={cache}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, [0.3], 1.2, 0.02)
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, solves = fn(prob, torch.from_numpy(b).cuda(), q=q, max_iter=1500, tol=1e-11,
                               bounds=bounds, keep_solves=True, kernel_cache=cache)
        assert info["kernel_cached"] == (cache == "on")
        ref, oinfo, t, w, X = ociq.ciq(lambda v: K @ v, b, bounds[0], bounds[1], q, 1500, 1e-11, mode,
                                       return_solves=True)
        out = out.cpu().numpy()
        if s > 2:
            assert np.all(out[:, 2] == 0.0)
        nz = np.linalg.norm(b, axis=0) > 0
        # both runs converged to 1e-11 residual: they agree to ~kappa * tol
        assert colwise_rel(out[:, nz], ref[:, nz]).max() < 1e-8
        np.testing.assert_allclose(info["t"], t, rtol=1e-12)
        sv = solves.cpu().numpy()                     # [n][q][s]
        for qi in range(q):
            assert colwise_rel(sv[:, qi, nz], X[qi][:, nz]).max() < 1e-8
        assert info["converged"]


@pytest.mark.parametrize("kind,n,s,d,ard", [("matern52", 3001, 20, 5, True), ("rbf", 5000, 64, 8, False),
                                            ("matern52", 4500, 64, 6, False), ("rbf", 700, 1, 12, True),
                                            ("rbf", 1200, 100, 3, False)])
def test_resident_matrix_small_j_parity(kind, n, s, d, ard):
    """The streamed resident matrix against the oracle at fixed small J over
    tile-spanning ragged sizes, including the one-range-per-XCD split
    (n >= 4096 rows, 64 columns), single-column products and more than 64
    columns (two column groups streaming the same matrix). The bar is 10x
    the oracle's own rounding spread (entries of K perturbed by one ulp), at
    least 1e-12."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(n + 7 * d)
    x = rng.random((n, d))
    b = rng.standard_normal((n, s))
    ls = list(np.linspace(0.25, 0.9, d)) if ard else [0.4]
    K = okern.kernel_matrix(kind, x, ls, 1.3, 0.05)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f64 resident K small-J {kind} n={n} s={s} d={d} ard={ard}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.3, 0.05)
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, _ = fn(prob, torch.from_numpy(b).cuda(), q=6, max_iter=6, tol=0.0, bounds=bounds,
                          kernel_cache="on")
        assert info["kernel_cached"]
        ref, oinfo = ociq.ciq(lambda v: K @ v, b, bounds[0], bounds[1], 6, 6, 0.0, mode)
        assert info["iters"] == oinfo.iters == 6
        bar = max(10.0 * _oracle_spread(K, b, bounds, 6, 6, 0.0, mode, ref), 1e-12)
        gap = colwise_rel(out.cpu().numpy(), ref).max()
        assert gap < bar, (mode, gap, bar)


def test_kernel_cache_policy():
    """auto keeps K only within the budget; FP64, FP32 and split FP16 cache,
    split BF16 never does."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(5)
    n = 1024                                   # resident matrix: 1024 x 1024 doubles = 8 MiB
    x = rng.random((n, 3))
    b = rng.standard_normal((n, 2))
    announce("kernel cache policy")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", [0.3], 1.0, 0.1)
    bt = torch.from_numpy(b).cuda()
    _, i_auto, _ = ciq.ciq_invsqrt_mvm(prob, bt, q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0))
    _, i_small, _ = ciq.ciq_invsqrt_mvm(prob, bt, q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0),
                                        cache_budget_mib=4)
    _, i_big, _ = ciq.ciq_invsqrt_mvm(prob, bt, q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0),
                                      cache_budget_mib=16)
    assert i_auto["kernel_cached"] and not i_small["kernel_cached"] and i_big["kernel_cached"]
    p32 = ciq.Problem(torch.from_numpy(x.astype(np.float32)).cuda(), "rbf", [0.3], 1.0, 0.1)
    _, i32, _ = ciq.ciq_invsqrt_mvm(p32, bt.float(), q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0),
                                    kernel_cache="on")
    assert i32["kernel_cached"]
    _, ix3, _ = ciq.ciq_invsqrt_mvm(p32, bt.float(), q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0),
                                    kernel_cache="on", precision="bf16x3")
    assert not ix3["kernel_cached"]
    _, i16, _ = ciq.ciq_invsqrt_mvm(p32, bt.float(), q=4, max_iter=5, tol=0.0, bounds=(0.1, 300.0),
                                    precision="f16x3")
    assert i16["kernel_cached"]


@pytest.mark.parametrize("cache", ["on", "off"])
@pytest.mark.parametrize("kind,n,s,d", [("matern52", 2000, 16, 6), ("rbf", 1500, 33, 8), ("rbf", 999, 64, 3),
                                        ("matern52", 4500, 64, 6), ("rbf", 1100, 130, 4)])
def test_fp32_matches_fp64_oracle(kind, n, s, d, cache):
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(n)
    x = rng.random((n, d)).astype(np.float32)
    b = rng.standard_normal((n, s)).astype(np.float32)
    ls = [0.3]
    K = okern.kernel_matrix(kind, x.astype(np.float64), ls, 1.0, 1e-2)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f32 {kind} n={n} s={s} d={d} cache={cache}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, ls, 1.0, 1e-2)
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, _ = fn(prob, torch.from_numpy(b).cuda(), q=12, max_iter=1000, tol=1e-6, bounds=bounds,
                          kernel_cache=cache)
        assert info["kernel_cached"] == (cache == "on")
        ref, _ = ociq.ciq(lambda v: K @ v, b.astype(np.float64), bounds[0], bounds[1], 12, 1000, 1e-10, mode)
        err = colwise_rel(out.cpu().numpy(), ref).max()
        assert err < 1e-4, (mode, err, info["iters"])


@pytest.mark.parametrize("prec,cache", [("f64", "off"), ("f64", "on"), ("f32", "on")])
def test_krylov_basis_matches_direction_recurrence(prec, cache):
    """The resident Lanczos basis (solution formed once from the logged
    direction coefficients) against the direction recurrence, same inputs and
    bounds, both modes, ragged sizes, a zero column, columns stopping at
    different iterations: the same iterate up to rounding."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(31)
    n, d, s = 2345, 4, 19
    dt = np.float64 if prec == "f64" else np.float32
    x = rng.random((n, d)).astype(dt)
    b = rng.standard_normal((n, s)).astype(dt)
    b[:, 3] = 0.0
    b[:, 5] *= 1e-4
    K = okern.kernel_matrix("matern52", x.astype(np.float64), [0.35], 1.1, 2e-3)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"krylov basis vs recurrence {prec} cache={cache}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "matern52", [0.35], 1.1, 2e-3)
    bt = torch.from_numpy(b).cuda()
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        kw = dict(q=12, max_iter=3000, tol=1e-9 if prec == "f64" else 1e-6, bounds=bounds, kernel_cache=cache)
        on, ion, _ = fn(prob, bt, krylov_basis="auto", **kw)
        off, ioff, _ = fn(prob, bt, krylov_basis="off", **kw)
        assert ion["krylov_basis"] and not ioff["krylov_basis"]
        assert ion["iters"] == ioff["iters"] and ion["converged"] and ioff["converged"]
        on, off = on.double().cpu().numpy(), off.double().cpu().numpy()
        assert np.all(on[:, 3] == 0.0) and np.all(off[:, 3] == 0.0)
        keep = [c for c in range(s) if c != 3]
        gap = colwise_rel(on[:, keep], off[:, keep]).max()
        ref, _ = ociq.ciq(lambda v: K @ v, b.astype(np.float64), bounds[0], bounds[1], 12, 3000, 1e-11, mode)
        err_on = colwise_rel(on[:, keep], ref[:, keep]).max()
        err_off = colwise_rel(off[:, keep], ref[:, keep]).max()
        print(f"{prec} {mode}: basis vs recurrence {gap:.2e}; vs oracle {err_on:.2e} / {err_off:.2e}", flush=True)
        assert gap < (1e-9 if prec == "f64" else 1e-6), gap
        assert err_on <= 1.5 * err_off + 1e-12


@pytest.mark.parametrize("s", [4, 8, 32])
def test_inner_product_passes_all_widths(s):
    """The 16-byte inner-product passes (four columns per lane) at the widths
    the workloads above do not use, ragged rows: FP64 at small J against the
    oracle to rounding (FP64 split partials), and the FP32 resident square
    root, whose products leave FP32 split partials, converged against the
    oracle at the FP32 bar."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(300 + s)
    n = 4099
    x = rng.random((n, 3))
    b = rng.standard_normal((n, s))
    K = okern.kernel_matrix("rbf", x, [0.3], 1.2, 0.02)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"inner-product passes s={s} n={n}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", [0.3], 1.2, 0.02)
    bt = torch.from_numpy(b).cuda()
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, _ = fn(prob, bt, q=8, max_iter=6, tol=0.0, bounds=bounds, kernel_cache="on")
        ref, oinfo = ociq.ciq(lambda v: K @ v, b, bounds[0], bounds[1], 8, 6, 0.0, mode)
        assert info["iters"] == oinfo.iters == 6
        gap = colwise_rel(out.cpu().numpy(), ref).max()
        assert gap < 1e-11, (mode, gap)
    x32, b32 = x.astype(np.float32), b.astype(np.float32)
    K32 = okern.kernel_matrix("rbf", x32.astype(np.float64), [0.3], 1.2, 0.02)
    lam32 = np.linalg.eigvalsh(K32)
    bounds32 = (lam32[0], lam32[-1])
    prob32 = ciq.Problem(torch.from_numpy(x32).cuda(), "rbf", [0.3], 1.2, 0.02)
    out, info, _ = ciq.ciq_sqrt_mvm(prob32, torch.from_numpy(b32).cuda(), q=12, max_iter=1000, tol=1e-6,
                                    bounds=bounds32, kernel_cache="on")
    ref, _ = ociq.ciq(lambda v: K32 @ v, b32.astype(np.float64), bounds32[0], bounds32[1], 12, 1000, 1e-10, "sqrt")
    err = colwise_rel(out.cpu().numpy(), ref).max()
    print(f"s={s}: FP32 resident square root vs oracle {err:.2e} ({info['iters']} iterations)", flush=True)
    assert info["converged"] and err < 1e-4, err


def test_krylov_basis_chunks_reused_across_calls(monkeypatch):
    """The basis slots live in chunks kept between calls. With 2 MiB chunks
    (five slots of n = 2345, s = 19) every run crosses many chunk boundaries
    while it iterates; the calls in a row reuse the chunks of the earlier ones
    (another problem size, the graph-replayed loop), a new chunk size starts
    the pool over, and after ciq_release_workspace the next call allocates
    afresh. Each result equals the direction recurrence's up to rounding."""
    torch = torch_cuda()
    ciq = ciq_module()
    ciq.ciq_release_workspace()

    def case(n, s, seed):
        r = np.random.default_rng(seed)
        x = r.random((n, 4))
        b = r.standard_normal((n, s))
        K = okern.kernel_matrix("matern52", x, [0.35], 1.1, 2e-3)
        lam = np.linalg.eigvalsh(K)
        prob = ciq.Problem(torch.from_numpy(x).cuda(), "matern52", [0.35], 1.1, 2e-3)
        return prob, torch.from_numpy(b).cuda(), (lam[0], lam[-1])

    big = case(2345, 19, 1)
    small = case(1000, 7, 2)
    steps = [("1", big, False, ciq.ciq_sqrt_mvm), ("1", big, True, ciq.ciq_invsqrt_mvm),
             ("1", small, False, ciq.ciq_sqrt_mvm), ("3", big, False, ciq.ciq_invsqrt_mvm),
             ("release", big, True, ciq.ciq_sqrt_mvm)]
    for chunk_mib, (prob, bt, bounds), graph, fn in steps:
        if chunk_mib == "release":
            ciq.ciq_release_workspace()
        else:
            monkeypatch.setenv("CIQ_BASIS_CHUNK_MIB", chunk_mib)
        announce(f"krylov basis chunks {chunk_mib} n={bt.shape[0]} s={bt.shape[1]} graph={graph} {fn.__name__}")
        kw = dict(q=12, max_iter=3000, tol=1e-9, bounds=bounds, kernel_cache="on", graph=graph)
        on, ion, _ = fn(prob, bt, krylov_basis="auto", **kw)
        off, ioff, _ = fn(prob, bt, krylov_basis="off", **kw)
        assert ion["krylov_basis"] and not ioff["krylov_basis"]
        assert ion["converged"] and ion["iters"] == ioff["iters"] and ion["iters"] > 50
        gap = colwise_rel(on.cpu().numpy(), off.cpu().numpy()).max()
        print(f"chunks {chunk_mib}: {ion['iters']} iterations, basis vs recurrence {gap:.2e}", flush=True)
        assert gap < 1e-9, gap
    monkeypatch.delenv("CIQ_BASIS_CHUNK_MIB")
    ciq.ciq_release_workspace()


@pytest.mark.parametrize("s", [16, 32])
def test_fp32_resident_inverse_root_has_no_accumulation_error(s):
    """The FP32 resident inverse root at <= 32 columns contracts the FP32
    entries on the FP64 MFMA: its result is the solve on the FP32-rounded
    matrix itself. Held to the oracle's msMINRES-CIQ on that matrix (the
    FP64 kernel entries rounded to FP32 once, the noise added in FP64) at
    5e-6, on a problem where FP32 sums cost several 1e-5 (d = 3, lengthscale
    0.25, noise 1e-2: strongly correlated rows). Against the unrounded
    matrix the error is then the rounding's own, below 1e-4. Bounds: the
    noise and the largest absolute row sum (Gershgorin), on both sides."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(77 + s)
    n, d, noise = 4000, 3, 1e-2
    x = rng.random((n, d)).astype(np.float32)
    b = rng.standard_normal((n, s)).astype(np.float32)
    Kk = okern.kernel_matrix("rbf", x.astype(np.float64), [0.25], 1.0, 0.0)
    K = Kk + noise * np.eye(n)
    K32 = Kk.astype(np.float32).astype(np.float64) + noise * np.eye(n)
    del Kk
    bounds = (noise, float(np.abs(K).sum(axis=1).max()))
    announce(f"ciq f32 resident inverse root vs oracle on the rounded matrix n={n} s={s}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", [0.25], 1.0, noise)
    out, info, _ = ciq.ciq_invsqrt_mvm(prob, torch.from_numpy(b).cuda(), q=12, max_iter=3000, tol=1e-9,
                                       bounds=bounds, kernel_cache="on")
    assert info["kernel_cached"] and info["converged"]
    out = out.cpu().numpy()
    b64 = b.astype(np.float64)
    ref32, _ = ociq.ciq(lambda v: K32 @ v, b64, bounds[0], bounds[1], 12, 3000, 1e-11)
    ref, _ = ociq.ciq(lambda v: K @ v, b64, bounds[0], bounds[1], 12, 3000, 1e-11)
    own = colwise_rel(out, ref32).max()
    full = colwise_rel(out, ref).max()
    print(f"s={s}: vs rounded-matrix oracle {own:.2e}, vs exact-matrix oracle {full:.2e} "
          f"({info['iters']} iterations)", flush=True)
    assert own < 5e-6, own
    assert full < 1e-4, full


@pytest.mark.parametrize("prec,cache,bar", [("bf16x3", "off", 5e-3), ("f16x3", "off", 5e-4), ("f16x3", "on", 1e-4)])
def test_split_forms_against_exact(prec, cache, bar):
    """The split-operand BF16 / FP16 products inside a full CIQ solve: the
    error against the exact K^{-1/2}B and K^{1/2}B (eigendecomposition) is
    stated per form, bounded loosely here (kappa ~ 2e4). With the resident
    split FP16 matrix (22-bit entries, three part products) the bar is the
    FP32 path's."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(21)
    n, d, s = 2000, 6, 8
    x = rng.random((n, d)).astype(np.float32)
    b = rng.standard_normal((n, s)).astype(np.float32)
    K = okern.kernel_matrix("matern52", x.astype(np.float64), [0.3], 1.0, 1e-2)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq {prec} split form n={n} s={s}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "matern52", [0.3], 1.0, 1e-2)
    for mode, fn, pw in [("invsqrt", ciq.ciq_invsqrt_mvm, -0.5), ("sqrt", ciq.ciq_sqrt_mvm, 0.5)]:
        out, info, _ = fn(prob, torch.from_numpy(b).cuda(), q=15, max_iter=3000, tol=1e-7, bounds=bounds,
                          precision=prec, kernel_cache=cache)
        assert info["kernel_cached"] == (cache == "on")
        exact = ociq.exact_power(K, b.astype(np.float64), pw)
        err = colwise_rel(out.cpu().numpy(), exact).max()
        print(f"{prec} {mode}: max rel err vs exact {err:.3e}, iters {info['iters']}", flush=True)
        assert info["converged"]
        assert err < bar, (mode, err)


@pytest.mark.parametrize("kind,n,s,d", [("matern52", 2000, 16, 6), ("rbf", 1500, 33, 8), ("rbf", 999, 64, 3),
                                        ("matern52", 4500, 64, 6), ("rbf", 1100, 130, 4)])
def test_f16x3_resident_matches_fp64_oracle(kind, n, s, d):
    """The resident split FP16 form in full solves (both modes) against the
    oracle run to 1e-10, at the FP32 path's 1e-4 bar; includes one column
    range per XCD (n = 4500) and two column groups (s = 130)."""
    torch = torch_cuda()
    ciq = ciq_module()
    rng = np.random.default_rng(n + 1)
    x = rng.random((n, d)).astype(np.float32)
    b = rng.standard_normal((n, s)).astype(np.float32)
    K = okern.kernel_matrix(kind, x.astype(np.float64), [0.3], 1.0, 1e-2)
    lam = np.linalg.eigvalsh(K)
    bounds = (lam[0], lam[-1])
    announce(f"ciq f16x3 resident {kind} n={n} s={s} d={d}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), kind, [0.3], 1.0, 1e-2)
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        out, info, _ = fn(prob, torch.from_numpy(b).cuda(), q=12, max_iter=1000, tol=1e-6, bounds=bounds,
                          precision="f16x3", kernel_cache="on")
        assert info["kernel_cached"]
        ref, _ = ociq.ciq(lambda v: K @ v, b.astype(np.float64), bounds[0], bounds[1], 12, 1000, 1e-10, mode)
        err = colwise_rel(out.cpu().numpy(), ref).max()
        print(f"f16x3 resident {mode} {kind} n={n}: {err:.2e} ({info['iters']} iterations)", flush=True)
        assert err < 1e-4, (mode, err, info["iters"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_eig_bounds_match_oracle(prec):
    torch = torch_cuda()
    ciq = ciq_module()
    dt = np.float64 if prec == "f64" else np.float32
    rng = np.random.default_rng(11)
    n = 1200
    x = rng.random((n, 3)).astype(dt)
    v0 = rng.standard_normal(n).astype(dt)
    K = okern.kernel_matrix("rbf", x.astype(np.float64), [0.2], 1.0, 1e-2)
    announce(f"eig bounds {prec} n={n}")
    prob = ciq.Problem(torch.from_numpy(x).cuda(), "rbf", [0.2], 1.0, 1e-2)
    lo, hi = ciq.ciq_eig_bounds(prob, steps=20, v0=torch.from_numpy(v0).cuda())
    olo, ohi, _, _ = olz.eig_bounds(lambda v: K @ v, v0.astype(np.float64), 20, 1e-2)
    lam = np.linalg.eigvalsh(K)
    tol = 1e-8 if prec == "f64" else 1e-3
    assert abs(hi - ohi) <= tol * ohi
    assert abs(lo - olo) <= tol * olo
    assert lo <= lam[0] * (1 + 1e-6) and hi >= 0.95 * lam[-1]


def test_default_bounds_path_runs_and_is_accurate():
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(2, n=3000, s=8)
    p = wl.problems[0]
    announce("ciq f32 estimated bounds matern n=3000 s=8")
    K = _dense(p)
    out, info, _ = ciq.ciq_invsqrt_mvm(_gpu_problem(ciq, torch, p), torch.from_numpy(p.b).cuda(), q=15,
                                       max_iter=2000, tol=1e-6, seed=3)
    lam = np.linalg.eigvalsh(K)
    assert info["lambda_min"] <= lam[0] * (1 + 1e-6)
    assert info["lambda_max"] >= 0.9 * lam[-1]
    exact = ociq.exact_power(K, p.b.astype(np.float64), -0.5)
    assert colwise_rel(out.cpu().numpy(), exact).max() < 1e-3
    assert info["mvm_count"] == info["iters"] + 20


def test_profile_counts_kernel_products():
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(2, n=4000, s=16)
    p = wl.problems[0]
    announce("ciq f32 profile n=4000 s=16")
    out, info, _ = ciq.ciq_invsqrt_mvm(_gpu_problem(ciq, torch, p), torch.from_numpy(p.b).cuda(), q=15,
                                       max_iter=60, tol=1e-4, bounds=(1e-3, 400.0), profile=True)
    assert info["mvm_timed"] == info["iters"] == 60
    assert info["mvm_ms"] > 0.0
