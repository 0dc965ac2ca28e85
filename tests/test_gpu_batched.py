"""Parity of the batched HIP path (ciq_invsqrt_mvm_batched: one persistent
kernel-product launch per iteration over every problem's row blocks) with the
oracle run problem by problem: shrunken instances of the 64-problem workload,
the full workload on a subset of its problems, and both product forms
(resident FP32 matrices and FP32 entries on the fly)."""
import numpy as np
import pytest

from gpu_util import announce, ciq_module, colwise_rel, torch_cuda
from oracle import ciq as ociq
from oracle import kernels as okern

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P,nmax,s", [(5, 900, 4), (12, 400, 16), (3, 1500, 1)])
def test_batched_matches_oracle(P, nmax, s):
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(4, n=nmax, s=s, n_problems=P)
    probs, bs, refs, bounds = [], [], [], None
    announce(f"batched P={P} nmax={nmax} s={s} ns={[p.n for p in wl.problems]}")
    for p in wl.problems:
        K = okern.kernel_matrix(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise)
        lam = np.linalg.eigvalsh(K)
        lo, hi = 1e-2, 1.05 * lam[-1]       # common bounds (noise is a certified lower bound)
        bounds = (lo, max(hi, bounds[1]) if bounds else hi)
    for p in wl.problems:
        K = okern.kernel_matrix(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise)
        ref, info = ociq.ciq(lambda v: K @ v, p.b.astype(np.float64), bounds[0], bounds[1], wl.q, 1000, 1e-10)
        refs.append(ref)
        probs.append(ciq.Problem(torch.from_numpy(p.x).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise))
        bs.append(torch.from_numpy(p.b).cuda())
    for cache in ("on", "off"):
        outs, infos = ciq.ciq_invsqrt_mvm_batched(probs, bs, q=wl.q, max_iter=1000, tol=1e-7, bounds=bounds,
                                                  kernel_cache=cache)
        for k in range(P):
            err = colwise_rel(outs[k].cpu().numpy(), refs[k]).max()
            assert err < 1e-4, (cache, k, err)
            assert infos[k]["converged"] and infos[k]["kernel_cached"] == (cache == "on")
    # independent problems stop independently
    assert len({i["iters"] for i in infos}) >= min(P, 2) or P == 1


def test_batched_equals_single_calls():
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(4, n=1200, s=8, n_problems=6)
    announce("batched vs single calls P=6")
    probs = [ciq.Problem(torch.from_numpy(p.x).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
             for p in wl.problems]
    bs = [torch.from_numpy(p.b).cuda() for p in wl.problems]
    bounds = (1e-2, 400.0)
    outs, infos = ciq.ciq_invsqrt_mvm_batched(probs, bs, q=wl.q, max_iter=500, tol=1e-6, bounds=bounds)
    for k in range(6):
        # the batched call streams one resident FP32 matrix per problem (FP64
        # entries rounded once), as the single call does with its resident matrix
        single, info, _ = ciq.ciq_invsqrt_mvm(probs[k], bs[k], q=wl.q, max_iter=500, tol=1e-6, bounds=bounds,
                                              kernel_cache="on")
        # the split of the j range differs between the two launches, so the
        # runs differ by rounding only: both stop within a few iterations of
        # each other at the same tolerance
        assert abs(infos[k]["iters"] - info["iters"]) <= 5
        assert colwise_rel(outs[k].cpu().numpy(), single.cpu().numpy()).max() < 1e-5


@pytest.mark.timeout(900)
def test_batched_full_workload_against_oracle():
    """The 64-problem batching workload at its real sizes (N_p log-uniform in
    [2,000, 20,000], d_p in 2..10, S = 16, Q = 12) in one batched call (the
    persistent product over every problem's row blocks, per-problem bounds
    and stopping), tol 1e-6, held to the oracle's msMINRES-CIQ on the dense
    FP64 matrix (its own Lanczos bounds, tol 1e-8) for the largest problem and
    the five smallest: 1e-4 per column."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    from oracle import lanczos as olz
    wl = workloads.workload(4)
    ns = [p.n for p in wl.problems]
    announce(f"batched full workload P={len(ns)} sum_n={sum(ns)}")
    probs = [ciq.Problem(torch.from_numpy(p.x).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
             for p in wl.problems]
    bs = [torch.from_numpy(p.b).cuda() for p in wl.problems]
    outs, infos = ciq.ciq_invsqrt_mvm_batched(probs, bs, q=wl.q, max_iter=3000, tol=1e-6, seed=4001)
    assert all(i["converged"] for i in infos)
    order = np.argsort(ns)
    check = list(order[:5]) + [int(order[-1])]
    for k in check:
        p = wl.problems[k]
        K = okern.kernel_matrix(p.kernel, p.x.astype(np.float64), p.lengthscale, p.outputscale, p.noise)
        lo, hi, _, _ = olz.eig_bounds(lambda v: K @ v, workloads.start_vector(p.n, 4004 + k, np.float64), 20,
                                      p.noise)
        ref, oinfo = ociq.ciq(lambda v: K @ v, p.b.astype(np.float64), lo, hi, wl.q, 5000, 1e-8)
        err = colwise_rel(outs[k].cpu().numpy(), ref).max()
        print(f"problem {k}: n={p.n} d={p.d} iters {infos[k]['iters']} (oracle {oinfo.iters}) rel err {err:.2e}",
              flush=True)
        assert err < 1e-4, (k, err)
