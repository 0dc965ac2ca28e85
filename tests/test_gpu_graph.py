"""The HIP-graph iteration loop (ciq_opts.graph = 1) against the eager loop:
the same kernels in the same order, so the results must be bitwise equal.
Each solve replays its graph many times with the host polling (a
synchronization) between replays; successive solves capture new graphs with
eager work (other solves) in between."""
import time

import numpy as np
import pytest

from gpu_util import announce, ciq_module, torch_cuda

pytestmark = pytest.mark.gpu


def _problem(ciq, torch, n, d, s, kind, dtype, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(dtype)
    b = rng.standard_normal((n, s)).astype(dtype)
    return ciq.Problem(torch.from_numpy(x).cuda(), kind, [0.3], 1.0, 1e-2), torch.from_numpy(b).cuda()


@pytest.mark.parametrize("n,d,s,kind,dtype,cache", [
    (1024, 3, 1, "rbf", np.float64, "on"),
    (1024, 3, 1, "rbf", np.float64, "off"),
    (3001, 6, 16, "matern52", np.float32, "on"),
    (777, 5, 33, "matern52", np.float32, "off"),
])
def test_graph_loop_equals_eager(n, d, s, kind, dtype, cache):
    torch = torch_cuda()
    ciq = ciq_module()
    prob, b = _problem(ciq, torch, n, d, s, kind, dtype, n + s)
    announce(f"graph vs eager n={n} s={s} {kind} cache={cache}")
    for mode, fn in [("invsqrt", ciq.ciq_invsqrt_mvm), ("sqrt", ciq.ciq_sqrt_mvm)]:
        kw = dict(q=8, max_iter=101, tol=1e-6, bounds=(1e-2, 400.0), kernel_cache=cache, keep_solves=True)
        e_out, e_info, e_sol = fn(prob, b, **kw)
        g_out, g_info, g_sol = fn(prob, b, graph=True, **kw)
        torch.cuda.synchronize()
        assert g_info["iters"] == e_info["iters"]
        assert torch.equal(g_out, e_out), mode
        assert torch.equal(g_sol, e_sol), mode


def test_graph_successive_solves_and_batched():
    torch = torch_cuda()
    ciq = ciq_module()
    announce("graph successive solves + batched")
    pa, ba = _problem(ciq, torch, 1500, 4, 8, "rbf", np.float32, 1)
    pb, bb = _problem(ciq, torch, 900, 7, 8, "rbf", np.float32, 2)
    kw = dict(q=10, max_iter=300, tol=1e-5, bounds=(1e-2, 400.0))
    ga, _, _ = ciq.ciq_invsqrt_mvm(pa, ba, graph=True, **kw)
    ea, _, _ = ciq.ciq_invsqrt_mvm(pa, ba, **kw)
    gb, _, _ = ciq.ciq_invsqrt_mvm(pb, bb, graph=True, **kw)
    eb, _, _ = ciq.ciq_invsqrt_mvm(pb, bb, **kw)
    ga2, _, _ = ciq.ciq_invsqrt_mvm(pa, ba, graph=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(ga, ea) and torch.equal(gb, eb) and torch.equal(ga2, ea)
    outs_g, infos_g = ciq.ciq_invsqrt_mvm_batched([pa, pb], [ba, bb], q=10, max_iter=300, tol=1e-5,
                                                  bounds=(1e-2, 400.0), graph=True)
    outs_e, infos_e = ciq.ciq_invsqrt_mvm_batched([pa, pb], [ba, bb], q=10, max_iter=300, tol=1e-5,
                                                  bounds=(1e-2, 400.0))
    torch.cuda.synchronize()
    for k in range(2):
        assert infos_g[k]["iters"] == infos_e[k]["iters"]
        assert torch.equal(outs_g[k], outs_e[k])


def test_graph_loop_latency_workload1():
    """The first workload (N = 1024, S = 1, J = 100): report the time per
    iteration of both loops (measured ~46 us for both: the dependent kernels'
    device latency, not host launch cost, sets it); the graph loop must not
    be slower."""
    torch = torch_cuda()
    ciq = ciq_module()
    import workloads
    wl = workloads.workload(1)
    p = wl.problems[0]
    prob = ciq.Problem(torch.from_numpy(p.x).cuda(), p.kernel, p.lengthscale, p.outputscale, p.noise)
    b = torch.from_numpy(p.b).cuda()
    announce("graph loop latency, first workload")
    kw = dict(q=wl.q, max_iter=wl.max_iter, tol=0.0, bounds=(1e-2, 100.0))
    res = {}
    for graph in (False, True):
        ciq.ciq_invsqrt_mvm(prob, b, graph=graph, **kw)       # warm-up (tuning, allocation)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            _, info, _ = ciq.ciq_invsqrt_mvm(prob, b, graph=graph, **kw)
        torch.cuda.synchronize()
        res[graph] = (time.perf_counter() - t0) / 5 / info["iters"] * 1e6
    print(f"us per iteration: eager {res[False]:.1f}, graph {res[True]:.1f}", flush=True)
    assert res[True] < 1.2 * res[False]
