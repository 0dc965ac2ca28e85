"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/ciq.h declares, its struct layouts match the binding, the
host-only quadrature agrees with the oracle, and invalid arguments are
rejected before any device work."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ciq.h")

L = pytest.importorskip("paper_2006_11267_amd._lib")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libciq.so not built")
    return L.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ciq_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ciq_[a-z0-9_]+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)
        assert n in L.PROTOTYPES, f"binding lacks {n}"


def test_struct_layout_matches_header(tmp_path):
    c = tmp_path / "layout.c"
    c.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ciq.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(ciq_problem), sizeof(ciq_opts), sizeof(ciq_info));
  printf("%zu %zu %zu %zu\n", offsetof(ciq_problem, lengthscale), offsetof(ciq_opts, seed),
         offsetof(ciq_opts, profile), offsetof(ciq_info, mvm_ms));
  return 0;
}
''')
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.dirname(HEADER),
                        str(c), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot compile the layout probe: " + r.stderr[:200])
    sizes, offs = subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n")[:2]
    assert [int(v) for v in sizes.split()] == [ctypes.sizeof(L.ciq_problem), ctypes.sizeof(L.ciq_opts),
                                                ctypes.sizeof(L.ciq_info)]
    assert [int(v) for v in offs.split()] == [L.ciq_problem.lengthscale.offset, L.ciq_opts.seed.offset,
                                               L.ciq_opts.profile.offset, L.ciq_info.mvm_ms.offset]


def _setup(lib, lmin, lmax, q):
    t = (ctypes.c_double * q)()
    w = (ctypes.c_double * q)()
    rc = lib.ciq_setup(lmin, lmax, q, t, w)
    return rc, np.array(t[:]), np.array(w[:])


@pytest.mark.parametrize("lmin,lmax,Q", [(1e-2, 87.0, 8), (1e-3, 2.5e3, 15), (0.3, 0.9, 4), (1e-4, 1e2, 12),
                                         (1.0, 1e8, 20), (2.0, 2.0, 5), (1e-3, 5e3, 64)])
def test_setup_matches_oracle(lib, lmin, lmax, Q):
    from oracle import quadrature as qd
    rc, t, w = _setup(lib, lmin, lmax, Q)
    assert rc == L.CIQ_OK
    to, wo = qd.hht_quadrature(lmin, lmax, Q)
    kappa = lmax / lmin
    # the oracle rounds the parameter 1 - k^2 (accuracy ~ eps * kappa); the
    # library never forms it (see the literal high-precision check below)
    rtol = 1e-13 + 4e-16 * kappa
    np.testing.assert_allclose(t, to, rtol=rtol)
    np.testing.assert_allclose(w, wo, rtol=rtol)
    assert np.all(np.diff(t) > 0) and np.all(w > 0)


@pytest.mark.parametrize("lmin,lmax,Q", [(1e-3, 2.5e3, 15), (1.0, 1e8, 20), (1e-2, 87.0, 8)])
def test_setup_matches_literal_formula(lib, lmin, lmax, Q):
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_quadrature import _literal_mpmath
    rc, t, w = _setup(lib, lmin, lmax, Q)
    assert rc == L.CIQ_OK
    tr, wr = _literal_mpmath(lmin, lmax, Q)
    np.testing.assert_allclose(t, tr, rtol=1e-12)
    np.testing.assert_allclose(w, wr, rtol=1e-12)


def test_setup_rejects(lib):
    for args in [(0.0, 1.0, 4), (2.0, 1.0, 4), (1.0, 2.0, 0), (1.0, 2.0, 65), (-1.0, 1.0, 2),
                 (1.0, float("inf"), 3), (float("nan"), 1.0, 3)]:
        rc, _, _ = _setup(lib, *args)
        assert rc == L.CIQ_EINVAL, args
    assert lib.ciq_setup(1.0, 2.0, 3, None, None) == L.CIQ_EINVAL


_KEEP = []


def _dev_ptr(nbytes=4096):
    """A small valid device buffer when a GPU is present, so that a validation
    regression shows as a wrong return code rather than device work on a bad
    address; without a GPU any non-null address serves (no device work may
    start, and none can)."""
    try:
        import torch
        if torch.cuda.is_available():
            t = torch.zeros(max(nbytes // 8, 1), dtype=torch.float64, device="cuda")
            _KEEP.append(t)
            return ctypes.c_void_p(t.data_ptr())
    except ImportError:
        pass
    return ctypes.c_void_p(512)


def _bad_problem(**kw):
    ls = (ctypes.c_double * 1)(0.3)
    fields = dict(n=10, d=3, x=_dev_ptr(), kernel=0, n_lengthscale=1,
                  lengthscale=ctypes.cast(ls, ctypes.POINTER(ctypes.c_double)), outputscale=1.0, noise=0.1)
    fields.update(kw)
    return L.ciq_problem(**fields), ls


@pytest.mark.parametrize("bad", [dict(n=0), dict(d=0), dict(d=17), dict(kernel=7), dict(n_lengthscale=2),
                                 dict(outputscale=0.0), dict(noise=-1.0), dict(x=None)])
def test_invalid_problem_rejected_before_device_work(lib, bad):
    p, keep = _bad_problem(**bad)
    o = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4)
    info = L.ciq_info()
    fake = _dev_ptr()
    for fn in (lib.ciq_invsqrt_mvm, lib.ciq_sqrt_mvm):
        assert fn(ctypes.byref(p), ctypes.byref(o), fake, 2, 2, fake, 2, None, ctypes.byref(info), None) \
            == L.CIQ_EINVAL
    assert lib.ciq_kernel_mvm(ctypes.byref(p), L.CIQ_F32, fake, 2, 2, fake, 2, None) == L.CIQ_EINVAL
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert lib.ciq_eig_bounds(ctypes.byref(p), L.CIQ_F32, 10, None, 0, ctypes.byref(lo), ctypes.byref(hi),
                              None) == L.CIQ_EINVAL
    del keep


@pytest.mark.parametrize("bad", [dict(q=0), dict(q=65), dict(max_iter=0), dict(tol=-1.0), dict(dtype=9),
                                 dict(tol=float("nan")), dict(check_every=-1), dict(precond_rank=-1),
                                 dict(precond_rank=1025)])
def test_invalid_options_rejected(lib, bad):
    p, keep = _bad_problem()
    o = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4)
    for k, v in bad.items():
        setattr(o, k, v)
    info = L.ciq_info()
    fake = _dev_ptr()
    assert lib.ciq_invsqrt_mvm(ctypes.byref(p), ctypes.byref(o), fake, 2, 2, fake, 2, None, ctypes.byref(info),
                               None) == L.CIQ_EINVAL
    del keep


def test_invalid_sizes_rejected(lib):
    p, keep = _bad_problem()
    o = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4)
    info = L.ciq_info()
    fake = _dev_ptr()
    for s, ldb, ldo in [(0, 1, 1), (4, 3, 4), (4, 4, 3)]:
        assert lib.ciq_invsqrt_mvm(ctypes.byref(p), ctypes.byref(o), fake, s, ldb, fake, ldo, None,
                                   ctypes.byref(info), None) == L.CIQ_EINVAL
    assert lib.ciq_invsqrt_mvm(ctypes.byref(p), ctypes.byref(o), None, 2, 2, fake, 2, None, ctypes.byref(info),
                               None) == L.CIQ_EINVAL
    assert lib.ciq_invsqrt_mvm(ctypes.byref(p), ctypes.byref(o), fake, 2, 2, fake, 2, None, None, None) \
        == L.CIQ_EINVAL
    probs = (L.ciq_problem * 1)(p)
    bp = (ctypes.c_void_p * 1)(_dev_ptr().value)
    infos = (L.ciq_info * 1)()
    assert lib.ciq_invsqrt_mvm_batched(0, probs, ctypes.byref(o), bp, 2, bp, infos, None) == L.CIQ_EINVAL
    del keep


def test_preconditioner_arguments_rejected(lib):
    """Preconditioning needs sigma^2 > 0; the batched call and the backward do
    not take it; the factor entry validates rank and pointers. All checked
    before any device work."""
    fake = _dev_ptr()
    info = L.ciq_info()
    p0, keep0 = _bad_problem(noise=0.0)
    o = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4, precond_rank=4)
    assert lib.ciq_sqrt_mvm(ctypes.byref(p0), ctypes.byref(o), fake, 2, 2, fake, 2, None, ctypes.byref(info),
                            None) == L.CIQ_EINVAL
    p, keep = _bad_problem()
    probs = (L.ciq_problem * 1)(p)
    bp = (ctypes.c_void_p * 1)(_dev_ptr().value)
    infos = (L.ciq_info * 1)()
    assert lib.ciq_invsqrt_mvm_batched(1, probs, ctypes.byref(o), bp, 2, bp, infos, None) == L.CIQ_ENOTSUP
    t = (ctypes.c_double * 8)(*([1.0] * 8))
    assert lib.ciq_backward(ctypes.byref(p), ctypes.byref(o), L.CIQ_INVSQRT, t, t, fake, fake, 2, 2, None, 2,
                            None, None, None, ctypes.byref(info), None) == L.CIQ_ENOTSUP
    piv = (ctypes.c_int * 20)()
    tr = ctypes.c_double()
    for rank in (0, 11, 1025):
        assert lib.ciq_pivoted_cholesky(ctypes.byref(p), L.CIQ_F32, rank, fake, piv, ctypes.byref(tr), None) \
            == L.CIQ_EINVAL
    assert lib.ciq_pivoted_cholesky(ctypes.byref(p), L.CIQ_F32, 4, None, piv, None, None) == L.CIQ_EINVAL
    assert lib.ciq_pivoted_cholesky(ctypes.byref(p), L.CIQ_F32, 4, fake, None, None, None) == L.CIQ_EINVAL
    assert lib.ciq_pivoted_cholesky(ctypes.byref(p), 9, 4, fake, piv, None, None) == L.CIQ_EINVAL
    del keep, keep0


def test_posterior_arguments_rejected(lib):
    p, keep = _bad_problem()
    o = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4)
    info = L.ciq_info()
    fake = _dev_ptr()
    args = dict(x=fake, n=5, noise=1e-2, mode=L.CIQ_SQRT)
    for bad in [dict(x=None), dict(n=0), dict(n=4097), dict(noise=-1.0), dict(noise=float("nan")), dict(mode=7)]:
        a = {**args, **bad}
        assert lib.ciq_posterior_mvm(ctypes.byref(p), a["x"], a["n"], a["noise"], a["mode"], ctypes.byref(o), fake,
                                     2, 2, fake, 2, ctypes.byref(info), None) == L.CIQ_EINVAL, bad
    o.precond_rank = 4
    assert lib.ciq_posterior_mvm(ctypes.byref(p), fake, 5, 1e-2, L.CIQ_SQRT, ctypes.byref(o), fake, 2, 2, fake, 2,
                                 ctypes.byref(info), None) == L.CIQ_ENOTSUP
    del keep


def test_csr_arguments_rejected(lib):
    fake = _dev_ptr()
    info = L.ciq_info()
    o = L.ciq_opts(dtype=L.CIQ_F64, q=8, max_iter=10, tol=1e-4)
    good = dict(n=10, nnz=30, row_ptr=fake, col_idx=fake, val=fake)
    for bad in [dict(n=0), dict(nnz=-1), dict(row_ptr=None), dict(col_idx=None), dict(val=None)]:
        a = L.ciq_csr(**{**good, **bad})
        assert lib.ciq_csr_mvm(ctypes.byref(a), L.CIQ_INVSQRT, ctypes.byref(o), fake, 2, 2, fake, 2,
                               ctypes.byref(info), None) == L.CIQ_EINVAL, bad
    a = L.ciq_csr(**good)
    assert lib.ciq_csr_mvm(ctypes.byref(a), 5, ctypes.byref(o), fake, 2, 2, fake, 2, ctypes.byref(info),
                           None) == L.CIQ_EINVAL
    assert lib.ciq_csr_mvm(ctypes.byref(a), L.CIQ_SQRT, ctypes.byref(o), fake, 2, 1, fake, 2, ctypes.byref(info),
                           None) == L.CIQ_EINVAL
    o32 = L.ciq_opts(dtype=L.CIQ_F32, q=8, max_iter=10, tol=1e-4)
    assert lib.ciq_csr_mvm(ctypes.byref(a), L.CIQ_SQRT, ctypes.byref(o32), fake, 2, 2, fake, 2, ctypes.byref(info),
                           None) == L.CIQ_ENOTSUP


def test_svgp_arguments_rejected(lib):
    p, keep = _bad_problem()
    fake = _dev_ptr()
    info = L.ciq_info()
    o = L.ciq_opts(dtype=L.CIQ_F64, q=8, max_iter=10, tol=1e-4)
    good = dict(x=fake, nb=4, theta=fake, Theta=fake, it=10, tol=1e-8, mean=fake, var=fake)
    for bad in [dict(x=None), dict(nb=0), dict(theta=None), dict(Theta=None), dict(it=0), dict(tol=-1.0),
                dict(mean=None), dict(var=None)]:
        a = {**good, **bad}
        assert lib.ciq_svgp_predict(ctypes.byref(p), a["x"], a["nb"], a["theta"], a["Theta"], ctypes.byref(o),
                                    a["it"], a["tol"], a["mean"], a["var"], None, ctypes.byref(info), None,
                                    None) == L.CIQ_EINVAL, bad
    o.dtype = L.CIQ_BF16X3
    assert lib.ciq_svgp_predict(ctypes.byref(p), fake, 4, fake, fake, ctypes.byref(o), 10, 1e-8, fake, fake, None,
                                ctypes.byref(info), None, None) == L.CIQ_ENOTSUP
    o.dtype = 9
    assert lib.ciq_svgp_predict(ctypes.byref(p), fake, 4, fake, fake, ctypes.byref(o), 10, 1e-8, fake, fake, None,
                                ctypes.byref(info), None, None) == L.CIQ_EINVAL
    del keep


def test_strerror(lib):
    for code in range(6):
        assert lib.ciq_strerror(code)
    assert b"unknown" in lib.ciq_strerror(99)


def test_release_workspace_rejects_bad_devices(lib):
    # range checks come before any runtime call
    assert lib.ciq_release_workspace(-1) == L.CIQ_EINVAL
    assert lib.ciq_release_workspace(64) == L.CIQ_EINVAL
