"""The host symmetric eigensolvers of the library (cyclic Jacobi for the
Lanczos tridiagonal of the eigenvalue bounds; Householder + implicit QR for
the preconditioner's Gram matrix), compiled from their source with g++ and
checked against LAPACK (numpy.linalg.eigh) on CPU: eigenvalues, residual
||A V - V diag(lam)|| and orthogonality, including rank-deficient, repeated
and indefinite cases."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2006_11267_amd", "csrc", "elliptic.cpp")

DRIVER = r'''
#include <vector>
#include <cstdio>
#include <cstdlib>
#include <cstring>
namespace ciq {
void sym_eig_jacobi(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v);
void sym_eig_tridiag(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v);
}
int main(int argc, char** argv) {
    int n = atoi(argv[2]);
    std::vector<double> a((size_t)n * n), ev, v;
    FILE* f = fopen(argv[3], "rb");
    if (fread(a.data(), 8, a.size(), f) != a.size()) return 1;
    fclose(f);
    if (strcmp(argv[1], "jacobi") == 0) ciq::sym_eig_jacobi(n, a, ev, v);
    else ciq::sym_eig_tridiag(n, a, ev, v);
    f = fopen(argv[4], "wb");
    fwrite(ev.data(), 8, n, f);
    fwrite(v.data(), 8, v.size(), f);
    fclose(f);
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("eig")
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + os.path.join(ROOT, "include"), str(d / "drv.cpp"), SRC, "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot compile the host eigensolver: " + r.stderr[:300])
    return d, exe


def _eig(driver, method, A):
    d, exe = driver
    n = A.shape[0]
    A.astype(np.float64).tofile(d / "a.bin")
    subprocess.run([str(exe), method, str(n), str(d / "a.bin"), str(d / "o.bin")], check=True)
    raw = np.fromfile(d / "o.bin")
    return raw[:n], raw[n:].reshape(n, n)


def _cases():
    rng = np.random.default_rng(0)
    out = []
    for n in (1, 2, 3, 7, 40, 150, 400):      # from n = 128 on, the tridiagonal solver runs on a thread team
        X = rng.standard_normal((3 * n, n)) * np.exp(-0.05 * np.arange(n))
        out.append((f"gram{n}", X.T @ X))
    X = rng.standard_normal((80, 25))
    out.append(("rank25", X @ X.T))
    out.append(("identity", np.eye(12)))
    out.append(("repeated", np.diag([1.0, 1.0, 2.0, 2.0, 2.0, 3.0])))
    out.append(("zero", np.zeros((4, 4))))
    B = rng.standard_normal((30, 30))
    out.append(("indefinite", B + B.T))
    L = np.zeros((60, 20))
    L[:, :12] = rng.standard_normal((60, 12))
    out.append(("zero_columns", L.T @ L))
    return out


@pytest.mark.parametrize("method", ["jacobi", "tridiag"])
@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] for c in _cases()])
def test_host_eigensolver(driver, method, name, A):
    lam, V = _eig(driver, method, A)
    n = A.shape[0]
    scale = max(np.abs(A).max(), 1e-300)
    ref = np.linalg.eigvalsh(A)
    assert np.abs(np.sort(lam) - ref).max() <= 1e-13 * scale * max(1, n / 10)
    assert np.abs(A @ V - V * lam).max() <= 1e-13 * scale * max(1, n / 10)
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-13 * max(1, n / 10)
