#!/usr/bin/env python3
"""Writes the oracle's reference K^{-1/2}B and K^{1/2}B for the first columns
of the large Matern-5/2 workload (N = 50,000 points on [0,1]^6, lengthscale
0.3, outputscale 1, noise 1e-3, Q = 15).

Only the oracle and the seeded input generators are used: the dense FP64
kernel matrix is assembled row block by row block with the oracle's
``kernel_rows`` (20 GB in host memory), the extreme-eigenvalue bounds come
from the oracle's Lanczos estimate (App. B.2) started from the workload's
seeded start vector, and the solve is the oracle's msMINRES-CIQ (Alg. S1,
App. C) run to a relative residual of 1e-10, far below the 1e-4 level the
GPU paths are held to. The square root is K times the inverse root (Sec. 3,
the rational approximation), the oracle's own composition.

Outputs (next to this script):
  matern52_n50000_s8_invsqrt.npy, matern52_n50000_s8_sqrt.npy   (N x 8, float64)
  matern52_n50000_s8_reference.json                            (bounds, iterations, residuals, command)

Run: python tests/golden/make_matern52_n50000_reference.py  (about an hour on 8 cores).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ciq as ociq          # noqa: E402
from oracle import kernels as okern     # noqa: E402
from oracle import lanczos as olan      # noqa: E402
import workloads                        # noqa: E402

COLUMNS = 8
Q = 15
TOL = 1e-10
MAX_ITER = 20000
BOUND_STEPS = 20


def main() -> int:
    wl = workloads.workload(2)
    p = wl.problems[0]
    n = p.n
    x = p.x.astype(np.float64)                  # the FP32-rounded points every path consumes
    b = p.b[:, :COLUMNS].astype(np.float64)
    t0 = time.perf_counter()
    K = np.empty((n, n))
    for r0 in range(0, n, 500):
        rows = np.arange(r0, min(r0 + 500, n))
        K[r0:r0 + rows.size] = okern.kernel_rows(p.kernel, x, p.lengthscale, p.outputscale, p.noise, rows)
    print(f"K assembled in {time.perf_counter() - t0:.0f} s", flush=True)

    calls = [0]
    t_start = time.perf_counter()

    def mvm(v):
        calls[0] += 1
        if calls[0] % 100 == 0:
            print(f"  product {calls[0]} at {time.perf_counter() - t_start:.0f} s", flush=True)
        return K @ v

    v0 = workloads.start_vector(n, 2004, dtype=np.float64)
    lo, hi, th_lo, th_hi = olan.eig_bounds(mvm, v0, BOUND_STEPS, p.noise)
    print(f"bounds [{lo:.6g}, {hi:.6g}] (Ritz values [{th_lo:.6g}, {th_hi:.6g}])", flush=True)

    inv, info = ociq.ciq(mvm, b, lo, hi, Q, MAX_ITER, TOL, mode="invsqrt")
    sq = mvm(inv)                              # K^{1/2} B = K (K^{-1/2} B)
    print(f"msMINRES: {info.iters} iterations, converged {bool(info.converged.all())}, "
          f"max rel residual {info.rel_residual.max():.3e}", flush=True)

    np.save(os.path.join(HERE, "matern52_n50000_s8_invsqrt.npy"), inv)
    np.save(os.path.join(HERE, "matern52_n50000_s8_sqrt.npy"), sq)
    meta = {
        "about": ("Oracle (CPU, FP64) K^{-1/2}B and K^{1/2}B for the first 8 right-hand sides of the "
                  "Matern-5/2 workload: N = 50,000 points Uniform[0,1]^6 (seed 2001, rounded to FP32), "
                  "lengthscale 0.3, outputscale 1, noise 1e-3, B ~ N(0,1) (seed 2002, rounded to FP32), "
                  "Q = 15 HHT shifts, msMINRES to relative residual 1e-10."),
        "written_by": "tests/golden/make_matern52_n50000_reference.py",
        "columns": COLUMNS, "n": n, "q": Q, "tol": TOL, "max_iter": MAX_ITER,
        "lambda_min": lo, "lambda_max": hi, "ritz_min": th_lo, "ritz_max": th_hi,
        "bound_steps": BOUND_STEPS, "bound_start_seed": 2004,
        "iters": int(info.iters), "converged": bool(info.converged.all()),
        "max_rel_residual": float(info.rel_residual.max()),
        "col_iters": [int(c) for c in info.col_iters],
        "seconds": time.perf_counter() - t0,
    }
    with open(os.path.join(HERE, "matern52_n50000_s8_reference.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print("written", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
