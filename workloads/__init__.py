"""Seeded synthetic inputs for the CIQ workloads.

This module only draws random inputs (points, right-hand sides, lengthscales,
batch shapes). It contains none of the method's arithmetic, so both the CPU
oracle and the HIP path can take their inputs from here without sharing any
computation.

Recipe (one per workload, numpy ``default_rng``): points are i.i.d.
Uniform[0, 1]^d, right-hand sides i.i.d. N(0, 1), ARD lengthscales
log-uniform on the stated interval. Every array is drawn in float64 and
rounded once to the dtype the GPU path consumes; both sides see the rounded
values. Seed of workload ``c`` for stream ``k`` is ``1000 * c + k`` with
k = 1 points, 2 right-hand sides, 3 lengthscales, 4 Lanczos start vector,
5 batch shapes.

The stand-ins: the paper's Bayesian-optimisation candidate sets live on the
unit cube, d = 6 with 50k candidates matches its Hartmann-6 posterior
sampling, d = 8 matches the input width of its Kin40k timing study, and
M = 5000 inducing points on a 10-d cube matches its SVGP whitening runs. None
of the paper's datasets is used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

RBF = "rbf"
MATERN52 = "matern52"


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_points(n: int, d: int, seed: int, dtype=np.float32) -> np.ndarray:
    """n x d points, i.i.d. Uniform[0,1], row-major, rounded to ``dtype``."""
    return _rng(seed).random((n, d)).astype(dtype)


def gaussian_rhs(n: int, s: int, seed: int, dtype=np.float32) -> np.ndarray:
    """n x s right-hand sides, i.i.d. N(0,1), rounded to ``dtype``."""
    return _rng(seed).standard_normal((n, s)).astype(dtype)


def loguniform(k: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """k values log-uniform on [lo, hi] (float64)."""
    u = _rng(seed).random(k)
    return np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


def start_vector(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Random start vector for the extreme-eigenvalue Lanczos run (N(0,1))."""
    return _rng(seed).standard_normal(n).astype(dtype)


@dataclass
class Problem:
    """One kernel matrix K = o^2 k(X, X) + sigma^2 I and its right-hand sides."""

    kernel: str
    x: np.ndarray            # n x d, rounded to the GPU input dtype
    lengthscale: np.ndarray  # length 1 (isotropic) or d (ARD), float64
    outputscale: float       # o^2
    noise: float             # sigma^2
    b: np.ndarray            # n x s

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def d(self) -> int:
        return self.x.shape[1]

    @property
    def s(self) -> int:
        return self.b.shape[1]


@dataclass
class Workload:
    name: str
    dtype: str               # "f64", "f32", "bf16x3", "f16x3"
    q: int
    max_iter: int
    tol: float
    problems: List[Problem] = field(default_factory=list)
    note: str = ""


def _np_dtype(dtype: str):
    return np.float64 if dtype == "f64" else np.float32


def workload(c: int, *, n: Optional[int] = None, s: Optional[int] = None,
             dtype: Optional[str] = None, n_problems: Optional[int] = None) -> Workload:
    """The five reference workloads; ``n``/``s`` shrink a workload for tests."""
    base = 1000 * c
    if c == 1:
        dt = dtype or "f64"
        nn, ss = n or 1024, s or 1
        x = uniform_points(nn, 3, base + 1, _np_dtype(dt))
        b = gaussian_rhs(nn, ss, base + 2, _np_dtype(dt))
        p = Problem(RBF, x, np.array([0.2]), 1.0, 1e-2, b)
        return Workload("rbf_n1024_d3_s1_fp64", dt, 8, 100, 1e-4, [p])
    if c == 2:
        dt = dtype or "f32"
        nn, ss = n or 50_000, s or 64
        x = uniform_points(nn, 6, base + 1, _np_dtype(dt))
        b = gaussian_rhs(nn, ss, base + 2, _np_dtype(dt))
        p = Problem(MATERN52, x, np.array([0.3]), 1.0, 1e-3, b)
        return Workload(f"matern52_n{nn}_d6_s{ss}", dt, 15, 200, 1e-4, [p])
    if c == 3:
        dt = dtype or "bf16x3"
        nn, ss = n or 100_000, s or 256
        x = uniform_points(nn, 8, base + 1, np.float32)
        b = gaussian_rhs(nn, ss, base + 2, np.float32)
        ls = loguniform(8, 0.1, 1.0, base + 3)
        p = Problem(RBF, x, ls, 1.0, 1e-3, b)
        return Workload(f"rbf_ard_n{nn}_d8_s{ss}", dt, 15, 1000, 1e-4, [p])
    if c == 4:
        dt = dtype or "f32"
        P = n_problems or 64
        r = _rng(base + 5)
        lo, hi = 2000, 20000
        ns = np.exp(np.log(lo) + r.random(P) * (np.log(hi) - np.log(lo))).astype(int)
        ds = r.integers(2, 11, size=P)
        if n is not None:  # shrink every problem proportionally for tests
            ns = np.maximum(1, (ns * n) // hi)
        ss = s or 16
        probs = []
        for p_i in range(P):
            x = uniform_points(int(ns[p_i]), int(ds[p_i]), base + 1 + 10 * p_i, np.float32)
            b = gaussian_rhs(int(ns[p_i]), ss, base + 2 + 10 * p_i, np.float32)
            probs.append(Problem(RBF, x, np.array([0.25]), 1.0, 1e-2, b))
        return Workload(f"batched_p{P}_rbf_s{ss}", dt, 12, 1000, 1e-4, probs)
    if c == 5:
        dt = dtype or "f32"
        nn, ss = n or 5000, s or 256
        x = uniform_points(nn, 10, base + 1, np.float32)
        b = gaussian_rhs(nn, ss, base + 2, np.float32)
        ls = loguniform(10, 0.1, 1.0, base + 3)
        p = Problem(RBF, x, ls, 1.0, 1e-4, b)
        return Workload(f"svgp_whiten_m{nn}_d10_s{ss}", dt, 15, 200, 1e-3, [p])
    raise ValueError(f"unknown workload {c}")
