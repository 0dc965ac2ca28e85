"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def ciq_module():
    import paper_2006_11267_amd as ciq
    ciq.load()   # raises if the HIP library is missing: no fallback
    return ciq


def announce(msg: str) -> None:
    print(f"\n[gpu-case] {msg}", flush=True)


def colwise_rel(a, ref):
    a = np.asarray(a, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    return np.linalg.norm(a - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
