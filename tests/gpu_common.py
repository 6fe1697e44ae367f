"""Shared helpers for the GPU parity tests (inputs come from `workloads`,
expected values from `oracle`)."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def dev():
    return torch.device("cuda", 0)


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def announce(msg):
    """Name the case before any GPU work, flushed, so a fault is attributable."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()
