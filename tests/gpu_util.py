"""Shared helpers for the GPU parity tests (not collected by pytest: no test_ prefix)."""

import sys

import numpy as np
import pytest

from conftest import gpu_available

needs_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a GPU")


def note(msg):
    """Print what the next GPU step is, flushed, so a fault names its case."""
    print("[gpu-step] " + msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
