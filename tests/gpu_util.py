"""Shared helpers for the GPU parity tests (not collected by pytest: no test_ prefix)."""

import os
import sys
import time

import numpy as np
import pytest

from conftest import gpu_available

needs_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a GPU")


def note(msg):
    """Print what the next GPU step is, flushed, so a fault names its case.  With
    MGIC_PROGRESS_FILE set, the line is also appended to that file (pytest captures stdout, so
    long steps leave their progress there)."""
    print("[gpu-step] " + msg, flush=True)
    sys.stdout.flush()
    path = os.environ.get("MGIC_PROGRESS_FILE")
    if path:
        with open(path, "a") as fh:
            fh.write("%.1f %s\n" % (time.time(), msg))


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
