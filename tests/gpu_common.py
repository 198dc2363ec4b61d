"""Helpers for the GPU tests: run the same problem through the HIP library and the oracle."""
import sys

import numpy as np
import pytest


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def gpu_sim(prob, dtype="f64", torch=False):
    from paper_1912_04855_amd.sim import from_problem
    return from_problem(prob, dtype=dtype, torch=torch)


def announce(*a):
    """Name the case before a GPU step, flushed, so a crash log says which case ran."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l1(a, b):
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / den) if den > 0 else float(np.sum(np.abs(a - b)))


def rel_l1_vars(a, b):
    """Largest per-variable relative L1 distance (each conserved variable on its own scale)."""
    out = []
    for v in range(a.shape[0]):
        den = np.sum(np.abs(b[v]))
        num = np.sum(np.abs(a[v] - b[v]))
        out.append(float(num / den) if den > 0 else float(num))
    return max(out)
