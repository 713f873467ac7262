"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(gpu, ref):
    """Per-channel |gpu - ref| / |ref| (ref > 0 for exp outputs)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(gpu - ref) / np.abs(ref)


def assert_rel(gpu, ref, tol, what=""):
    e = rel_err(gpu, ref)
    worst = float(np.max(e)) if e.size else 0.0
    assert worst <= tol, f"{what}: max rel err {worst:.3e} > {tol:.1e} " \
                         f"(p99.9 {np.quantile(e, 0.999):.3e}, above tol: {int((e > tol).sum())})"
    return worst
