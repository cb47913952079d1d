"""Shared helpers of the test suite: error metrics and tensor plumbing.

Holds no force, integrator or ordering arithmetic: the expected values always
come from the oracle, the HIP values from the library."""
import numpy as np
import pytest


def rms_rel(a, ref):
    """sqrt(mean_i (|a_i - ref_i| / |ref_i|)^2) over rows (vectors) or entries."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if a.ndim == 1:
        a, ref = a[:, None], ref[:, None]
    num = np.linalg.norm(a - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return float(np.sqrt(np.mean((num / den) ** 2)))


def max_rel(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if a.ndim == 1:
        a, ref = a[:, None], ref[:, None]
    return float(np.max(np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)))


def normwise(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_2292_amd as nb
    nb.lib()
    return torch, nb


def to_dev(torch, arr, dtype):
    return torch.as_tensor(np.ascontiguousarray(arr), dtype=dtype).cuda().contiguous()


def host(t):
    return t.detach().cpu().double().numpy()


def widen32(arr):
    """The exact FP32 values a FP32 kernel sees, widened to FP64."""
    return np.asarray(arr, dtype=np.float32).astype(np.float64)
