"""Helpers shared by the GPU parity tests (imported only when a GPU is used)."""
import numpy as np
import scipy.sparse as sp


def f32_ulp_diff(a: np.ndarray, b: np.ndarray) -> int:
    """Largest distance in units in the last place between two float32 arrays
    of nonnegative finite values."""
    ia = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return int(np.max(np.abs(ia - ib), initial=0))


def csr_of(A):
    """scipy CSR from a workloads.RandomCSR."""
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))


def to_dev(arr, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_normwise(got, want) -> float:
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    den = max(np.max(np.abs(want), initial=0.0), 1e-300)
    return float(np.max(np.abs(got - want), initial=0.0) / den)


def banner(msg: str):
    print(f"[gpu] {msg}", flush=True)
