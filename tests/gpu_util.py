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


def check_trajectory(tr, res, ref, ref_G0, ref_stop, delta=None, tol=1e-6, slack=None):
    """Compare a GPU solve with the oracle's trajectory of the same problem.

    tr: the GPU trace [(k, backtracks, lambda, step_sq, G)] and res its
    result; ref: the oracle's trace [(k, lambda, backtracks, step_sq, G)],
    run at least as far as the GPU's stop index, and ref_G0 its G(x_1);
    ref_stop: the iteration at
    which the oracle stopped (its own stopping rule), None when both ran a
    fixed count; delta: the stopping tolerance when the stopping rule was on.

    Every index: same numbering, backtracks and step; G within tol relative
    (plus `slack(k, G)` absolute when given).  The GPU's final G is compared
    with the oracle's G at the GPU's stop index.  The stop indices agree, or
    the GPU's own trace shows it applied step 5 correctly and the oracle's
    relative change at the first index where the two decisions differ lies
    within what the worst measured G error can move it (a decision that
    close to delta can go either way in float32 arithmetic).
    Returns (worst relative G error, GPU stop index, oracle stop index)."""
    K = len(tr)
    assert K == res.iterations and K <= len(ref), (K, res.iterations, len(ref))
    assert abs(res.G_initial - ref_G0) <= tol * abs(ref_G0), (res.G_initial, ref_G0)
    worst = 0.0
    for (k, m, lam, s, G), (rk, rlam, rm, rs, rG) in zip(tr, ref[:K]):
        assert k == rk and m == rm and lam == rlam, (k, m, rm, lam, rlam)
        bound = tol * abs(rG) + (slack(k, rG) if slack else 0.0)
        assert abs(G - rG) <= bound, (k, G, rG)
        worst = max(worst, abs(G - rG) / abs(rG) if rG else 0.0)
    if K:
        rG = ref[K - 1][4]
        assert abs(res.G_final - rG) <= tol * abs(rG) + (slack(K, rG) if slack else 0.0), (res.G_final, rG)
    if ref_stop is None:
        return worst, K, None
    Gs = [res.G_initial] + [e[4] for e in tr]
    rGs = [ref_G0] + [e[4] for e in ref]

    def stops(g, k):
        return g[k] == 0.0 or abs(g[k] - g[k - 1]) / g[k] < delta

    # the GPU's own stopping decisions
    for k in range(1, K):
        assert not stops(Gs, k), ("GPU continued past its stopping test", k)
    if res.status == 0:
        assert K >= 1 and stops(Gs, K), ("GPU stopped without its test holding", K)
    if K != ref_stop:
        k = min(K, ref_stop)
        rho = abs(rGs[k] - rGs[k - 1]) / rGs[k]
        assert abs(rho - delta) <= 2.0 * worst * (1.0 + rho) + 1e-15, (K, ref_stop, rho, worst)
    return worst, K, ref_stop


def dose_rounding_slack(pen):
    """Absolute G bound from float32 dose rounding at one x: each dose carries
    a relative error of about u = 2^-24 (d_j >= 0 is a sum of nonnegative
    products), and dG/dd_j = 2 r_j, so |dG| <= 2 u sum_j |r_j| d_j
    <= 2 u sqrt(G) sqrt(sum_active w_j d_j^2) by Cauchy-Schwarz with
    r_j^2 / w_j = F_j.  An active voxel has d_j <= T_j + |d_j - T_j|, so
    sum_active w_j d_j^2 <= 2 S + 2 G with S = sum_j (w_u T_u^2 + w_o T_o^2).
    Near the optimum of a long solve G falls to a level where this term, not
    1e-6 G, decides the comparison with the float64 oracle."""
    u = 2.0 ** -24
    S = float(np.sum(pen.w_under * pen.T_under ** 2 + pen.w_over * pen.T_over ** 2))
    return lambda k, G: 2.0 * u * np.sqrt(abs(G) * (2.0 * S + 2.0 * abs(G)))
