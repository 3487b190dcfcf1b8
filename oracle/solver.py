"""FP64 oracle: gradient projection with Armijo's line search (Section 2.2).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.

The iteration follows the paper's initialisation and five steps:

  init   x_1 >= 0; choose eps in (0, 1), alpha > 1, lambda_0; k = 1
  1      search direction -grad G(x_k)
  2      lambda = lambda_0; trial x_{k+1} = max(0, x_k - lambda grad G(x_k))
  3      accept when G(x_{k+1}) < C_k, where Eq. (5) gives
         C_k = G(x_k) - (eps/lambda) * ||x_{k+1} - x_k||^2
  4      otherwise lambda = lambda/alpha, recompute the trial, back to 3
  5      stop when the relative change of G is below delta, else k = k + 1

Readings taken where the paper is silent or garbled:
  * Eq. (5) multiplies a row vector by its transpose: the squared Euclidean
    norm of the step.  C_k is recomputed for every trial lambda.
  * lambda restarts from lambda_0 in every iteration (step 2).  A variant
    (``warm_start``, not the paper's step 2) starts iteration k + 1 at alpha
    times the step accepted in iteration k; the first iteration starts at
    lambda_0.
  * Step 5 is applied after acceptance to the newest pair,
    |G_{k+1} - G_k| / G_{k+1} < delta; G_{k+1} == 0 also stops.
  * A trial with ||x_{k+1} - x_k|| == 0 can never pass the strict test of
    step 3; the solve then stops as "stalled" (x_k is a stationary point).
  * The line search gives up after ``max_backtracks`` reductions.
  * The dose of the accepted trial feeds the next gradient (identical in
    exact arithmetic to recomputing it).
  * lambda_0 is not given in the paper: ``lambda0_from_power_iteration``
    takes the smallest power of two >= 2/L, with L = 2 * max weight *
    sigma_max(D)^2 and sigma_max from a seeded power iteration.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import model

CONVERGED, MAX_ITER, STALLED, LS_FAIL, NUMERIC = 0, 1, 2, 3, 4
STATUS_NAMES = {CONVERGED: "converged", MAX_ITER: "max_iter", STALLED: "stalled",
                LS_FAIL: "line_search_failed", NUMERIC: "non_finite"}


@dataclass
class TraceEntry:
    k: int            # accepted iteration count after this step
    lam: float        # accepted step size
    backtracks: int   # number of lambda reductions in this line search
    step_sq: float    # ||x_{k+1} - x_k||^2
    G: float          # G(x_{k+1})


@dataclass
class SolveResult:
    x: np.ndarray
    G: float
    status: int
    iterations: int
    forward_products: int
    adjoint_products: int
    G_initial: float
    trace: List[TraceEntry] = field(default_factory=list)
    dose: Optional[np.ndarray] = None


def lambda0_from_power_iteration(D, pen: model.VoxelPenalties, v0: np.ndarray,
                                 iters: int = 50):
    """Initial Armijo step lambda_0 = smallest power of two >= 2 / L.

    L = 2 * max_j max(w_u,j, w_o,j) * s^2, where s^2 = ||D v||^2 for the unit
    vector v reached by ``iters`` power iterations v <- D^T D v / ||D^T D v||
    from ``v0``.  Returns (lambda_0, s).
    """
    Df = model.as_f64_matrix(D)
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    for _ in range(iters):
        w = Df.T @ (Df @ v)
        v = w / np.linalg.norm(w)
    dv = Df @ v
    s2 = float(dv @ dv)
    wmax = float(max(np.max(pen.w_under, initial=0.0), np.max(pen.w_over, initial=0.0)))
    L = 2.0 * wmax * s2
    return power_of_two_at_least(2.0 / L), math.sqrt(s2)


def power_of_two_at_least(q: float) -> float:
    """Smallest power of two that is >= q (q > 0, finite)."""
    mant, ex = math.frexp(q)
    return q if mant == 0.5 else math.ldexp(1.0, ex)


def solve(D, pen: model.VoxelPenalties, x1: np.ndarray, *, eps: float, alpha: float,
          lambda0: float, delta: float = 1e-5, max_iter: int = 20000,
          max_backtracks: int = 60, fixed_iters: bool = False,
          keep_trace: bool = True, warm_start: bool = False) -> SolveResult:
    """Run the Armijo gradient-projection method from ``x1`` (float64)."""
    if not (0.0 < eps < 1.0) or not (alpha > 1.0) or not (lambda0 > 0.0):
        raise ValueError("need 0 < eps < 1, alpha > 1, lambda0 > 0")
    x = np.asarray(x1, dtype=np.float64).copy()
    if np.any(x < 0) or not np.all(np.isfinite(x)):
        raise ValueError("x1 must be finite and >= 0")
    Df = model.as_f64_matrix(D)
    z = Df @ x
    G = model.objective_from_dose(z, pen)
    G_init = G
    n_fwd, n_adj, k = 1, 0, 0
    lam_start = lambda0
    trace: List[TraceEntry] = []
    status = None
    if max_iter <= 0:
        status = MAX_ITER
    while status is None:
        g = 2.0 * (Df.T @ model.residual(z, pen))        # step 1
        n_adj += 1
        lam, m = lam_start, 0                             # step 2
        while True:
            xt = model.project(x - lam * g)
            step = xt - x
            s = float(step @ step)
            if s == 0.0:
                status = STALLED
                break
            zt = Df @ xt
            n_fwd += 1
            Gt = model.objective_from_dose(zt, pen)
            if not math.isfinite(Gt):
                status = NUMERIC
                break
            C = G - (eps / lam) * s                       # Eq. (5)
            if Gt < C:                                    # step 3
                break
            m += 1                                        # step 4
            if m > max_backtracks:
                status = LS_FAIL
                break
            lam = lam / alpha
        if status is not None:
            break
        G_prev = G
        x, z, G = xt, zt, Gt
        k += 1
        if warm_start:
            lam_start = alpha * lam
        if keep_trace:
            trace.append(TraceEntry(k, lam, m, s, G))
        if fixed_iters:                                   # step 5
            if k >= max_iter:
                status = MAX_ITER
        elif G == 0.0 or abs(G - G_prev) / G < delta:
            status = CONVERGED
        elif k >= max_iter:
            status = MAX_ITER
    return SolveResult(x=x, G=G, status=status, iterations=k, forward_products=n_fwd,
                       adjoint_products=n_adj, G_initial=G_init, trace=trace, dose=z)


def kkt_residual(D, pen: model.VoxelPenalties, x: np.ndarray) -> float:
    """Projected-gradient residual ||x - max(0, x - grad G(x))||_inf."""
    g = model.gradient(D, x, pen)
    return float(np.max(np.abs(x - model.project(x - g)), initial=0.0))
