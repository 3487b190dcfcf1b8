"""Pins of the oracle's Armijo gradient-projection solver (CPU only)."""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from oracle import model, phantom, solver
from oracle_pins import armijo_trace_errors, floats, worked_example
from workloads import TINY, PhantomSpec, penalty_table, power_start_vector, random_penalties


def test_worked_example_three_iterations_golden():
    """Three hand-worked Armijo iterations, including backtracks."""
    g, D, pen = worked_example()
    res = solver.solve(D, pen, floats(g["x1"]), eps=float(g["eps"]), alpha=float(g["alpha"]),
                       lambda0=float(g["lambda0"]), max_iter=3, fixed_iters=True)
    assert res.status == solver.MAX_ITER and res.iterations == 3
    for e, key in zip(res.trace, ("trace1", "trace2", "trace3")):
        k, lam, m, s, G = floats(g[key])
        assert (e.k, e.lam, e.backtracks, e.step_sq, e.G) == (k, lam, m, s, G)
    assert np.array_equal(res.x, floats(g["x4"]))
    assert res.forward_products == int(g["forward_products"])
    assert res.adjoint_products == int(g["adjoint_products"])
    assert res.G_initial == float(g["G1"])


def test_worked_example_converges_to_known_minimiser():
    g, D, pen = worked_example()
    res = solver.solve(D, pen, floats(g["x1"]), eps=1e-4, alpha=2.0, lambda0=1.0,
                       delta=1e-15, max_iter=5000)
    np.testing.assert_allclose(res.x, floats(g["x_star"]), atol=1e-7)
    assert res.G <= 1e-13


def _dense_problem(seed, nv=60, nb=6):
    rng = np.random.default_rng(seed)
    Dd = rng.uniform(0.0, 1.0, (nv, nb))
    Dd[rng.random((nv, nb)) < 0.3] = 0.0
    return sp.csr_matrix(Dd.astype(np.float32)), rng


def test_unconstrained_least_squares_closed_form():
    """Projection inactive: the solve reaches lstsq(W^1/2 D, W^1/2 T)."""
    D, rng = _dense_problem(20)
    Dd = D.toarray().astype(np.float64)
    x_true = rng.uniform(1.0, 2.0, D.shape[1])
    T = Dd @ x_true + 0.05 * rng.standard_normal(D.shape[0])
    w = rng.uniform(0.5, 1.5, D.shape[0])
    pen = model.VoxelPenalties(T, T, w, w)
    sw = np.sqrt(w)
    x_star = np.linalg.lstsq(sw[:, None] * Dd, sw * T, rcond=None)[0]
    assert np.all(x_star > 0)
    L = 2 * np.linalg.norm(sw[:, None] * Dd, 2) ** 2
    lam0 = solver.power_of_two_at_least(2.0 / L)
    res = solver.solve(D, pen, np.ones(D.shape[1]), eps=1e-4, alpha=2.0, lambda0=lam0,
                       max_iter=4000, fixed_iters=True)
    assert np.linalg.norm(res.x - x_star) / np.linalg.norm(x_star) <= 1e-8
    G_star = float(np.sum(w * (Dd @ x_star - T) ** 2))
    assert abs(res.G - G_star) <= 1e-10 * G_star


def test_active_bounds_match_nnls():
    """Two-sided everywhere: weighted NNLS (scipy.optimize.nnls)."""
    D, rng = _dense_problem(21, nv=80, nb=8)
    Dd = D.toarray().astype(np.float64)
    x_true = rng.uniform(-1.0, 2.0, D.shape[1])
    T = np.maximum(Dd @ x_true, 0.0) + 0.1 * rng.standard_normal(D.shape[0])
    w = rng.uniform(0.5, 1.5, D.shape[0])
    sw = np.sqrt(w)
    x_nn, rnorm = so.nnls(sw[:, None] * Dd, sw * T)
    assert np.any(x_nn == 0)
    pen = model.VoxelPenalties(T, T, w, w)
    L = 2 * np.linalg.norm(sw[:, None] * Dd, 2) ** 2
    res = solver.solve(D, pen, np.ones(D.shape[1]), eps=1e-4, alpha=2.0,
                       lambda0=solver.power_of_two_at_least(2.0 / L), max_iter=20000, fixed_iters=True)
    assert abs(res.G - rnorm ** 2) <= 1e-10 * rnorm ** 2
    np.testing.assert_allclose(res.x, x_nn, atol=1e-7)
    g1 = np.max(np.abs(model.gradient(D, np.ones(D.shape[1]), pen)))
    assert solver.kkt_residual(D, pen, res.x) <= 1e-8 * g1


SMALL_ONE_SIDED = PhantomSpec(name="kkt_16x16x8", nx=16, ny=16, nz=8, h=5.0, r_ptv=12.5,
                              r_rectum=5.0, r_bladder=7.5, n_beams=5, beamlet=10.0,
                              sigma=4.0, tau=0.01)


def test_one_sided_phantom_matches_lbfgsb_and_kkt():
    """One-sided penalties on a small phantom: an independent bound-constrained
    quasi-Newton solve gives the same optimum; the projected-gradient KKT
    residual vanishes; G decreases monotonically under Armijo."""
    D = phantom.build_dose_matrix(SMALL_ONE_SIDED)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(SMALL_ONE_SIDED))
    lam0, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, 0))
    x1 = np.ones(D.nb)
    res = solver.solve(D.csr, pen, x1, eps=1e-4, alpha=2.0, lambda0=lam0,
                       delta=1e-14, max_iter=200000)
    Gs = [e.G for e in res.trace]
    assert all(b < a for a, b in zip(Gs, Gs[1:]))
    ref = so.minimize(lambda x: model.objective(D.csr, x, pen), x1,
                      jac=lambda x: model.gradient(D.csr, x, pen), method="L-BFGS-B",
                      bounds=[(0, None)] * D.nb,
                      options=dict(ftol=1e-16, gtol=1e-12, maxiter=100000, maxfun=200000))
    assert abs(res.G - ref.fun) <= 1e-8 * ref.fun
    # this phantom is ill-conditioned (mirror-symmetric beamlets): ~1e5
    # iterations reach a projected-gradient residual of ~1.5e-8 relative
    g1 = np.max(np.abs(model.gradient(D.csr, x1, pen)))
    assert solver.kkt_residual(D.csr, pen, res.x) <= 1e-7 * g1


def test_armijo_rule_replayed_on_tiny_phantom():
    D = phantom.build_dose_matrix(TINY)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    x1 = np.ones(D.nb)
    # a large lambda_0 forces backtracking in every iteration
    res = solver.solve(D.csr, pen, x1, eps=1e-4, alpha=2.0, lambda0=0.125, max_iter=12,
                       fixed_iters=True)
    assert res.iterations == 12
    assert sum(e.backtracks for e in res.trace) >= 12
    assert armijo_trace_errors(D.csr, pen, x1, res, 1e-4, 2.0, 0.125) == []


def test_random_problem_armijo_replay_with_backtracks():
    D, rng = _dense_problem(22, nv=50, nb=7)
    pens = random_penalties(4, 9, scale=2.0)
    sid = rng.integers(0, 4, D.shape[0])
    pen = model.VoxelPenalties.from_structures(sid, np.array(
        [[p.T_under, p.T_over, p.w_under, p.w_over] for p in pens]))
    x1 = np.full(D.shape[1], 0.5)
    res = solver.solve(D, pen, x1, eps=0.3, alpha=3.0, lambda0=2.0, max_iter=25,
                       fixed_iters=True)
    assert any(e.backtracks > 0 for e in res.trace)
    assert armijo_trace_errors(D, pen, x1, res, 0.3, 3.0, 2.0) == []


def test_lambda0_power_iteration_against_svd():
    D = phantom.build_dose_matrix(SMALL_ONE_SIDED)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(SMALL_ONE_SIDED))
    lam0, s = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, 0), 50)
    smax = np.linalg.svd(D.csr.toarray().astype(np.float64), compute_uv=False)[0]
    assert s <= smax * (1 + 1e-12) and s >= smax * (1 - 1e-6)
    L = 2.0 * 1.0 * s * s          # largest penalty weight is the PTV's 1.0
    assert lam0 >= 2.0 / L and lam0 < 4.0 / L
    assert math.frexp(lam0)[0] == 0.5


@pytest.mark.parametrize("q,want", [(3.0, 4.0), (4.0, 4.0), (0.3, 0.5), (2.0 ** -30, 2.0 ** -30),
                                    (1e-3, 2.0 ** -9), (5.0000001, 8.0)])
def test_power_of_two_at_least(q, want):
    assert solver.power_of_two_at_least(q) == want


def test_stalled_at_stationary_start():
    """x = 0 minimises sum w (Dx)^2 over x >= 0: the first trial equals x_k."""
    D, _ = _dense_problem(23)
    n = D.shape[0]
    pen = model.VoxelPenalties(np.zeros(n), np.zeros(n), np.zeros(n), np.ones(n))
    res = solver.solve(D, pen, np.zeros(D.shape[1]), eps=1e-4, alpha=2.0, lambda0=1.0)
    assert res.status == solver.STALLED and res.iterations == 0


def test_line_search_failure_and_fixed_iteration_count():
    g, D, pen = worked_example()
    res = solver.solve(D, pen, floats(g["x1"]), eps=1e-4, alpha=2.0, lambda0=1.0, max_backtracks=1)
    assert res.status == solver.LS_FAIL and res.iterations == 0
    res = solver.solve(D, pen, floats(g["x1"]), eps=1e-4, alpha=2.0, lambda0=0.25, max_iter=7,
                       fixed_iters=True)
    assert res.status == solver.MAX_ITER and res.iterations == 7
    with pytest.raises(ValueError):
        solver.solve(D, pen, -floats(g["x1"]), eps=1e-4, alpha=2.0, lambda0=1.0)
    with pytest.raises(ValueError):
        solver.solve(D, pen, floats(g["x1"]), eps=1.5, alpha=2.0, lambda0=1.0)


def test_stopping_rule_relative_change():
    """Stops at the first accepted iteration whose relative change is below delta."""
    D = phantom.build_dose_matrix(TINY)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    res = solver.solve(D.csr, pen, np.ones(D.nb), eps=1e-4, alpha=2.0, lambda0=2.0 ** -7,
                       delta=1e-3, max_iter=10000)
    assert res.status == solver.CONVERGED
    Gs = [res.G_initial] + [e.G for e in res.trace]
    rel = [abs(b - a) / b for a, b in zip(Gs, Gs[1:])]
    assert rel[-1] < 1e-3 and all(r >= 1e-3 for r in rel[:-1])


def _one_voxel():
    """One voxel, one beamlet, D = [1], two-sided threshold 4 with unit
    weights: G(x) = (x - 4)^2 and grad G = 2 (x - 4); every value below is a
    dyadic rational, exact in float64."""
    D = sp.csr_matrix(np.array([[1.0]], dtype=np.float32))
    pen = model.VoxelPenalties(np.array([4.0]), np.array([4.0]), np.array([1.0]), np.array([1.0]))
    return D, pen


def test_warm_start_closed_form():
    """Warm start: lambda of iteration k + 1 starts at 2 lambda_k.  From x = 0
    with lambda_0 = 1/8 the steps are 1/8, 1/4, 1/2: x = 1, 2.5, 4, G = 9,
    2.25, 0 (stop at G = 0).  Restarting at lambda_0 instead shrinks the
    error by 3/4 per iteration: G = 16 (9/16)^k."""
    D, pen = _one_voxel()
    w = solver.solve(D, pen, np.zeros(1), eps=1e-4, alpha=2.0, lambda0=0.125, warm_start=True)
    assert w.status == solver.CONVERGED and w.iterations == 3
    assert [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in w.trace] == \
        [(1, 0.125, 0, 1.0, 9.0), (2, 0.25, 0, 2.25, 2.25), (3, 0.5, 0, 2.25, 0.0)]
    assert w.x[0] == 4.0
    c = solver.solve(D, pen, np.zeros(1), eps=1e-4, alpha=2.0, lambda0=0.125, max_iter=3, fixed_iters=True)
    assert [e.lam for e in c.trace] == [0.125] * 3
    assert [e.G for e in c.trace] == [16.0 * (9.0 / 16.0) ** k for k in (1, 2, 3)]


def test_warm_start_with_backtracking_closed_form():
    """lambda_0 = 3/4 overshoots to x = 6 (G = 4); from then on the doubled
    step 3/2 always overshoots (rejected) and 3/4 is accepted after one
    reduction: x = 3, 4.5 with G = 1, 1/4."""
    D, pen = _one_voxel()
    w = solver.solve(D, pen, np.zeros(1), eps=1e-4, alpha=2.0, lambda0=0.75, max_iter=3, fixed_iters=True,
                     warm_start=True)
    assert [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in w.trace] == \
        [(1, 0.75, 0, 36.0, 4.0), (2, 0.75, 1, 9.0, 1.0), (3, 0.75, 1, 2.25, 0.25)]
    assert w.forward_products == 1 + 1 + 2 + 2 and w.x[0] == 4.5
