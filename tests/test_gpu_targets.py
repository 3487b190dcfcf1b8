"""Matrices partitioned by per-plan targets (the rule of the batch search and
the server) take 8-wave forward workgroups, several side by side on a compute
unit -- as many as the registers and the LDS that the staged vectors of nb
beamlets need allow.  For nb that fit three, two and one such workgroup per
compute unit: products, objective and a short Armijo trajectory against the
FP64 oracle, and the solve alone equal to the same solve batched with another
plan."""
import numpy as np
import pytest

from gpu_util import banner, check_trajectory, csr_of, to_dev, to_host
from oracle import model, solver
from workloads import power_start_vector, random_csr, random_penalties

pytestmark = pytest.mark.gpu

ITERS = 25


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


def _problem(ctx, nb, seed):
    from paper_0908_4421_amd.imrt import Dose, Plan
    A = random_csr(30000, nb, 25.0, seed, empty_frac=0.25, nstruct=4)
    pens = random_penalties(4, seed, scale=3.0)
    table = np.array([[p.T_under, p.T_over, p.w_under, p.w_over] for p in pens])
    lib = Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)
    lib.repartition_targets(128, 32)
    plan = Plan(ctx, lib)
    plan.set_structures(A.struct_id, 4)
    plan.set_penalties(table)
    return A, table, lib, plan


@pytest.mark.parametrize("nb", [700, 9000, 20000])
def test_target_partition_against_oracle(ctx, nb):
    A, table, lib, plan = _problem(ctx, nb, 40 + nb % 97)
    D = csr_of(A)
    pen = model.VoxelPenalties.from_structures(A.struct_id, table)
    rng = np.random.default_rng(nb)
    x = rng.uniform(0, 0.6, A.nb).astype(np.float32)
    r = rng.standard_normal(A.nv).astype(np.float32)
    d = to_host(lib.apply(to_dev(x)))
    d_ref = model.dose(D, x.astype(np.float64))
    assert np.all(np.abs(d - d_ref) <= 1e-5 * np.abs(d_ref) + 1e-30)
    y = to_host(lib.apply_transpose(to_dev(r)))
    y_ref = model.adjoint(D, r.astype(np.float64))
    assert np.all(np.abs(y - y_ref) <= 1e-6 * (abs(D).T @ np.abs(r.astype(np.float64))) + 1e-30)
    G = plan.objective(to_dev(x))
    G_ref = model.objective(D, x.astype(np.float64), pen)
    assert abs(G - G_ref) <= 1e-6 * G_ref
    lam0, _ = solver.lambda0_from_power_iteration(D, pen, power_start_vector(A.nb, 3), 30)
    ref = solver.solve(D, pen, np.ones(A.nb), eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=ITERS,
                       fixed_iters=True)
    xs = to_dev(np.ones(A.nb, np.float32))
    res, tr = plan.solve(xs, eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=ITERS, fixed_iters=True, trace=True)
    worst, K, _ = check_trajectory(tr, res, [[e.k, e.lam, e.backtracks, e.step_sq, e.G] for e in ref.trace],
                                   ref.G_initial, None)
    banner(f"targets, nb {nb}: {K} iterations, worst G error {worst:.1e}")


def test_target_partition_batched_equals_alone(ctx):
    from paper_0908_4421_amd.imrt import Plan
    probs = [_problem(ctx, nb, s) for nb, s in ((9000, 7), (20000, 8))]
    lams = [2.0 ** -9, 2.0 ** -9]
    solo = []
    for (_, _, lib, plan), lam in zip(probs, lams):
        x = to_dev(np.ones(lib.nb, np.float32))
        res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=ITERS, fixed_iters=True, trace=True)
        solo.append((res, tr, to_host(x)))
    xs = [to_dev(np.ones(p[2].nb, np.float32)) for p in probs]
    out = Plan.solve_batch([p[3] for p in probs], xs, eps=1e-4, alpha=2.0, lambda0s=lams, max_iter=ITERS,
                           fixed_iters=True, trace=True)
    for (rs, ts, x_solo), (rb, tb), xb in zip(solo, out, xs):
        assert tb == ts
        assert (rb.iterations, rb.status, rb.G_final) == (rs.iterations, rs.status, rs.G_final)
        assert np.array_equal(to_host(xb), x_solo)
