"""Batched solve (imrt_solve_batch) on the GPU: every plan of a batch of
uneven instances ends bit-identical to its solo solve (trace, final state and
x), including plans that share one dose matrix, plans that finish at
different iterations, 16-bit storage, and the argument checks."""
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from workloads import (SMALL, TINY, PAPER_SCALE_SETTINGS, draw_batch_instance, penalty_table,
                       power_start_vector, random_penalties)

pytestmark = pytest.mark.gpu

ST = PAPER_SCALE_SETTINGS


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


def _plan(ctx, dose, table):
    from paper_0908_4421_amd.imrt import Plan
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(table)
    return plan


def _lambda0(plan, dose, seed):
    return plan.lambda0(to_dev(power_start_vector(dose.nb, seed).astype(np.float32)), ST.power_iters)[0]


def _solo_then_batch(plans, doses, lams, **kw):
    from paper_0908_4421_amd.imrt import Plan
    solo = []
    for plan, dose, lam in zip(plans, doses, lams):
        x = to_dev(np.full(dose.nb, ST.x0, np.float32))
        res, tr = plan.solve(x, eps=ST.eps, alpha=ST.alpha, lambda0=lam, trace=True, **kw)
        solo.append((res, tr, to_host(x)))
    xs = [to_dev(np.full(d.nb, ST.x0, np.float32)) for d in doses]
    out = Plan.solve_batch(plans, xs, eps=ST.eps, alpha=ST.alpha, lambda0s=lams, trace=True, **kw)
    for (rs, ts, xs_solo), (rb, tb), xb in zip(solo, out, xs):
        assert tb == ts
        assert (rb.iterations, rb.status, rb.forward_passes, rb.adjoint_passes) == \
            (rs.iterations, rs.status, rs.forward_passes, rs.adjoint_passes)
        assert rb.G_final == rs.G_final and rb.G_initial == rs.G_initial
        assert np.array_equal(to_host(xb), xs_solo)
    return solo, out


def test_uneven_instances_bit_identical_to_solo(ctx):
    from paper_0908_4421_amd.imrt import Dose
    specs = [TINY, SMALL] + [draw_batch_instance(s) for s in (100, 101, 102, 105)]
    banner("batch of " + ", ".join(s.name for s in specs))
    doses = [Dose.from_geometry(ctx, s) for s in specs]
    plans = [_plan(ctx, d, penalty_table(s)) for d, s in zip(doses, specs)]
    lams = [_lambda0(p, d, s.seed) for p, d, s in zip(plans, doses, specs)]
    solo, _ = _solo_then_batch(plans, doses, lams, delta=ST.delta, max_iter=3000)
    iters = [r.iterations for r, _, _ in solo]
    banner(f"iterations per plan {iters}")
    assert len(set(iters)) > 1          # the plans finish at different iterations


def test_shared_dose_matrix_and_fixed_iterations(ctx):
    """Two plans on one dose matrix with different penalties (new thresholds
    for a resident patient), plus a third plan; fixed iteration counts differ
    per plan through the stopping test being off and max_iter equal."""
    from paper_0908_4421_amd.imrt import Dose
    d0 = Dose.from_geometry(ctx, SMALL)
    d1 = Dose.from_geometry(ctx, TINY)
    t0 = penalty_table(SMALL)
    t1 = t0.copy()
    t1[0, :2] = 66.0      # PTV threshold of a re-plan
    t1[1:, 1] *= 1.05
    plans = [_plan(ctx, d0, t0), _plan(ctx, d0, t1), _plan(ctx, d1, penalty_table(TINY))]
    doses = [d0, d0, d1]
    lams = [_lambda0(p, d, 3) for p, d in zip(plans, doses)]
    _solo_then_batch(plans, doses, lams, max_iter=150, fixed_iters=True)


def test_random_penalties_and_bf16_storage(ctx):
    from paper_0908_4421_amd.imrt import Dose
    specs = [SMALL, draw_batch_instance(103), draw_batch_instance(104)]
    doses = [Dose.from_geometry(ctx, s, storage="bf16") for s in specs]
    tables = [np.array([[p.T_under, p.T_over, p.w_under, p.w_over] for p in random_penalties(4, 40 + i, 50.0)])
              for i in range(3)]
    plans = [_plan(ctx, d, t) for d, t in zip(doses, tables)]
    lams = [_lambda0(p, d, 7) for p, d in zip(plans, doses)]
    _solo_then_batch(plans, doses, lams, delta=ST.delta, max_iter=2000)


def test_batch_argument_checks(ctx):
    from paper_0908_4421_amd import imrt
    from paper_0908_4421_amd.imrt import Dose, Plan
    d = Dose.from_geometry(ctx, TINY)
    d16 = Dose.from_geometry(ctx, TINY, storage="f16")
    p = _plan(ctx, d, penalty_table(TINY))
    p16 = _plan(ctx, d16, penalty_table(TINY))
    x = to_dev(np.ones(d.nb, np.float32))
    y = to_dev(np.ones(d.nb, np.float32))
    for plans in ([p, p], [p, p16]):
        with pytest.raises(imrt.ImrtError) as e:
            Plan.solve_batch(plans, [x, y], eps=1e-4, alpha=2.0, lambda0s=[2.0 ** -7] * 2, max_iter=5)
        assert e.value.code == imrt.IMRT_EINVAL
    with pytest.raises(imrt.ImrtError) as e:
        Plan.solve_batch([p], [to_dev(-np.ones(d.nb, np.float32))], eps=1e-4, alpha=2.0, lambda0s=[2.0 ** -7],
                         max_iter=5)
    assert e.value.code == imrt.IMRT_EINVAL
    # per-plan targets give a matrix 8-wave forward workgroups, a new matrix
    # 16-wave ones: one batched dispatch cannot hold both
    d2 = Dose.from_geometry(ctx, TINY)
    p2 = _plan(ctx, d2, penalty_table(TINY))
    d2.repartition_targets(128, 32)
    with pytest.raises(imrt.ImrtError) as e:
        Plan.solve_batch([p, p2], [x, y], eps=1e-4, alpha=2.0, lambda0s=[2.0 ** -7] * 2, max_iter=5)
    assert e.value.code == imrt.IMRT_EINVAL and "workgroup size" in str(e.value)


def test_repartition_and_autotune(ctx):
    """Coarser work partitions (as a batch prefers) keep every product within
    the oracle's bounds and the batch bit-identical to solo; the autotuner
    leaves one of its candidates applied to every dose matrix."""
    from oracle import model
    from paper_0908_4421_amd.imrt import Dose, Plan
    from gpu_util import csr_of
    from workloads import random_csr
    A = random_csr(20000, 300, 30.0, 21, empty_frac=0.3)
    d = Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)
    D = csr_of(A)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2, A.nb).astype(np.float32)
    r = rng.standard_normal(A.nv).astype(np.float32)
    for adj, bpw in ((1024, 1), (4096, 2), (65536, 8), (16, 1)):
        d.repartition(adj, bpw)
        assert d.partition() == (adj, bpw)
        dd = to_host(d.apply(to_dev(x)))
        yy = to_host(d.apply_transpose(to_dev(r)))
        d_ref = model.dose(D, x.astype(np.float64))
        y_ref = model.adjoint(D, r.astype(np.float64))
        assert np.all(np.abs(dd - d_ref) <= 1e-5 * np.abs(d_ref) + 1e-30)
        assert np.all(np.abs(yy - y_ref) <= 1e-6 * (abs(D).T @ np.abs(r.astype(np.float64))) + 1e-30)
    specs = [SMALL, TINY, draw_batch_instance(106)]
    doses = [Dose.from_geometry(ctx, s) for s in specs]
    plans = [_plan(ctx, dz, penalty_table(s)) for dz, s in zip(doses, specs)]
    lams = [_lambda0(p, dz, s.seed) for p, dz, s in zip(plans, doses, specs)]
    xs = [to_dev(np.full(dz.nb, ST.x0, np.float32)) for dz in doses]
    ta, tf = Plan.autotune_batch(plans, xs, eps=ST.eps, alpha=ST.alpha, lambda0s=lams, tune_iters=20)
    banner(f"autotune chose {ta} adjoint and {tf} forward workgroups per plan")
    assert (ta, tf) in ((32, 16), (128, 32), (128, 128), (512, 64), (512, 256), (2048, 512))
    for dz in doses:   # each matrix carries its own partition from the chosen per-plan targets
        a = min(32768, max(1024, -(-dz.nnz // ta)))
        b = min(4, max(1, (dz.nnz // 512 + 1) // (8 * tf)))   # 8-wave forward workgroups
        assert dz.partition() == (a, b), (dz.nnz, dz.partition(), (a, b))
    # the start points were not modified by the search
    assert all(np.all(to_host(x0) == ST.x0) for x0 in xs)
    _solo_then_batch(plans, doses, lams, delta=ST.delta, max_iter=2000)


def test_warm_start_batch_bit_identical_to_solo(ctx):
    from paper_0908_4421_amd.imrt import Dose
    specs = [SMALL, TINY, draw_batch_instance(107)]
    doses = [Dose.from_geometry(ctx, s) for s in specs]
    plans = [_plan(ctx, d, penalty_table(s)) for d, s in zip(doses, specs)]
    lams = [_lambda0(p, d, s.seed) for p, d, s in zip(plans, doses, specs)]
    solo, _ = _solo_then_batch(plans, doses, lams, delta=ST.delta, max_iter=1500, warm_start=True)
    banner(f"warm start: iterations {[r.iterations for r, _, _ in solo]}")


def test_full_batch_workload_bit_identical_to_solo(ctx):
    """The benchmark's batched re-plan workload at full size (32 instances,
    seeds 100-131, 40 M nonzeros) with the partition the launch-shape search
    picks: every plan bit-identical to its solo solve on that partition."""
    from paper_0908_4421_amd.imrt import Dose, Plan
    from workloads import batch_instances
    specs = batch_instances(100, 32)
    doses = [Dose.from_geometry(ctx, s) for s in specs]
    banner(f"full batch: {sum(d.nnz for d in doses)} nonzeros")
    plans = [_plan(ctx, d, penalty_table(s)) for d, s in zip(doses, specs)]
    lams = [_lambda0(p, d, s.seed) for p, d, s in zip(plans, doses, specs)]
    xs = [to_dev(np.full(d.nb, ST.x0, np.float32)) for d in doses]
    part = Plan.autotune_batch(plans, xs, eps=ST.eps, alpha=ST.alpha, lambda0s=lams, delta=ST.delta, tune_iters=20)
    banner(f"full batch partition {part}")
    solo, _ = _solo_then_batch(plans, doses, lams, delta=ST.delta, max_iter=ST.max_iter)
    assert all(r.status == 0 for r, _, _ in solo)


def _oracle_runs(problems, delta, max_iter):
    """For each (D, penalties, lambda0): the oracle's stop index under the
    stopping rule and its trajectory continued 40 iterations past it."""
    from oracle import solver
    out = []
    for D, pen, lam in problems:
        x1 = np.full(D.shape[1], ST.x0)
        stop = solver.solve(D, pen, x1, eps=ST.eps, alpha=ST.alpha, lambda0=lam, delta=delta,
                            max_iter=max_iter, keep_trace=False)
        ext = solver.solve(D, pen, x1, eps=ST.eps, alpha=ST.alpha, lambda0=lam,
                           max_iter=stop.iterations + 40, fixed_iters=True)
        out.append((stop.iterations, ext.G_initial, [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in ext.trace]))
    return out


def test_batch_against_oracle(ctx):
    """A batch of the tiny and small phantoms, a re-plan of the small one on
    the same dose matrix, and two drawn re-plan geometries, solved together to
    the stopping rule: each plan's trajectory against the FP64 oracle's (same
    steps and backtracks, G within 1e-6 at every index, final G at the GPU's
    stop index)."""
    from oracle import model, phantom, solver
    from paper_0908_4421_amd.imrt import Dose, Plan
    from gpu_util import check_trajectory
    specs = [TINY, SMALL, SMALL, draw_batch_instance(105), draw_batch_instance(113)]
    tables = [penalty_table(s) for s in specs]
    tables[2] = tables[2].copy()
    tables[2][1, :2] = 68.0     # the re-plan: new target thresholds, new organ limits
    tables[2][2:, 1] *= 0.95
    Ds = {}
    problems, doses, plans = [], [], []
    for i, (sp, t) in enumerate(zip(specs, tables)):
        if sp.name not in Ds:
            Ds[sp.name] = (phantom.build_dose_matrix(sp), Dose.from_geometry(ctx, sp))
        D, lib = Ds[sp.name]
        pen = model.VoxelPenalties.from_structures(D.struct_id, t)
        lam, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, sp.seed + i))
        problems.append((D.csr, pen, lam))
        doses.append(lib)
        plans.append(_plan(ctx, lib, t))
    assert doses[1] is doses[2]
    banner("batch against the oracle: " + ", ".join(s.name for s in specs))
    refs = _oracle_runs(problems, ST.delta, 3000)
    xs = [to_dev(np.full(d.nb, ST.x0, np.float32)) for d in doses]
    out = Plan.solve_batch(plans, xs, eps=ST.eps, alpha=ST.alpha, lambda0s=[p[2] for p in problems],
                           delta=ST.delta, max_iter=3000, trace=True)
    for sp, (res, tr), (stop, G0, ref) in zip(specs, out, refs):
        worst, K, Ko = check_trajectory(tr, res, ref, G0, stop, delta=ST.delta)
        banner(f"{sp.name}: {K} iterations (oracle {Ko}), worst G error {worst:.2e}")
