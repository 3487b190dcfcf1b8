"""Re-plan server (imrt_server_*) on the GPU: requests submitted together
(new patients and re-plans of resident patients with new thresholds) each
end exactly as the same plan solved alone; a small HBM budget serialises
admissions and evicts unused matrices; a failed request fails alone."""
import time
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from workloads import SMALL, TINY, draw_batch_instance, penalty_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


def _replan_table(spec, rng):
    from workloads import replan_penalty_table
    return replan_penalty_table(spec, rng)


def _alone(ctx, dose, table, lam, max_iter=3000, fixed=False):
    from paper_0908_4421_amd.imrt import Plan
    p = Plan(ctx, dose)
    p.set_structures(None, len(table))
    p.set_penalties(table)
    x = to_dev(np.ones(dose.nb, np.float32))
    res, _ = p.solve(x, eps=1e-4, alpha=2.0, lambda0=lam, delta=1e-5, max_iter=max_iter, fixed_iters=fixed)
    return res, to_host(x)


def test_mix_equals_alone(ctx):
    from paper_0908_4421_amd.imrt import Dose, Server
    rng = np.random.default_rng(3)
    specs = [SMALL, TINY, draw_batch_instance(1000), draw_batch_instance(1001), draw_batch_instance(1002)]
    doses = [Dose.from_geometry(ctx, sp) for sp in specs]
    part = (ctx.get_option("serve_adjoint_workgroups"), ctx.get_option("serve_forward_workgroups"))
    for d in doses:             # the server's matrices carry this partition
        d.repartition_targets(*part)
    srv = Server(ctx, budget_bytes=8 << 30, max_live=16)
    reqs = []   # (patient, spec or None, table)
    for i, sp in enumerate(specs):
        reqs.append((i, sp, penalty_table(sp)))
    reqs.append((0, SMALL, _replan_table(SMALL, rng)))      # re-plans of resident patients
    reqs.append((2, specs[2], _replan_table(specs[2], rng)))
    reqs.append((1, None, _replan_table(TINY, rng)))        # resident only: no geometry needed
    banner(f"serve mix of {len(reqs)} requests")
    tickets = [srv.submit(p, sp, t, max_iter=3000) for p, sp, t in reqs]
    got = []
    for (pat, sp, t), tk in zip(reqs, tickets):
        got.append(srv.wait(tk, doses[pat].nb))
        banner(f"ticket {tk} done: {got[-1][0].iterations} iterations")
    st = srv.stats()
    srv.close()
    assert st["served"] == len(reqs) and st["resident_matrices"] == len(specs)
    for (pat, sp, t), (res, times, x) in zip(reqs, got):
        ref, xr = _alone(ctx, doses[pat], t, times.lambda0)
        assert (res.iterations, res.status) == (ref.iterations, ref.status)
        assert res.G_final == ref.G_final and res.G_initial == ref.G_initial
        assert np.array_equal(x, xr)
        assert 0.0 <= times.queue_ms <= times.plan_ms
        assert (times.nv, times.nb, times.nnz) == (doses[pat].nv, doses[pat].nb, doses[pat].nnz)
    banner("plan ms " + ", ".join(f"{times.plan_ms:.1f}" for _, times, _ in got))


def test_small_budget_evicts_and_serialises(ctx):
    from paper_0908_4421_amd.imrt import Server
    specs = [draw_batch_instance(s) for s in (1000, 1001, 1002, 1005)] + [SMALL, draw_batch_instance(1000)]
    budget = 40 << 20
    srv = Server(ctx, budget_bytes=budget, max_live=4)
    patients = [10, 11, 12, 13, 14, 10]   # the last re-plans the first patient (evicted by then, or not)
    tickets = [srv.submit(pt, sp, penalty_table(sp), max_iter=2000) for pt, sp in zip(patients, specs)]
    out = []
    for tk in tickets:
        out.append(srv.wait(tk))
        banner(f"ticket {tk} done")
    st = srv.stats()
    srv.close()
    banner(f"budget {budget >> 20} MiB: peak {st['peak_bytes'] / 2**20:.1f} MiB, resident {st['resident_matrices']}")
    assert st["served"] == len(specs)
    assert all(r.status == 0 for r, _, _ in out)
    assert st["peak_bytes"] <= budget


def test_failed_request_fails_alone(ctx):
    """A request that cannot be served fails alone; an x_out of the wrong
    length is refused without losing the result; a ticket is handed out once."""
    from paper_0908_4421_amd import imrt
    from paper_0908_4421_amd.imrt import Dose, Server
    nb_tiny = Dose.from_geometry(ctx, TINY).nb
    srv = Server(ctx, budget_bytes=1 << 30, max_live=4)
    bad = srv.submit(99, None, penalty_table(TINY))          # not resident, no geometry
    good = srv.submit(1, TINY, penalty_table(TINY), max_iter=50, fixed_iters=True)
    with pytest.raises(imrt.ImrtError) as e:
        srv.wait(bad)
    assert e.value.code == imrt.IMRT_EINVAL
    # an x_out of the wrong length is refused and leaves the result pending
    with pytest.raises(imrt.ImrtError) as e:
        srv.wait(good, nb_tiny + 1)
    assert e.value.code == imrt.IMRT_EINVAL
    res, times, x = srv.wait(good, nb_tiny)
    assert res.iterations == 50 and x.shape == (nb_tiny,) and np.all(np.isfinite(x))
    for tk in (good, 0, 999):     # waited on already, never issued
        with pytest.raises(imrt.ImrtError) as e:
            srv.wait(tk)
        assert e.value.code == imrt.IMRT_EINVAL
    srv.close()


def test_storage_change_waits_for_the_live_mix(ctx):
    """Requests in float32, bfloat16, float32 submitted together: each waits
    until the solves of the other storage ahead of it are done (arrival order
    is kept), and every plan equals the same plan solved alone."""
    from paper_0908_4421_amd.imrt import Dose, Server
    part = (ctx.get_option("serve_adjoint_workgroups"), ctx.get_option("serve_forward_workgroups"))
    reqs = [(20, TINY, "f32"), (21, SMALL, "bf16"), (22, draw_batch_instance(1003), "f32")]
    srv = Server(ctx, budget_bytes=4 << 30, max_live=8)
    tables = [penalty_table(sp) for _, sp, _ in reqs]
    tickets, sub_s = [], []
    for (pt, sp, st), tab in zip(reqs, tables):
        sub_s.append(time.perf_counter())
        tickets.append(srv.submit(pt, sp, tab, storage=st, max_iter=400, fixed_iters=True))
    got = []
    for tk in tickets:
        got.append(srv.wait(tk, 0))
        banner(f"ticket {tk} done")
    srv.close()
    for (pt, sp, st), (res, times, _) in zip(reqs, got):
        d = Dose.from_geometry(ctx, sp, storage=st)
        d.repartition_targets(*part)
        ref, _ = _alone(ctx, d, penalty_table(sp), times.lambda0, max_iter=400, fixed=True)
        assert res.iterations == ref.iterations == 400
        assert res.G_final == ref.G_final
    # admitted one after the other: request i+1 waits from its submission
    # until request i is done, so its queue time is at least request i's
    # time to plan less the time between the two submissions (measured here,
    # plus 1 ms for the server's own clock reads)
    for i in (0, 1):
        gap = 1e3 * (sub_s[i + 1] - sub_s[i]) + 1.0
        assert got[i + 1][1].queue_ms >= got[i][1].plan_ms - gap


def test_served_workload_mix_equals_alone(ctx):
    """24 requests of the served re-plan workload (bfloat16 matrices, 30 %
    re-plans of resident patients with new thresholds) submitted at once:
    every plan equals the same plan solved alone."""
    from paper_0908_4421_amd.imrt import Dose, Server
    from workloads import served_requests
    reqs = served_requests(20.0, 24, seed=200)
    part = (ctx.get_option("serve_adjoint_workgroups"), ctx.get_option("serve_forward_workgroups"))
    srv = Server(ctx, budget_bytes=16 << 30, max_live=64)
    tickets = [srv.submit(r.patient, r.spec, r.table, storage="bf16", max_iter=20000) for r in reqs]
    got = [srv.wait(tk, 0) for tk in tickets]
    st = srv.stats()
    srv.close()
    banner(f"served mix: {sum(r.replan for r in reqs)} re-plans, {st['resident_matrices']} matrices, "
           f"iterations {[g[0].iterations for g in got]}")
    doses = {}
    for r, (res, times, _) in zip(reqs, got):
        if r.patient not in doses:
            d = Dose.from_geometry(ctx, r.spec, storage="bf16")
            d.repartition_targets(*part)
            doses[r.patient] = d
        ref, _ = _alone(ctx, doses[r.patient], r.table, times.lambda0, max_iter=20000)
        assert (res.iterations, res.status) == (ref.iterations, ref.status)
        assert res.G_final == ref.G_final


@pytest.mark.parametrize("storage,share", [("f32", 0), ("bf16", 1)], ids=["f32", "bf16_shared_adjoint"])
def test_served_against_oracle(storage, share):
    """Requests served together (new patients and a re-plan of a resident
    one, continuous batching; in bfloat16 with the shared-matrix adjoint, so
    the re-plan and its patient's first plan share adjoint passes while both
    are live) against the FP64 oracle: every served plan's
    trajectory (traced by the server) has the oracle's steps and backtracks,
    G within 1e-6 relative plus the float32 dose-rounding bound at every index
    and at the served stop index (a plan that runs to the 3000-iteration cap
    reaches G near 1e-4 of its start, where that bound decides); with
    bfloat16 storage the oracle runs on the stored matrix D~."""
    from oracle import model, phantom, quantize, solver
    from paper_0908_4421_amd.imrt import Server
    from gpu_util import check_trajectory, dose_rounding_slack
    rng = np.random.default_rng(11)
    specs = [TINY, SMALL, draw_batch_instance(105)]
    reqs = [(0, TINY, penalty_table(TINY)), (1, SMALL, penalty_table(SMALL)),
            (2, specs[2], penalty_table(specs[2])), (1, None, _replan_table(SMALL, rng))]
    mats = {}
    for pat, sp in enumerate(specs):
        D = phantom.build_dose_matrix(sp)
        Dv = D.csr if storage == "f32" else quantize.store(D.csr, storage).Dq
        mats[pat] = (D, Dv)
    refs, lams = [], []
    for pat, sp, t in reqs:
        D, Dv = mats[pat]
        pen = model.VoxelPenalties.from_structures(D.struct_id, t)
        lam, _ = solver.lambda0_from_power_iteration(Dv, pen, np.ones(D.nb))
        x1 = np.ones(D.nb)
        stop = solver.solve(Dv, pen, x1, eps=1e-4, alpha=2.0, lambda0=lam, delta=1e-5, max_iter=3000,
                            keep_trace=False)
        ext = solver.solve(Dv, pen, x1, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=stop.iterations + 40,
                           fixed_iters=True)
        refs.append((stop.iterations, ext.G_initial,
                     [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in ext.trace],
                     dose_rounding_slack(pen)))
        lams.append(lam)
    from paper_0908_4421_amd.imrt import Context
    srv = Server(Context(0, serve_shared_adjoint=share), budget_bytes=8 << 30, max_live=16)
    banner(f"served against the oracle ({storage}, shared adjoint {share}): {len(reqs)} requests")
    tickets = [srv.submit(p, sp, t, storage=storage, lambda0=lam, max_iter=3000, trace=True)
               for (p, sp, t), lam in zip(reqs, lams)]
    for (pat, sp, t), tk, (stop, G0, ref, slack) in zip(reqs, tickets, refs):
        res, times, _ = srv.wait(tk)
        tr = srv.trace_of(tk, res.iterations)
        worst, K, Ko = check_trajectory(tr, res, ref, G0, stop, delta=1e-5, slack=slack)
        banner(f"ticket {tk}: {K} iterations (oracle {Ko}), worst G error {worst:.2e}")
    st = srv.stats()
    assert (st["adjoint_groups_shared"] > 0) == bool(share)
    srv.close()


@pytest.mark.parametrize("adj_wgs", [0, 2], ids=["default_targets", "two_adjoint_workgroups"])
def test_shared_matrix_adjoint_equals_alone(adj_wgs):
    """Four re-plans of one patient, two of another and a single new patient,
    submitted together: the live solves on one resident matrix share each
    adjoint pass (groups of four and two), and every plan equals the same
    plan solved alone and served without sharing, bit for bit.  With two
    adjoint workgroups per plan each workgroup walks 80 to 240 columns, so
    the shared pass reloads its column chunk (64 at a time) mid-range."""
    from paper_0908_4421_amd.imrt import Context, Dose, Server
    from workloads import replan_penalty_table
    rng = np.random.default_rng(21)
    reqs = [(30, SMALL, penalty_table(SMALL))] + [(30, SMALL, replan_penalty_table(SMALL, rng)) for _ in range(3)]
    reqs += [(31, TINY, penalty_table(TINY)), (31, TINY, replan_penalty_table(TINY, rng))]
    reqs += [(32, draw_batch_instance(1004), penalty_table(draw_batch_instance(1004)))]
    opts = {"serve_adjoint_workgroups": adj_wgs} if adj_wgs else {}
    ctx = Context(0, **opts)
    part = (ctx.get_option("serve_adjoint_workgroups"), ctx.get_option("serve_forward_workgroups"))
    doses = {}
    for pat, sp, _ in reqs:
        if pat not in doses:
            d = Dose.from_geometry(ctx, sp)
            d.repartition_targets(*part)
            doses[pat] = d
    out = {}
    for share in (1, 0):
        c = Context(0, serve_shared_adjoint=share, **opts)
        srv = Server(c, budget_bytes=8 << 30, max_live=16)
        tickets = [srv.submit(p, sp, t, max_iter=1500) for p, sp, t in reqs]
        out[share] = [srv.wait(tk, doses[p].nb) for tk, (p, _, _) in zip(tickets, reqs)]
        st = srv.stats()
        srv.close()
        banner(f"shared adjoint {share}: {st['adjoint_groups_shared']} of {st['adjoint_groups']} adjoint groups "
               f"shared, iterations {[g[0].iterations for g in out[share]]}")
        if share:
            assert st["adjoint_groups_shared"] > 0
        else:
            assert st["adjoint_groups_shared"] == 0
    for (pat, sp, t), (res, times, x), (res0, _, x0) in zip(reqs, out[1], out[0]):
        assert (res.iterations, res.status, res.G_final) == (res0.iterations, res0.status, res0.G_final)
        assert np.array_equal(x, x0)
        ref, xr = _alone(ctx, doses[pat], t, times.lambda0, max_iter=1500)
        assert (res.iterations, res.status) == (ref.iterations, ref.status)
        assert res.G_final == ref.G_final and res.G_initial == ref.G_initial
        assert np.array_equal(x, xr)
