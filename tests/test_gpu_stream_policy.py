"""Cache policy of the solve passes' matrix streams (context option
stream_nt: 0 never non-temporal, 1 always, 2 when the matrices exceed the
last-level cache).  The policy changes how the loads use the caches, not
what they read, so a solve or a batch with non-temporal streams must be bit
for bit the same as with the default policy: traces, final states and x."""
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from workloads import SMALL, TINY, PAPER_SCALE_SETTINGS, draw_batch_instance, penalty_table, power_start_vector

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


def test_option_range(ctx):
    from paper_0908_4421_amd import imrt
    assert ctx.get_option("stream_nt") == 2
    for bad in (-1, 3):
        with pytest.raises(imrt.ImrtError) as e:
            ctx.set_option("stream_nt", bad)
        assert e.value.code == imrt.IMRT_EINVAL
    assert ctx.get_option("stream_nt") == 2


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("trials", [1, 2])
def test_non_temporal_solve_bit_identical(ctx, storage, trials):
    from paper_0908_4421_amd.imrt import Dose
    dose = Dose.from_geometry(ctx, SMALL, storage=storage)
    plan = _plan(ctx, dose, penalty_table(SMALL))
    lam = plan.lambda0(to_dev(power_start_vector(dose.nb, SMALL.seed).astype(np.float32)), ST.power_iters)[0]
    out = {}
    try:
        for policy in (0, 1):
            ctx.set_option("stream_nt", policy)
            banner(f"small phantom, {storage}, {trials} trial(s) per pass, stream_nt {policy}")
            x = to_dev(np.full(dose.nb, ST.x0, np.float32))
            res, tr = plan.solve(x, eps=ST.eps, alpha=ST.alpha, lambda0=lam, delta=ST.delta, max_iter=3000,
                                 trace=True, trials_per_pass=trials)
            out[policy] = (res, tr, to_host(x))
    finally:
        ctx.set_option("stream_nt", 2)
    (r0, t0, x0), (r1, t1, x1) = out[0], out[1]
    assert r0.status == 0 and r0.iterations > 100
    assert t1 == t0
    assert (r1.iterations, r1.status, r1.forward_passes, r1.adjoint_passes) == \
        (r0.iterations, r0.status, r0.forward_passes, r0.adjoint_passes)
    assert r1.G_final == r0.G_final and r1.G_initial == r0.G_initial
    assert np.array_equal(x1, x0)


def test_non_temporal_batch_bit_identical(ctx):
    from paper_0908_4421_amd.imrt import Dose, Plan
    specs = [TINY, SMALL] + [draw_batch_instance(s) for s in (100, 101)]
    doses = [Dose.from_geometry(ctx, s) for s in specs]
    plans = [_plan(ctx, d, penalty_table(s)) for d, s in zip(doses, specs)]
    lams = [p.lambda0(to_dev(power_start_vector(d.nb, s.seed).astype(np.float32)), ST.power_iters)[0]
            for p, d, s in zip(plans, doses, specs)]
    out = {}
    try:
        for policy in (0, 1):
            ctx.set_option("stream_nt", policy)
            banner(f"batch of {len(specs)}, stream_nt {policy}")
            xs = [to_dev(np.full(d.nb, ST.x0, np.float32)) for d in doses]
            res = Plan.solve_batch(plans, xs, eps=ST.eps, alpha=ST.alpha, lambda0s=lams, trace=True,
                                   delta=ST.delta, max_iter=3000)
            out[policy] = [(r, t, to_host(x)) for (r, t), x in zip(res, xs)]
    finally:
        ctx.set_option("stream_nt", 2)
    for (r0, t0, x0), (r1, t1, x1) in zip(out[0], out[1]):
        assert r0.status == 0
        assert t1 == t0
        assert (r1.iterations, r1.forward_passes, r1.adjoint_passes) == \
            (r0.iterations, r0.forward_passes, r0.adjoint_passes)
        assert r1.G_final == r0.G_final
        assert np.array_equal(x1, x0)
