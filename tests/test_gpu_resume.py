"""Checkpoint and resume of a GPU solve (Section 2.2's iteration continued
from a stored iterate): a solve interrupted after K iterations and resumed
from x_K with G(x_{K-1}) and the step accepted last reproduces the
uninterrupted trajectory bit for bit, with the paper's cold line search and
with the warm-started variant, one and two trial steps per pass, in float32
and bfloat16 storage; a resume at the point where the uninterrupted solve
stopped stops at once; argument errors."""
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from workloads import SMALL, TINY, penalty_table, power_start_vector

pytestmark = pytest.mark.gpu

EPS, ALPHA, DELTA, CAP = 1e-4, 2.0, 1e-5, 4000


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


def _plan(ctx, spec, storage):
    from paper_0908_4421_amd.imrt import Dose, Plan
    dose = Dose.from_geometry(ctx, spec, storage=storage)
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(spec))
    lam0, _ = plan.lambda0(to_dev(power_start_vector(dose.nb, spec.seed).astype(np.float32)), 50)
    return dose, plan, lam0


def _resume_point(res, tr, K):
    """(k0, G_prev, lambda_prev) after iteration K of a traced solve."""
    G_prev = tr[K - 2][4] if K >= 2 else res.G_initial
    return K, G_prev, tr[K - 1][2]


@pytest.mark.parametrize("spec,storage,warm,nt", [(TINY, "f32", False, 1), (TINY, "f32", True, 1),
                                                  (SMALL, "f32", True, 2), (SMALL, "bf16", False, 1)],
                         ids=["tiny_cold", "tiny_warm", "small_warm_2trials", "small_bf16_cold"])
def test_interrupted_and_resumed_equals_uninterrupted(ctx, spec, storage, warm, nt):
    dose, plan, lam0 = _plan(ctx, spec, storage)
    kw = dict(eps=EPS, alpha=ALPHA, lambda0=lam0, warm_start=warm, trials_per_pass=nt, trace=True)
    x = to_dev(np.ones(dose.nb, np.float32))
    full, tfull = plan.solve(x, delta=DELTA, max_iter=CAP, **kw)
    x_full = to_host(x)
    N = full.iterations
    banner(f"{spec.name} {storage} warm={warm} nt={nt}: {N} iterations uninterrupted, status {full.status}")
    assert N > 10
    for K in (1, N // 3, N - 1):
        # the first K iterations (stopping test off, so that the checkpoint is
        # taken wherever it is asked for), then the rest from the checkpoint
        xk = to_dev(np.ones(dose.nb, np.float32))
        r1, t1 = plan.solve(xk, delta=DELTA, max_iter=K, fixed_iters=True, **kw)
        assert r1.iterations == K and t1 == tfull[:K]
        r2, t2 = plan.solve(xk, delta=DELTA, max_iter=CAP - K, resume=_resume_point(r1, t1, K), **kw)
        assert t1 + t2 == tfull, K
        assert (r2.status, r2.iterations, r2.G_final) == (full.status, N - K, full.G_final)
        assert r2.G_initial == tfull[K - 1][4]
        assert np.array_equal(to_host(xk), x_full), K


def test_resume_at_the_stop_stops(ctx):
    """Checkpointed exactly where the uninterrupted solve stopped: with G_prev
    step 5 holds at once (0 iterations, converged, same G and x); a fresh
    start from the same x would iterate on."""
    dose, plan, lam0 = _plan(ctx, TINY, "f32")
    kw = dict(eps=EPS, alpha=ALPHA, lambda0=lam0, trace=True)
    x = to_dev(np.ones(dose.nb, np.float32))
    full, tfull = plan.solve(x, delta=DELTA, max_iter=CAP, **kw)
    assert full.status == 0
    N = full.iterations
    xk = to_dev(np.ones(dose.nb, np.float32))
    r1, t1 = plan.solve(xk, max_iter=N, fixed_iters=True, **kw)
    r2, t2 = plan.solve(xk, delta=DELTA, max_iter=CAP, resume=_resume_point(r1, t1, N), **kw)
    assert (r2.status, r2.iterations, r2.G_final, r2.G_initial) == (0, 0, full.G_final, full.G_final)
    assert t2 == [] and np.array_equal(to_host(xk), to_host(x))
    r3, _ = plan.solve(xk, delta=DELTA, max_iter=CAP, **kw)
    assert r3.iterations >= 1


def test_resume_argument_errors(ctx):
    from paper_0908_4421_amd.imrt import ImrtError, IMRT_EINVAL
    dose, plan, lam0 = _plan(ctx, TINY, "f32")
    x = to_dev(np.ones(dose.nb, np.float32))
    for bad in [(0, 1.0, 1.0), (3, -1.0, 1.0), (3, float("nan"), 1.0), (3, 1.0, 0.0), (3, 1.0, float("inf"))]:
        with pytest.raises(ImrtError) as e:
            plan.solve(x, eps=EPS, alpha=ALPHA, lambda0=lam0, max_iter=5, resume=bad)
        assert e.value.code == IMRT_EINVAL
