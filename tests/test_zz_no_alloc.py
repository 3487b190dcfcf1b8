"""The allocation-free gradient (imrt_gradient_noalloc) against imrt_gradient:
the same kernels and partition on the library's static per-device scratch,
so g and G must equal the plan-buffer entry point's bit for bit -- on two
calls in a row (the paper-scale plan, then the smaller tiny plan, which
reuses the scratch the first call left behind) and again on the first plan;
plans beyond the scratch are refused with IMRT_EINVAL."""
import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from workloads import PAPER_SCALE, TINY, penalty_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


def _plan(ctx, spec):
    from paper_0908_4421_amd.imrt import Dose, Plan
    dose = Dose.from_geometry(ctx, spec)
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(spec))
    return dose, plan


def _check(plan, nb, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = to_dev(rng.uniform(0.0, 3.0, nb).astype(np.float32))
    g_ref, G_ref = plan.gradient(x)
    g = torch.full((nb,), float("nan"), dtype=torch.float32, device="cuda")
    G = plan.gradient_noalloc(x, g)
    assert G == G_ref, (G, G_ref)
    assert np.array_equal(to_host(g), to_host(g_ref))
    # enqueue-only form (no copy back), then the same result
    g.fill_(float("nan"))
    assert plan.gradient_noalloc(x, g, want_G=False) is None
    assert np.array_equal(to_host(g), to_host(g_ref))
    return G


def test_noalloc_gradient_equals_gradient(ctx):
    big_dose, big = _plan(ctx, PAPER_SCALE)
    small_dose, small = _plan(ctx, TINY)
    banner(f"noalloc gradient: {big_dose.nv} voxels, then {small_dose.nv}")
    G1 = _check(big, big_dose.nb, 0)
    G2 = _check(small, small_dose.nb, 1)      # second call, smaller input
    G3 = _check(big, big_dose.nb, 2)
    banner(f"G {G1:.6g}, {G2:.6g}, {G3:.6g}")


def test_noalloc_refuses_plans_beyond_the_scratch(ctx):
    from paper_0908_4421_amd import imrt
    from paper_0908_4421_amd.imrt import Dose, Plan
    import torch
    nv, nb = 5_000_000, 4          # residual alone needs 20 MB > 16 MiB
    row_ptr = np.zeros(nv + 1, np.int32)
    row_ptr[1:] = np.minimum(np.arange(1, nv + 1), 8)   # 8 nonzeros in the first 8 rows
    col_idx = (np.arange(8) % nb).astype(np.int32)
    val = np.full(8, 0.5, np.float32)
    dose = Dose.from_csr(ctx, nv, nb, row_ptr, col_idx, val)
    plan = Plan(ctx, dose)
    plan.set_structures(np.zeros(nv, np.uint8), 1)
    plan.set_penalties(np.array([[1.0, 1.0, 1.0, 1.0]]))
    x = torch.ones(nb, dtype=torch.float32, device="cuda")
    g = torch.zeros(nb, dtype=torch.float32, device="cuda")
    with pytest.raises(imrt.ImrtError) as e:
        plan.gradient_noalloc(x, g)
    assert e.value.code == imrt.IMRT_EINVAL
    assert "scratch" in str(e.value)
    g_ref, G_ref = plan.gradient(x)    # the plan-buffer entry point still serves it
    assert np.isfinite(G_ref)
