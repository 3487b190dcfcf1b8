"""GPU objective, gradient, projection and step-size estimate against the
FP64 oracle at the same float32 inputs."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import banner, csr_of, rel_normwise, to_dev, to_host
from oracle import model, phantom, solver
from workloads import TINY, penalty_table, power_start_vector, random_csr, random_penalties

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[1, 0], ids=["voxel_tiles", "grid_order"])
def ctx(request):
    """Built phantoms with rows in voxel tiles (default) or grid order: the
    structure ids, voxel targets and dose outputs cross the API in grid order."""
    from paper_0908_4421_amd.imrt import Context
    return Context(0, voxel_tiles=request.param)


@pytest.fixture(scope="module")
def tiny(ctx):
    from paper_0908_4421_amd.imrt import Dose, Plan
    D = phantom.build_dose_matrix(TINY)
    lib = Dose.from_geometry(ctx, TINY)
    plan = Plan(ctx, lib)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(TINY))
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    return D, lib, plan, pen


def test_objective_dose_gradient_tiny(tiny):
    banner("objective/gradient tiny")
    D, lib, plan, pen = tiny
    rng = np.random.default_rng(0)
    for scale in (1.0, 10.0, 40.0):       # under-dosed, mixed, over-dosed regimes
        x = (rng.uniform(0.0, 1.0, D.nb) * scale).astype(np.float32)
        xd = to_dev(x)
        import torch
        dose = torch.empty(D.nv, dtype=torch.float32, device="cuda")
        G = plan.objective(xd, dose)
        x64 = x.astype(np.float64)
        z = model.dose(D.csr, x64)
        G_ref = model.objective_from_dose(z, pen)
        assert abs(G - G_ref) <= 1e-6 * G_ref
        d = to_host(dose)
        assert np.max(np.abs(d - z) / np.maximum(np.abs(z), 1e-30)) <= 1e-5
        g, G2 = plan.gradient(xd)
        assert G2 == G
        g_ref = model.gradient(D.csr, x64, pen)
        assert rel_normwise(to_host(g), g_ref) <= 1e-5


def test_voxel_targets_mode(tiny):
    """Per-voxel thresholds (the paper's T_j) replace the structure thresholds."""
    D, lib, plan, pen = tiny
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 20.0, D.nb).astype(np.float32)
    Tu = rng.uniform(10, 60, D.nv).astype(np.float32)
    To = (Tu + rng.uniform(0, 10, D.nv)).astype(np.float32)
    plan.set_voxel_targets(Tu, To)
    try:
        G = plan.objective(to_dev(x))
        g, _ = plan.gradient(to_dev(x))
    finally:
        plan.set_voxel_targets(None, None)
    pv = pen.with_targets(Tu.astype(np.float64), To.astype(np.float64))
    G_ref = model.objective(D.csr, x.astype(np.float64), pv)
    assert abs(G - G_ref) <= 1e-6 * G_ref
    assert rel_normwise(to_host(g), model.gradient(D.csr, x.astype(np.float64), pv)) <= 1e-5
    # and the structure thresholds are back
    G0 = plan.objective(to_dev(x))
    assert abs(G0 - model.objective(D.csr, x.astype(np.float64), pen)) <= 1e-6 * G0


@pytest.mark.parametrize("seed", [0, 1])
def test_random_structures_and_penalties(ctx, seed):
    from paper_0908_4421_amd.imrt import Dose, Plan
    A = random_csr(4000, 150, 10.0, 20 + seed, empty_frac=0.4, nstruct=6)
    D = csr_of(A)
    pens = random_penalties(6, seed, scale=3.0)
    table = np.array([[p.T_under, p.T_over, p.w_under, p.w_over] for p in pens])
    lib = Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)
    plan = Plan(ctx, lib)
    plan.set_structures(A.struct_id, 6)
    plan.set_penalties(table)
    pen = model.VoxelPenalties.from_structures(A.struct_id, table)
    x = np.random.default_rng(seed).uniform(0, 0.6, A.nb).astype(np.float32)
    G = plan.objective(to_dev(x))
    G_ref = model.objective(D, x.astype(np.float64), pen)
    assert abs(G - G_ref) <= 1e-6 * G_ref
    g, _ = plan.gradient(to_dev(x))
    assert rel_normwise(to_host(g), model.gradient(D, x.astype(np.float64), pen)) <= 1e-5


def test_projection_exact(tiny):
    D, lib, plan, pen = tiny
    rng = np.random.default_rng(2)
    x = np.abs(rng.standard_normal(D.nb)).astype(np.float32)
    g = rng.standard_normal(D.nb).astype(np.float32)
    for lam in (0.5, 2.0 ** -7, 3.0):
        out, s = plan.project(to_dev(x), to_dev(g), lam)
        want = model.project(x.astype(np.float64) - lam * g.astype(np.float64)).astype(np.float32)
        got = to_host(out)
        assert np.array_equal(got, want)
        s_ref = float(np.sum((want.astype(np.float64) - x.astype(np.float64)) ** 2))
        assert abs(s - s_ref) <= 1e-12 * s_ref


def test_lambda0_estimate(tiny):
    D, lib, plan, pen = tiny
    v0 = power_start_vector(D.nb, TINY.seed)
    lam, sig = plan.lambda0(to_dev(v0.astype(np.float32)), 50)
    lam_ref, sig_ref = solver.lambda0_from_power_iteration(D.csr, pen, v0.astype(np.float32).astype(np.float64), 50)
    assert abs(sig - sig_ref) <= 1e-5 * sig_ref
    assert lam == lam_ref


def test_not_ready_errors(ctx):
    from paper_0908_4421_amd import imrt
    from paper_0908_4421_amd.imrt import Dose, Plan
    A = random_csr(50, 5, 3.0, 3)
    lib = Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)
    plan = Plan(ctx, lib)
    x = to_dev(np.ones(5, np.float32))
    with pytest.raises(imrt.ImrtError) as e:
        plan.objective(x)
    assert e.value.code == imrt.IMRT_ENOTREADY
    with pytest.raises(imrt.ImrtError) as e:
        plan.set_structures(np.full(50, 3, np.uint8), 3)          # id 3 >= nstruct
    assert e.value.code == imrt.IMRT_EINVAL
    plan.set_structures(np.zeros(50, np.uint8), 1)
    with pytest.raises(imrt.ImrtError) as e:
        plan.set_penalties([(1.0, 2.0, -1.0, 1.0)])               # negative weight
    assert e.value.code == imrt.IMRT_EINVAL
