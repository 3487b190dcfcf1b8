"""Wide beamlet kernels, as in the paper's scenarios (Table 1: about 300
nonzeros per voxel): the small wide phantom's matrix bit-exact against the
oracle's and its solve trajectory against the oracle's, with 16-bit and
32-bit forward column indices (rows of up to 656 nonzeros fit one 764-entry
block, but stream over several 508-entry blocks); the scenario-3-shaped
phantom's sizes and sampled columns against the oracle."""
import numpy as np
import pytest

from gpu_util import banner, f32_ulp_diff, to_dev, to_host
from oracle import model, phantom, solver
from workloads import SCENARIO3_SHAPE, WIDE, penalty_table, power_start_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[1, 0], ids=["col16", "col32"])
def ctx(request):
    from paper_0908_4421_amd.imrt import Context
    return Context(0, fwd_col16=request.param)


@pytest.fixture(scope="module")
def wide():
    D = phantom.build_dose_matrix(WIDE)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(WIDE))
    lam0, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, WIDE.seed))
    ref = solver.solve(D.csr, pen, np.ones(D.nb), eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=60,
                       fixed_iters=True)
    return D, pen, lam0, ref


def test_wide_phantom_matrix_and_solve(ctx, wide):
    from paper_0908_4421_amd.imrt import Dose, Plan
    import torch
    D, pen, lam0, ref = wide
    banner(f"wide phantom nnz {D.nnz}, longest row {np.diff(D.csr.indptr).max()}")
    lib = Dose.from_geometry(ctx, WIDE)
    assert (lib.nv, lib.nb, lib.nnz) == (D.nv, D.nb, D.nnz)
    ex = lib.export(structures=True)
    assert np.array_equal(ex["row_ptr"], D.csr.indptr) and np.array_equal(ex["col_idx"], D.csr.indices)
    assert np.array_equal(ex["row_idx"], D.csc.indices) and np.array_equal(ex["struct_id"], D.struct_id)
    assert f32_ulp_diff(ex["val"], D.csr.data) <= 1
    plan = Plan(ctx, lib)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(WIDE))
    x = to_dev(np.ones(D.nb, np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=60, fixed_iters=True, trace=True)
    assert abs(res.G_initial - ref.G_initial) <= 1e-6 * ref.G_initial
    assert len(tr) == len(ref.trace)
    for (k, m, lam, s, G), e in zip(tr, ref.trace):
        assert k == e.k and m == e.backtracks and lam == e.lam
        assert abs(G - e.G) <= 1e-6 * e.G, (k, G, e.G)
    xg = to_host(x).astype(np.float64)
    d = torch.empty(D.nv, dtype=torch.float32, device="cuda")
    assert plan.objective(x, d) == res.G_final
    z = model.dose(D.csr, xg)
    assert np.max(np.abs(to_host(d) - z) / np.maximum(z, 1e-30)) <= 1e-5


def test_scenario3_shape_sizes_and_sampled_columns():
    from paper_0908_4421_amd.imrt import Context, Dose
    ctx = Context(0)
    spec = SCENARIO3_SHAPE
    bls = phantom.beamlets(spec)
    banner(f"scenario-3 shape: {len(bls)} beamlets")
    lib = Dose.from_geometry(ctx, spec)
    assert (lib.nv, lib.nb) == (spec.nx * spec.ny * spec.nz, len(bls))
    banner(f"scenario-3 shape: nnz {lib.nnz}")
    assert 3.5e7 < lib.nnz < 5e7
    ex = lib.export()
    which = list(np.random.default_rng(8).choice(len(bls), 12, replace=False))
    _, cols = phantom.build_columns(spec, which)
    for i, (rows, vals) in zip(which, cols):
        a, b = ex["col_ptr"][i], ex["col_ptr"][i + 1]
        assert np.array_equal(ex["row_idx"][a:b], rows)
        assert f32_ulp_diff(ex["cval"][a:b], vals) <= 1
