"""Unspecified tissue at twice the voxel size (Section 3.1) on the GPU: the
library's own coarse layout against the oracle's.  Small phantoms (an even
grid and an odd one with incomplete blocks, rows in voxel tiles and in API
order): sparsity, structure ids and CSC bit for bit, values within one
float32 ulp, and the 200-iteration trajectory.  Paper scale: the oracle's
stored fingerprint and trajectory (tests/golden/paper_scale_coarse_oracle.json,
written by make_paper_scale_fixture.py --coarse from the oracle alone),
sampled rows and columns computed here, and the final dose over every voxel."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import banner, check_trajectory, f32_ulp_diff, to_dev, to_host
from oracle import model, phantom, solver
from workloads import (PAPER_SCALE_COARSE, PAPER_SCALE_SETTINGS, SMALL_COARSE, TINY_COARSE, penalty_table,
                       power_start_vector, start_point)

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_scale_coarse_oracle.json")


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.fixture(scope="module", params=[1, 0], ids=["voxel_tiles", "api_order"])
def ctx(request):
    from paper_0908_4421_amd.imrt import Context
    return Context(0, voxel_tiles=request.param)


@pytest.mark.parametrize("spec", [TINY_COARSE, SMALL_COARSE], ids=lambda s: s.name)
def test_coarse_matrix_bit_exact(ctx, spec):
    from paper_0908_4421_amd.imrt import Dose
    D = phantom.build_dose_matrix(spec)
    fine, blocks = phantom.voxel_layout(spec)
    banner(f"coarse layout {spec.name}: {len(fine)} grid voxels + {len(blocks)} coarse, nnz {D.nnz}")
    lib = Dose.from_geometry(ctx, spec)
    assert (lib.nv, lib.nb, lib.nnz) == (D.nv, D.nb, D.nnz)
    ex = lib.export(structures=True)
    assert np.array_equal(ex["row_ptr"], D.csr.indptr) and np.array_equal(ex["col_idx"], D.csr.indices)
    assert np.array_equal(ex["col_ptr"], D.csc.indptr) and np.array_equal(ex["row_idx"], D.csc.indices)
    assert f32_ulp_diff(ex["val"], D.csr.data) <= 1 and f32_ulp_diff(ex["cval"], D.csc.data) <= 1
    assert np.array_equal(ex["struct_id"], D.struct_id)


def test_coarse_tiny_trajectory(ctx):
    """200 fixed iterations from x = 1: same steps and backtracks as the
    oracle, G within 1e-6 at every index; dose over every voxel within 1e-5."""
    import torch
    from paper_0908_4421_amd.imrt import Dose, Plan
    spec = TINY_COARSE
    D = phantom.build_dose_matrix(spec)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(spec))
    lam, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, spec.seed))
    ref = solver.solve(D.csr, pen, np.ones(D.nb), eps=1e-4, alpha=2.0, lambda0=lam, max_iter=200, fixed_iters=True)
    lib = Dose.from_geometry(ctx, spec)
    plan = Plan(ctx, lib)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(spec))
    x = torch.ones(D.nb, dtype=torch.float32, device="cuda")
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=200, fixed_iters=True, trace=True)
    worst, K, _ = check_trajectory(tr, res, [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in ref.trace],
                                   ref.G_initial, None)
    assert K == 200
    d = torch.empty(D.nv, dtype=torch.float32, device="cuda")
    plan.objective(x, d)
    Dx = D.csr.astype(np.float64) @ to_host(x).astype(np.float64)
    err = float(np.max(np.abs(to_host(d) - Dx)) / np.max(np.abs(Dx)))
    banner(f"coarse tiny: worst G error {worst:.2e}, dose error {err:.2e}")
    assert err <= 1e-5


@pytest.fixture(scope="module")
def fx():
    with open(FIXTURE) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def paper():
    from paper_0908_4421_amd.imrt import Context, Dose, Plan
    banner("paper-scale coarse build")
    c = Context(0)
    dose = Dose.from_geometry(c, PAPER_SCALE_COARSE)
    plan = Plan(c, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(PAPER_SCALE_COARSE))
    return c, dose, plan, dose.export(structures=True)


def test_paper_scale_coarse_fingerprint_and_samples(paper, fx):
    c, dose, plan, ex = paper
    assert (dose.nv, dose.nb, dose.nnz) == (fx["nv"], fx["nb"], fx["nnz"])
    for key, dt in (("row_ptr", "<i4"), ("col_idx", "<i4"), ("col_ptr", "<i4"), ("row_idx", "<i4")):
        assert sha(ex[key], dt) == fx["sha256_" + key], key
    assert sha(ex["struct_id"], "u1") == fx["sha256_struct_id"]
    rng = np.random.default_rng(9)
    cols = sorted(rng.choice(dose.nb, size=8, replace=False).tolist())
    _, oc = phantom.build_columns(PAPER_SCALE_COARSE, cols)
    for i, (rows, vals) in zip(cols, oc):
        a, b = ex["col_ptr"][i], ex["col_ptr"][i + 1]
        assert np.array_equal(ex["row_idx"][a:b], rows)
        assert f32_ulp_diff(ex["cval"][a:b], vals) <= 1
    lens = np.diff(ex["row_ptr"])
    nfine = len(phantom.voxel_layout(PAPER_SCALE_COARSE)[0])
    rows = np.concatenate([rng.choice(np.nonzero(lens[:nfine] > 0)[0], 30, replace=False),
                           nfine + rng.choice(np.nonzero(lens[nfine:] > 0)[0], 30, replace=False)])
    orow = phantom.dose_rows(PAPER_SCALE_COARSE, rows, np.array(fx["emin"]))
    for j, (cc, v) in zip(rows, orow):
        a, b = ex["row_ptr"][j], ex["row_ptr"][j + 1]
        assert np.array_equal(ex["col_idx"][a:b], cc)
        assert f32_ulp_diff(ex["val"][a:b], v) <= 1


def test_paper_scale_coarse_solve(paper, fx):
    """λ0 equal to the oracle's; the solve to the stopping rule against the
    oracle's trajectory (G within 1e-6 at every index and at the GPU's stop
    index); the final dose over every voxel within 1e-5 of D x in float64."""
    import scipy.sparse as sp
    import torch
    c, dose, plan, ex = paper
    st = PAPER_SCALE_SETTINGS
    v0 = power_start_vector(dose.nb, PAPER_SCALE_COARSE.seed).astype(np.float32)
    lam, sig = plan.lambda0(to_dev(v0), st.power_iters)
    assert lam == fx["lambda0"] and abs(sig - fx["sigma"]) <= 1e-5 * fx["sigma"]
    x = to_dev(start_point(dose.nb, st).astype(np.float32))
    res, tr = plan.solve(x, eps=st.eps, alpha=st.alpha, lambda0=lam, delta=st.delta, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks, trace=True)
    worst, K, Ko = check_trajectory(tr, res, fx["trace"], fx["G_initial"], fx["iterations"], delta=st.delta)
    d = torch.empty(dose.nv, dtype=torch.float32, device="cuda")
    plan.objective(x, d)
    xg = to_host(x).astype(np.float64)
    Dx = sp.csr_matrix((ex["val"].astype(np.float64), ex["col_idx"], ex["row_ptr"]),
                       shape=(dose.nv, dose.nb)) @ xg
    err = float(np.max(np.abs(to_host(d) - Dx)) / np.max(np.abs(Dx)))
    banner(f"paper-scale coarse: {res.iterations} iterations (oracle {Ko}) in {res.device_ms:.1f} ms, "
           f"worst G error {worst:.2e}, dose error {err:.2e}")
    assert err <= 1e-5
