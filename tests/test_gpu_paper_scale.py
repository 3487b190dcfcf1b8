"""Paper-scale phantom (9 fields, 2.5 mm voxels, 5 mm beamlets) on the GPU,
in the launch configuration the benchmark times, against the oracle's stored
fingerprint and trajectory (tests/golden/paper_scale_oracle.json, written by
make_paper_scale_fixture.py from the oracle alone) and against oracle rows
and columns computed here one by one."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import banner, check_trajectory, f32_ulp_diff, to_dev, to_host
from oracle import phantom
from workloads import PAPER_SCALE, PAPER_SCALE_SETTINGS, penalty_table, power_start_vector, start_point

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_scale_oracle.json")


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def fx():
    with open(FIXTURE) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def built():
    from paper_0908_4421_amd.imrt import Context, Dose, Plan
    banner("paper-scale build")
    ctx = Context(0)
    dose = Dose.from_geometry(ctx, PAPER_SCALE)
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(PAPER_SCALE))
    return ctx, dose, plan, dose.export(structures=True)


def test_sparsity_and_structures_bit_exact(built, fx):
    ctx, dose, plan, ex = built
    assert (dose.nv, dose.nb, dose.nnz) == (fx["nv"], fx["nb"], fx["nnz"])
    assert sha(ex["row_ptr"], "<i4") == fx["sha256_row_ptr"]
    assert sha(ex["col_idx"], "<i4") == fx["sha256_col_idx"]
    assert sha(ex["col_ptr"], "<i4") == fx["sha256_col_ptr"]
    assert sha(ex["row_idx"], "<i4") == fx["sha256_row_idx"]
    assert sha(ex["struct_id"], "u1") == fx["sha256_struct_id"]
    v = ex["val"].astype(np.float64)
    assert abs(v.sum() - fx["val_sum"]) <= 1e-7 * fx["val_sum"]
    assert abs((v * v).sum() - fx["val_sumsq"]) <= 1e-7 * fx["val_sumsq"]


def test_sampled_columns_and_rows_against_oracle(built, fx):
    ctx, dose, plan, ex = built
    rng = np.random.default_rng(5)
    cols = sorted(rng.choice(dose.nb, size=10, replace=False).tolist())
    _, oc = phantom.build_columns(PAPER_SCALE, cols)
    for i, (rows, vals) in zip(cols, oc):
        a, b = ex["col_ptr"][i], ex["col_ptr"][i + 1]
        assert np.array_equal(ex["row_idx"][a:b], rows)
        assert f32_ulp_diff(ex["cval"][a:b], vals) <= 1
    lens = np.diff(ex["row_ptr"])
    rows = np.concatenate([rng.choice(np.nonzero(lens > 0)[0], 40, replace=False),
                           rng.choice(dose.nv, 10, replace=False)])
    orow = phantom.dose_rows(PAPER_SCALE, rows, np.array(fx["emin"]))
    for j, (c, v) in zip(rows, orow):
        a, b = ex["row_ptr"][j], ex["row_ptr"][j + 1]
        assert np.array_equal(ex["col_idx"][a:b], c)
        assert f32_ulp_diff(ex["val"][a:b], v) <= 1


def test_lambda0_matches_oracle(built, fx):
    ctx, dose, plan, ex = built
    v0 = power_start_vector(dose.nb, PAPER_SCALE.seed).astype(np.float32)
    lam, sig = plan.lambda0(to_dev(v0), PAPER_SCALE_SETTINGS.power_iters)
    assert abs(sig - fx["sigma"]) <= 1e-5 * fx["sigma"]
    assert lam == fx["lambda0"]


def test_full_solve_trajectory(built, fx):
    """Run to the stopping rule; G at every iteration index agrees with the
    oracle's trajectory within 1e-6 relative; dose at sampled voxels agrees
    with the oracle's rows applied to the GPU's plan within 1e-5."""
    banner("paper-scale solve")
    _check_full_solve(built, fx)


def test_full_solve_trajectory_block_forward(built, fx):
    """The same with workgroup-wide forward row blocks and eight adjoint
    workgroups per compute unit."""
    from paper_0908_4421_amd.imrt import Context, Dose, Plan
    banner("paper-scale solve, workgroup forward blocks")
    ctx = Context(0, fwd_wave=0, adj_wg_per_cu=8)
    dose = Dose.from_geometry(ctx, PAPER_SCALE)
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(PAPER_SCALE))
    _check_full_solve((ctx, dose, plan, built[3]), fx)


def test_full_solve_trajectory_two_trials(built, fx):
    """The same with two trial steps per forward pass:
    the trajectory does not depend on how the trials are grouped."""
    banner("paper-scale solve, two trials per pass")
    _check_full_solve(built, fx, nt=2)


def _check_full_solve(built, fx, nt=1):
    import scipy.sparse as sp
    import torch
    ctx, dose, plan, ex = built
    st = PAPER_SCALE_SETTINGS
    x = to_dev(start_point(dose.nb, st).astype(np.float32))
    res, tr = plan.solve(x, eps=st.eps, alpha=st.alpha, lambda0=fx["lambda0"], delta=st.delta,
                         max_iter=st.max_iter, max_backtracks=st.max_backtracks, trace=True, trials_per_pass=nt)
    banner(f"paper-scale solve: {res.iterations} iterations, {res.device_ms:.1f} ms")
    assert res.status == 0
    # every iteration, and the final objective at the GPU's own stop index,
    # within 1e-6 of the oracle's trajectory (stored 40 iterations past its stop)
    worst, K, Ko = check_trajectory(tr, res, fx["trace"], fx["G_initial"], fx["iterations"], delta=st.delta)
    d = torch.empty(dose.nv, dtype=torch.float32, device="cuda")
    G_at = plan.objective(x, d)
    assert G_at == res.G_final
    d = to_host(d).astype(np.float64)
    xg = to_host(x).astype(np.float64)
    assert np.all(xg >= 0)
    # dose of the final plan over every voxel: ||d - D x||_inf / ||D x||_inf
    # with D x in float64 from the exported matrix (whose index arrays hash to
    # the oracle's and whose values are within one float32 ulp of them)
    Dx = sp.csr_matrix((ex["val"].astype(np.float64), ex["col_idx"], ex["row_ptr"]),
                       shape=(dose.nv, dose.nb)) @ xg
    err_all = float(np.max(np.abs(d - Dx)) / np.max(np.abs(Dx)))
    # and per voxel, with oracle rows computed here at sampled voxels
    lens = np.diff(ex["row_ptr"])
    rng = np.random.default_rng(7)
    rows = rng.choice(np.nonzero(lens > 0)[0], 200, replace=False)
    orow = phantom.dose_rows(PAPER_SCALE, rows, np.array(fx["emin"]))
    err = 0.0
    for j, (c, v) in zip(rows, orow):
        z = float(v.astype(np.float64) @ xg[c])
        err = max(err, abs(d[j] - z) / max(abs(z), 1e-30))
    banner(f"paper-scale: stop {K} (oracle {Ko}), worst G error {worst:.2e}, dose error {err_all:.2e} "
           f"over all voxels, {err:.2e} per voxel (200 sampled)")
    assert err_all <= 1e-5
    assert err <= 1e-5
