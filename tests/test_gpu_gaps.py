"""Rows without nonzeros between the forward's row blocks.  Runs of 16 or
more empty rows are never visited by the wave forward; their penalty at zero
dose enters G as a constant of the plan, and their dose output is zero.
Checked against the FP64 oracle on a matrix with long empty runs at the
start, in the middle and at the end, short empty runs inside blocks, and
penalties whose under-dose terms make the skipped rows count in G:
objective, dose (every voxel, the skipped ones zero), gradient, per-voxel
targets, the allocation-free gradient and a 60-iteration solve."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import banner, check_trajectory, rel_normwise, to_dev, to_host
from oracle import model, solver
from workloads import penalty_table, random_penalties

pytestmark = pytest.mark.gpu


def _gapped(seed=41):
    """CSR with empty runs of lengths 700 (leading), 3, 40, 15, 16, 2,000,
    5 and 900 (trailing) between ragged non-empty rows."""
    rng = np.random.default_rng(seed)
    nb = 48
    pattern = [("e", 700), ("n", 300), ("e", 3), ("n", 120), ("e", 40), ("n", 80), ("e", 15), ("n", 60),
               ("e", 16), ("n", 500), ("e", 2000), ("n", 250), ("e", 5), ("n", 90), ("e", 900)]
    lens = []
    for kind, n in pattern:
        lens += [0] * n if kind == "e" else list(np.minimum(rng.geometric(1 / 9.0, n), nb))
    lens = np.array(lens)
    nv = len(lens)
    row_ptr = np.zeros(nv + 1, np.int32)
    np.cumsum(lens, out=row_ptr[1:])
    cols = np.concatenate([np.sort(rng.choice(nb, k, replace=False)) for k in lens if k > 0]).astype(np.int32)
    vals = rng.uniform(0.05, 1.0, len(cols)).astype(np.float32)
    sid = rng.integers(0, 4, nv).astype(np.uint8)
    return nv, nb, row_ptr, cols, vals, sid


@pytest.fixture(scope="module")
def gapped():
    from paper_0908_4421_amd.imrt import Context, Dose, Plan
    ctx = Context(0)
    nv, nb, rp, ci, v, sid = _gapped()
    table = penalty_table(random_penalties(4, 17, scale=3.0))
    lib = Dose.from_csr(ctx, nv, nb, rp, ci, v)
    plan = Plan(ctx, lib)
    plan.set_structures(sid, 4)
    plan.set_penalties(table)
    D = sp.csr_matrix((v, ci, rp), shape=(nv, nb))
    pen = model.VoxelPenalties.from_structures(sid, table)
    empty = np.diff(rp) == 0
    F0 = model.voxel_objective(np.zeros(nv), pen)
    banner(f"gapped matrix: {nv} rows, {int(empty.sum())} empty, zero-dose objective of empty rows "
           f"{F0[empty].sum():.4g}")
    assert F0[empty].sum() > 0       # the skipped rows carry objective
    return ctx, lib, plan, D, pen, sid, table


def test_objective_dose_gradient_with_gaps(gapped):
    import torch
    ctx, lib, plan, D, pen, sid, table = gapped
    rng = np.random.default_rng(3)
    for scale in (0.5, 4.0):
        x = (rng.uniform(0.0, 1.0, D.shape[1]) * scale).astype(np.float32)
        xd = to_dev(x)
        dose = torch.full((D.shape[0],), float("nan"), dtype=torch.float32, device="cuda")
        G = plan.objective(xd, dose)
        z = model.dose(D, x.astype(np.float64))
        G_ref = model.objective_from_dose(z, pen)
        assert abs(G - G_ref) <= 1e-6 * G_ref, (G, G_ref)
        d = to_host(dose)
        assert np.all(np.isfinite(d)) and np.all(d[np.diff(D.indptr) == 0] == 0.0)
        assert np.max(np.abs(d - z) / np.maximum(np.abs(z), 1e-30)) <= 1e-5
        g, G2 = plan.gradient(xd)
        assert G2 == G
        assert rel_normwise(to_host(g), model.gradient(D, x.astype(np.float64), pen)) <= 1e-5
        gn = torch.zeros_like(g)
        assert plan.gradient_noalloc(xd, gn) == G
        assert torch.equal(gn, g)
        plain = torch.full((D.shape[0],), float("nan"), dtype=torch.float32, device="cuda")
        lib.apply(xd, plain)
        assert np.array_equal(to_host(plain), d)


def test_voxel_targets_with_gaps(gapped):
    ctx, lib, plan, D, pen, sid, table = gapped
    rng = np.random.default_rng(5)
    nv = D.shape[0]
    Tu = rng.uniform(0.0, 2.0, nv).astype(np.float32)
    To = (Tu + rng.uniform(0.0, 1.0, nv)).astype(np.float32)
    plan.set_voxel_targets(Tu, To)
    try:
        x = rng.uniform(0.0, 1.0, D.shape[1]).astype(np.float32)
        G = plan.objective(to_dev(x))
        pv = pen.with_targets(Tu.astype(np.float64), To.astype(np.float64))
        G_ref = model.objective_from_dose(model.dose(D, x.astype(np.float64)), pv)
        assert abs(G - G_ref) <= 1e-6 * G_ref, (G, G_ref)
    finally:
        plan.set_voxel_targets(None, None)
    G_back = plan.objective(to_dev(x))
    G_tab = model.objective_from_dose(model.dose(D, x.astype(np.float64)), pen)
    assert abs(G_back - G_tab) <= 1e-6 * G_tab


def test_solve_with_gaps(gapped):
    """60 fixed iterations from x = 1: the oracle's steps and backtracks, G
    within 1e-6 at every index."""
    import torch
    ctx, lib, plan, D, pen, sid, table = gapped
    lam, _ = solver.lambda0_from_power_iteration(D, pen, np.ones(D.shape[1]))
    ref = solver.solve(D, pen, np.ones(D.shape[1]), eps=1e-4, alpha=2.0, lambda0=lam, max_iter=60, fixed_iters=True)
    x = torch.ones(D.shape[1], dtype=torch.float32, device="cuda")
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=60, fixed_iters=True, trace=True)
    worst, K, _ = check_trajectory(tr, res, [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in ref.trace],
                                   ref.G_initial, None)
    banner(f"gapped solve: 60 iterations, worst G error {worst:.2e}")
    assert K == 60
