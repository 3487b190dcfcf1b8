"""GPU Armijo gradient-projection solve against the FP64 oracle: the
hand-worked example, the tiny phantom's 200 fixed iterations, forced
backtracking with 1/2/4 trial steps per pass, stopping statuses and errors."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import banner, to_dev, to_host
from oracle import model, phantom, solver
from oracle_pins import floats, worked_example
from workloads import TINY, TINY_SETTINGS, penalty_table, power_start_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(1024, 1, 1), (16, 0, 1), (16, 1, 1), (1024, 1, 0)],
                ids=["default", "shared_cols_block_fwd", "shared_cols_wave_fwd", "col32_wave_fwd"])
def ctx(request):
    """Default launch settings, or many short adjoint workgroup ranges (most
    beamlet columns shared by several workgroups) with workgroup-wide or
    wave-wide forward row blocks, or the wave forward over 32-bit column
    indices (512-entry blocks) instead of 16-bit ones (768-entry blocks)."""
    from paper_0908_4421_amd.imrt import Context
    min_nnz, wave, col16 = request.param
    return Context(0, adj_min_nnz=min_nnz, fwd_wave=wave, fwd_col16=col16)


@pytest.fixture(scope="module")
def tiny(ctx):
    from paper_0908_4421_amd.imrt import Dose, Plan
    D = phantom.build_dose_matrix(TINY)
    lib = Dose.from_geometry(ctx, TINY)
    plan = Plan(ctx, lib)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(TINY))
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    lam0, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, TINY.seed))
    return D, lib, plan, pen, lam0


def _plan_from_csr(ctx, D, sid, table):
    from paper_0908_4421_amd.imrt import Dose, Plan
    D = sp.csr_matrix(D)
    lib = Dose.from_csr(ctx, D.shape[0], D.shape[1], D.indptr, D.indices, D.data)
    plan = Plan(ctx, lib)
    plan.set_structures(sid, len(table))
    plan.set_penalties(table)
    return lib, plan


@pytest.mark.parametrize("nt", [1, 2, 4])
def test_worked_example_exact(ctx, nt):
    """The hand-worked three iterations (all values dyadic, exact in float32)."""
    banner(f"worked example nt={nt}")
    g, D, pen = worked_example()
    # voxels 0,1 structure 0 (two-sided 4 Gy), voxel 2 structure 1 (over 1 Gy, w 1/2)
    table = [(4.0, 4.0, 1.0, 1.0), (0.0, 1.0, 0.0, 0.5)]
    lib, plan = _plan_from_csr(ctx, D, np.array([0, 0, 1], np.uint8), table)
    x = to_dev(floats(g["x1"]).astype(np.float32))
    res, tr = plan.solve(x, eps=float(g["eps"]), alpha=float(g["alpha"]), lambda0=float(g["lambda0"]),
                         max_iter=3, fixed_iters=True, trials_per_pass=nt, trace=True)
    assert res.status == 1 and res.iterations == 3
    assert res.G_initial == float(g["G1"])
    for (k, m, lam, s, G), key in zip(tr, ("trace1", "trace2", "trace3")):
        assert (k, lam, m, s, G) == tuple(floats(g[key]))
    assert np.array_equal(to_host(x), floats(g["x4"]).astype(np.float32))
    assert res.adjoint_passes == int(g["adjoint_products"])
    # forward passes: 1 initial + ceil((backtracks+1)/nt) per iteration
    per_iter = [3, 2, 3]
    assert res.forward_passes == 1 + sum(-(-t // nt) for t in per_iter)


def test_worked_example_eps_large(ctx):
    g, D, pen = worked_example()
    table = [(4.0, 4.0, 1.0, 1.0), (0.0, 1.0, 0.0, 0.5)]
    lib, plan = _plan_from_csr(ctx, D, np.array([0, 0, 1], np.uint8), table)
    x = to_dev(floats(g["x1"]).astype(np.float32))
    res, tr = plan.solve(x, eps=float(g["eps_large"]), alpha=2.0, lambda0=1.0, max_iter=1,
                         fixed_iters=True, trace=True)
    k, m, lam, s, G = tr[0]
    assert (k, lam, m, s, G) == tuple(floats(g["eps_large_trace1"]))


def _compare_traces(tr, ref, rel=1e-6):
    assert len(tr) == len(ref.trace)
    for (k, m, lam, s, G), e in zip(tr, ref.trace):
        assert k == e.k and m == e.backtracks and lam == e.lam, (k, m, e.backtracks)
        assert abs(G - e.G) <= rel * abs(e.G), (k, G, e.G)
        assert abs(s - e.step_sq) <= 1e-4 * e.step_sq + 1e-30


def test_tiny_phantom_200_iterations(tiny):
    """The tiny phantom's configuration: exactly 200 iterations from x = 1."""
    banner("tiny 200 iterations")
    D, lib, plan, pen, lam0 = tiny
    st = TINY_SETTINGS
    x1 = np.ones(D.nb)
    ref = solver.solve(D.csr, pen, x1, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                       max_backtracks=st.max_backtracks, fixed_iters=True)
    x = to_dev(x1.astype(np.float32))
    res, tr = plan.solve(x, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks, fixed_iters=True, trace=True)
    assert res.status == 1 and res.iterations == 200
    assert abs(res.G_initial - ref.G_initial) <= 1e-6 * ref.G_initial
    _compare_traces(tr, ref)
    assert abs(res.G_final - ref.G) <= 1e-6 * ref.G
    # dose of the GPU's own plan against the oracle's product at the same x
    import torch
    xg = to_host(x).astype(np.float64)
    dose = torch.empty(D.nv, dtype=torch.float32, device="cuda")
    G_at = plan.objective(x, dose)
    z = model.dose(D.csr, xg)
    assert np.max(np.abs(to_host(dose) - z)) <= 1e-5 * np.max(np.abs(z))
    assert abs(G_at - model.objective_from_dose(z, pen)) <= 1e-6 * G_at
    assert G_at == res.G_final
    # x agrees with the oracle's iterate
    assert np.max(np.abs(xg - ref.x)) <= 1e-4 * np.max(np.abs(ref.x))
    # a second solve is bit-identical
    x2 = to_dev(x1.astype(np.float32))
    res2, tr2 = plan.solve(x2, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                           max_backtracks=st.max_backtracks, fixed_iters=True, trace=True)
    assert tr2 == tr and np.array_equal(to_host(x2), to_host(x))


@pytest.mark.parametrize("nt", [1, 2, 4])
def test_forced_backtracking(tiny, nt):
    """A large lambda_0 makes every line search backtrack; 1, 2 or 4 trial
    steps per pass over D give the same sequence as the oracle."""
    banner(f"backtracking nt={nt}")
    D, lib, plan, pen, _ = tiny
    x1 = np.ones(D.nb)
    ref = solver.solve(D.csr, pen, x1, eps=1e-4, alpha=2.0, lambda0=0.125, max_iter=15, fixed_iters=True)
    x = to_dev(x1.astype(np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=0.125, max_iter=15, fixed_iters=True,
                         trials_per_pass=nt, trace=True)
    assert sum(e[1] for e in tr) >= 15
    _compare_traces(tr, ref)
    passes = sum(-(-(e.backtracks + 1) // nt) for e in ref.trace)
    assert res.forward_passes == 1 + passes


def test_converged_status_tiny(tiny):
    D, lib, plan, pen, lam0 = tiny
    x1 = np.ones(D.nb)
    ref = solver.solve(D.csr, pen, x1, eps=1e-4, alpha=2.0, lambda0=lam0, delta=1e-3, max_iter=5000)
    x = to_dev(x1.astype(np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam0, delta=1e-3, max_iter=5000, trace=True)
    assert res.status == 0 and ref.status == 0
    assert res.iterations == ref.iterations
    _compare_traces(tr, ref)


def test_stalled_and_line_search_failure(ctx):
    rng = np.random.default_rng(23)
    Dd = rng.uniform(0.0, 1.0, (60, 6))
    Dd[rng.random((60, 6)) < 0.3] = 0.0
    # over-dose only, threshold 0: x = 0 is optimal, the first trial equals x_1 = 0
    lib, plan = _plan_from_csr(ctx, Dd.astype(np.float32), np.zeros(60, np.uint8), [(0.0, 0.0, 0.0, 1.0)])
    x = to_dev(np.zeros(6, np.float32))
    res, _ = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=1.0, max_iter=10)
    assert res.status == 2 and res.iterations == 0
    g, D, pen = worked_example()
    table = [(4.0, 4.0, 1.0, 1.0), (0.0, 1.0, 0.0, 0.5)]
    lib, plan = _plan_from_csr(ctx, D, np.array([0, 0, 1], np.uint8), table)
    x = to_dev(floats(g["x1"]).astype(np.float32))
    res, _ = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=1.0, max_iter=10, max_backtracks=1)
    assert res.status == 3 and res.iterations == 0
    assert np.array_equal(to_host(x), floats(g["x1"]).astype(np.float32))
    res, _ = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=1.0, max_iter=0)
    assert res.status == 1 and res.iterations == 0 and res.G_final == float(g["G1"])


def test_invalid_solve_arguments(tiny):
    from paper_0908_4421_amd import imrt
    D, lib, plan, pen, lam0 = tiny
    x = np.ones(D.nb, np.float32)
    x[3] = -1.0
    with pytest.raises(imrt.ImrtError) as e:
        plan.solve(to_dev(x), eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=5)
    assert e.value.code == imrt.IMRT_EINVAL
    ok = to_dev(np.ones(D.nb, np.float32))
    for kw in (dict(eps=1.5, alpha=2.0, lambda0=lam0), dict(eps=1e-4, alpha=1.0, lambda0=lam0),
               dict(eps=1e-4, alpha=2.0, lambda0=0.0), dict(eps=1e-4, alpha=2.0, lambda0=lam0, trials_per_pass=3)):
        with pytest.raises(imrt.ImrtError) as e:
            plan.solve(ok, max_iter=5, **kw)
        assert e.value.code == imrt.IMRT_EINVAL


def test_empty_matrix(ctx):
    """D with no nonzeros (every voxel out of every beam): both products are
    zero, the objective is the structures' under-dose penalty at zero dose,
    the gradient vanishes, so the first trial equals x_1 and the solve stops
    as stalled (as the oracle does); the lambda_0 estimate reports the zero
    vector it reaches."""
    from paper_0908_4421_amd import imrt
    nv, nb = 300, 17
    Dz = sp.csr_matrix((nv, nb), dtype=np.float32)
    sid = (np.arange(nv) % 3).astype(np.uint8)
    table = [(5.0, 6.0, 1.0, 0.5), (0.0, 2.0, 0.0, 0.3), (0.0, 1.0, 0.0, 0.1)]
    lib, plan = _plan_from_csr(ctx, Dz, sid, table)
    assert (lib.nv, lib.nb, lib.nnz) == (nv, nb, 0)
    assert np.all(to_host(lib.apply(to_dev(np.ones(nb, np.float32)))) == 0.0)
    assert np.all(to_host(lib.apply_transpose(to_dev(np.ones(nv, np.float32)))) == 0.0)
    pen = model.VoxelPenalties.from_structures(sid, np.array(table))
    x1 = np.full(nb, 2.0)
    ref = solver.solve(Dz, pen, x1, eps=1e-4, alpha=2.0, lambda0=1.0, max_iter=10)
    assert ref.status == solver.STALLED and ref.iterations == 0
    x = to_dev(x1.astype(np.float32))
    res, _ = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=1.0, max_iter=10)
    assert res.status == ref.status and res.iterations == 0
    assert res.G_initial == ref.G_initial == 100 * 25.0
    assert np.all(to_host(x) == 2.0)
    with pytest.raises(imrt.ImrtError) as e:
        plan.lambda0(to_dev(np.ones(nb, np.float32)), 50)
    assert e.value.code == imrt.IMRT_EINVAL


@pytest.mark.parametrize("nt", [1, 2, 4])
def test_warm_start_one_voxel_exact(ctx, nt):
    """The warm-start variant (iteration k+1 starts at alpha times the
    accepted step) on D = [1], threshold 4: the oracle's closed-form
    trajectories, bit for bit (all values dyadic)."""
    D = np.array([[1.0]], dtype=np.float32)
    lib, plan = _plan_from_csr(ctx, D, np.zeros(1, np.uint8), [(4.0, 4.0, 1.0, 1.0)])
    x = to_dev(np.zeros(1, np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=0.125, max_iter=50, trials_per_pass=nt, trace=True,
                         warm_start=True)
    assert res.status == 0 and res.iterations == 3
    assert tr == [(1, 0, 0.125, 1.0, 9.0), (2, 0, 0.25, 2.25, 2.25), (3, 0, 0.5, 2.25, 0.0)]
    assert to_host(x)[0] == 4.0
    x = to_dev(np.zeros(1, np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=0.75, max_iter=3, fixed_iters=True, trials_per_pass=nt,
                         trace=True, warm_start=True)
    assert tr == [(1, 0, 0.75, 36.0, 4.0), (2, 1, 0.75, 9.0, 1.0), (3, 1, 0.75, 2.25, 0.25)]
    assert to_host(x)[0] == 4.5
    # one pass per trial group: 1 initial + 1 + 2 + 2 with one trial per pass
    assert res.forward_passes == 1 + sum(-(-(m + 1) // nt) for m in (0, 1, 1))


@pytest.mark.parametrize("nt", [1, 2])
def test_warm_start_tiny_phantom(tiny, nt):
    D, lib, plan, pen, lam0 = tiny
    x1 = np.ones(D.nb)
    ref = solver.solve(D.csr, pen, x1, eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=120, fixed_iters=True,
                       warm_start=True)
    assert sum(e.backtracks for e in ref.trace) > 0      # the doubled steps do get rejected
    x = to_dev(x1.astype(np.float32))
    res, tr = plan.solve(x, eps=1e-4, alpha=2.0, lambda0=lam0, max_iter=120, fixed_iters=True,
                         trials_per_pass=nt, trace=True, warm_start=True)
    # the same steps, backtracks and objective; the step norms are squared
    # differences of float32 iterates, and the overshooting trials of the
    # warm start make them follow the iterates' float32 rounding more
    # closely than the cold start's (1e-3 instead of 1e-4)
    assert len(tr) == len(ref.trace)
    for (k, m, lam, s, G), e in zip(tr, ref.trace):
        assert k == e.k and m == e.backtracks and lam == e.lam, (k, m, e.backtracks)
        assert abs(G - e.G) <= 1e-6 * abs(e.G), (k, G, e.G)
        assert abs(s - e.step_sq) <= 1e-3 * e.step_sq + 1e-30, (k, s, e.step_sq)
    assert abs(res.G_final - ref.G) <= 1e-6 * ref.G
