"""The paper's re-plan workload on the host (Section 2.1: the thresholds T_j
of Eq. (1) are the original plan's dose, reproduced on the day's anatomy by
re-optimising the fluence): the day's beams are a subset of the original
beams with identical columns of D, and the oracle's re-optimisation model
reaches G = 0 exactly where the dose equals the targets."""
import numpy as np

from oracle import model, phantom, solver
from workloads import PTV, SMALL, day_geometry, penalty_table, power_start_vector


def _keys(spec):
    return [(b.beam, b.m, b.n) for b in phantom.beamlets(spec)]


def test_day_beamlets_are_original_columns():
    day = day_geometry(SMALL)
    k0, k1 = _keys(SMALL), _keys(day)
    pos = {k: i for i, k in enumerate(k0)}
    assert all(k in pos for k in k1) and len(k1) < len(k0)
    idx = np.array([pos[k] for k in k1])
    assert np.all(np.diff(idx) > 0)           # column order kept
    D0 = phantom.build_dose_matrix(SMALL)
    D1 = phantom.build_dose_matrix(day)
    sub = D0.csc[:, idx]
    assert (sub != D1.csc).nnz == 0           # identical values and pattern
    # the anatomy moved: labels differ, the target shrank
    assert np.count_nonzero(D1.struct_id == PTV) < np.count_nonzero(D0.struct_id == PTV)


def test_reoptimisation_of_an_unchanged_anatomy_is_stationary():
    """T_j = (D x*)_j on the same anatomy: G(x*) = 0, the gradient vanishes,
    and the solver stops at once (the trial step equals x*)."""
    D = phantom.build_dose_matrix(SMALL)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 2.0, D.nb)
    x[rng.random(D.nb) < 0.2] = 0.0
    T = model.dose(D.csr, x)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(SMALL)).with_targets(T, T)
    assert model.objective(D.csr, x, pen) == 0.0
    assert np.all(model.gradient(D.csr, x, pen) == 0.0)
    lam, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, 1))
    r = solver.solve(D.csr, pen, x, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=10)
    assert r.status == solver.STALLED and r.iterations == 0
    # a perturbed start moves towards it: G falls monotonically, well below its start
    x2 = x * rng.uniform(0.8, 1.2, D.nb)
    r2 = solver.solve(D.csr, pen, x2, eps=1e-4, alpha=2.0, lambda0=lam, max_iter=50, fixed_iters=True)
    Gs = [r2.G_initial] + [e.G for e in r2.trace]
    assert all(b < a for a, b in zip(Gs, Gs[1:]))
    assert r2.G < 0.2 * r2.G_initial
