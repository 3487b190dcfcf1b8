"""Pins of the oracle's penalty model, gradient and projection (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import model, phantom
from oracle_pins import fd_gradient_error, floats, worked_example
from workloads import TINY, penalty_table, random_csr, random_penalties


def test_single_voxel_branches_golden():
    """Eq. (1) branch values worked by hand (golden file)."""
    g, _, _ = worked_example()
    D = sp.csr_matrix(np.array([[2.0]], dtype=np.float32))
    x = np.array([3.0])
    for key in ("branch_under", "branch_inside", "branch_over"):
        lhs, rhs = g[key].split("->")
        tu, to, wu, wo = floats(lhs)
        F, r, grad = floats(rhs)
        pen = model.VoxelPenalties(np.array([tu]), np.array([to]), np.array([wu]), np.array([wo]))
        z = model.dose(D, x)
        assert z[0] == 6.0
        assert model.objective(D, x, pen) == F
        assert model.residual(z, pen)[0] == r
        assert model.gradient(D, x, pen)[0] == grad


def test_worked_example_first_objective_and_gradient():
    g, D, pen = worked_example()
    x1 = floats(g["x1"])
    assert model.objective(D, x1, pen) == float(g["G1"])
    assert np.array_equal(model.gradient(D, x1, pen), floats(g["grad1"]))


def test_objective_zero_inside_band():
    rng = np.random.default_rng(3)
    A = random_csr(200, 30, 6, seed=4)
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))
    x = rng.uniform(0, 2, A.nb)
    z = model.dose(D, x)
    pen = model.VoxelPenalties(z - rng.uniform(0, 1, z.size), z + rng.uniform(0, 1, z.size),
                               np.ones(z.size), np.ones(z.size))
    assert model.objective(D, x, pen) == 0.0
    assert np.all(model.gradient(D, x, pen) == 0.0)


def test_two_sided_equals_weighted_least_squares():
    """All voxels two-sided with T_u = T_o: G = ||W^1/2 (D x - T)||^2 (numpy norm)."""
    rng = np.random.default_rng(5)
    A = random_csr(300, 40, 8, seed=6, empty_frac=0.1)
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))
    Dd = D.toarray().astype(np.float64)
    x = rng.uniform(0, 3, A.nb)
    T = rng.uniform(0, 5, A.nv)
    w = rng.uniform(0.1, 2.0, A.nv)
    pen = model.VoxelPenalties(T, T, w, w)
    want = np.linalg.norm(np.sqrt(w) * (Dd @ x - T)) ** 2
    assert abs(model.objective(D, x, pen) - want) <= 1e-13 * want
    # its gradient is the normal-equations residual 2 D^T W (D x - T)
    gw = 2 * Dd.T @ (w * (Dd @ x - T))
    np.testing.assert_allclose(model.gradient(D, x, pen), gw, rtol=1e-12, atol=1e-12 * np.abs(gw).max())


def test_dose_and_adjoint_against_dense():
    """Sparse products against dense numpy, and <Dx, r> = <x, D^T r>."""
    D = phantom.build_dose_matrix(TINY)
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 2, D.nb)
    r = rng.standard_normal(D.nv)
    Dd = D.csr.toarray().astype(np.float64)
    np.testing.assert_allclose(model.dose(D.csr, x), Dd @ x, rtol=1e-13)
    np.testing.assert_allclose(model.adjoint(D.csr, r), Dd.T @ r, rtol=1e-12, atol=1e-12)
    lhs = model.dose(D.csr, x) @ r
    rhs = x @ model.adjoint(D.csr, r)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt((model.dose(D.csr, x) ** 2).sum() * (r ** 2).sum())
    # a row sum is the dose of x = 1
    np.testing.assert_allclose(model.dose(D.csc, np.ones(D.nb)), Dd.sum(axis=1), rtol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_central_differences_random(seed):
    A = random_csr(150, 25, 5, seed=10 + seed)
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))
    pen = model.VoxelPenalties.from_structures(A.struct_id, np.array(
        [[p.T_under, p.T_over, p.w_under, p.w_over] for p in random_penalties(4, seed, scale=3.0)]))
    x = np.random.default_rng(seed).uniform(0, 1.5, A.nb)
    err, used = fd_gradient_error(D, pen, x, range(A.nb))
    assert used >= 20
    assert err <= 1e-6


def test_gradient_central_differences_tiny_phantom():
    D = phantom.build_dose_matrix(TINY)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    rng = np.random.default_rng(11)
    x = rng.uniform(0.5, 20.0, D.nb)
    coords = rng.choice(D.nb, size=30, replace=False)
    err, used = fd_gradient_error(D.csr, pen, x, coords)
    assert used >= 20
    assert err <= 1e-6


def test_projection_is_the_closed_form_argmin():
    rng = np.random.default_rng(12)
    y = rng.standard_normal(500) * 3
    p = model.project(y)
    assert np.all(p >= 0)
    assert np.array_equal(model.project(p), p)
    # coordinate-wise: the nearest nonnegative number is y if y >= 0 else 0
    assert np.array_equal(p, np.where(y >= 0, y, 0.0))
    # no random feasible point is closer to y
    for _ in range(200):
        q = np.abs(rng.standard_normal(500)) * rng.uniform(0, 3)
        assert np.linalg.norm(y - p) <= np.linalg.norm(y - q)
