"""Planted mistakes: each plausible slip in the oracle must fail a pin.

The mistakes are planted in the oracle only, on the CPU, by monkeypatching;
the pins are the same checkers the oracle tests use.
"""
import numpy as np
import scipy.sparse as sp

from oracle import model, phantom, solver
from oracle_pins import fd_gradient_error, floats, kkt_closed_form_errors, worked_example
from workloads import TINY, random_csr, random_penalties


def _problem():
    A = random_csr(150, 25, 5, seed=31)
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))
    pen = model.VoxelPenalties.from_structures(A.struct_id, np.array(
        [[p.T_under, p.T_over, p.w_under, p.w_over] for p in random_penalties(4, 5, scale=3.0)]))
    x = np.random.default_rng(1).uniform(0, 1.5, A.nb)
    return D, pen, x


def test_pins_hold_without_mistakes():
    D, pen, x = _problem()
    assert fd_gradient_error(D, pen, x, range(25))[0] <= 1e-6
    assert kkt_closed_form_errors() == []


def test_constant_kkt_residual_is_caught(monkeypatch):
    """A residual that always reads 0 (it would pass every check made at an
    optimum) fails the hand-worked one-voxel cases."""
    monkeypatch.setattr(solver, "kkt_residual", lambda D_, p, x_: 0.0)
    assert len(kkt_closed_form_errors()) == 4


def test_kkt_residual_without_projection_is_caught(monkeypatch):
    """Dropping the projection (|grad G| instead of |x - max(0, x - grad G)|)
    fails the cases where the bound x >= 0 is active."""
    monkeypatch.setattr(solver, "kkt_residual",
                        lambda D_, p, x_: float(np.max(np.abs(model.gradient(D_, x_, p)))))
    assert kkt_closed_form_errors() != []


def test_dropped_underdose_term_is_caught(monkeypatch):
    D, pen, x = _problem()
    monkeypatch.setattr(model, "residual", lambda z, p: p.w_over * np.maximum(z - p.T_over, 0.0))
    assert fd_gradient_error(D, pen, x, range(25))[0] > 1e-3


def test_wrong_residual_sign_is_caught(monkeypatch):
    D, pen, x = _problem()
    orig = model.residual
    monkeypatch.setattr(model, "residual", lambda z, p: -orig(z, p))
    assert fd_gradient_error(D, pen, x, range(25))[0] > 1e-3


def test_missing_factor_two_is_caught(monkeypatch):
    D, pen, x = _problem()
    monkeypatch.setattr(model, "gradient",
                        lambda D_, x_, p: model.adjoint(D_, model.residual(model.dose(D_, x_), p)))
    assert fd_gradient_error(D, pen, x, range(25))[0] > 1e-3


def test_transposed_adjoint_is_caught(monkeypatch):
    """A square D makes D r type-check; the adjoint identity still fails."""
    rng = np.random.default_rng(2)
    Dd = rng.uniform(0, 1, (30, 30)).astype(np.float32)
    D = sp.csr_matrix(Dd)
    x, r = rng.uniform(0, 1, 30), rng.standard_normal(30)
    monkeypatch.setattr(model, "adjoint", lambda D_, r_: model.as_f64_matrix(D_) @ r_)
    lhs, rhs = model.dose(D, x) @ r, x @ model.adjoint(D, r)
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


def test_wrong_threshold_in_overdose_is_caught(monkeypatch):
    """Using T_under in the over-dose term breaks the hand-worked branch case."""
    g, _, _ = worked_example()
    monkeypatch.setattr(model, "under_over", lambda z, p: (np.minimum(z - p.T_under, 0.0),
                                                           np.maximum(z - p.T_under, 0.0)))
    D = sp.csr_matrix(np.array([[2.0]], dtype=np.float32))
    lhs, rhs = g["branch_inside"].split("->")
    tu, to, wu, wo = floats(lhs)
    pen = model.VoxelPenalties(np.array([tu]), np.array([to]), np.array([wu]), np.array([wo]))
    assert model.objective(D, np.array([3.0]), pen) != floats(rhs)[0]


def test_eps_large_golden_decides_sufficient_decrease():
    """With eps = 0.45 the sufficient-decrease term (eps/lambda)*s decides the
    line search (hand-worked); eps*lambda or a missing term gives another count."""
    g, D, pen = worked_example()
    res = solver.solve(D, pen, floats(g["x1"]), eps=float(g["eps_large"]), alpha=2.0,
                       lambda0=1.0, max_iter=1, fixed_iters=True)
    e = res.trace[0]
    assert (e.k, e.lam, e.backtracks, e.step_sq, e.G) == tuple(floats(g["eps_large_trace1"]))


def test_mirrored_lateral_axis_is_caught(monkeypatch):
    """Flipping the lateral axis sign moves beam-0 columns off their closed form."""
    orig = phantom.beam_depth_and_u
    def bad(spec, x, y, c, s):
        d, u = orig(spec, x, y, c, s)
        return d, -u
    monkeypatch.setattr(phantom, "beam_depth_and_u", bad)
    bls, cols = phantom.build_columns(TINY, which=[3])
    x, y, z = phantom.voxel_centres(TINY)
    b = bls[3]
    dense = np.exp(-(TINY.mu * (x + TINY.nx * TINY.h / 2)
                     + ((y - b.u_c) ** 2 + (z - b.v_c) ** 2) / (2 * TINY.sigma ** 2)))
    rows, _ = cols[0]
    want = np.nonzero(dense >= TINY.tau * dense.max())[0]
    assert not np.array_equal(rows, want)


def _round_variant(how):
    """round_to_format with the rounding step replaced (planted mistakes)."""
    from oracle import quantize

    def f(v, fmt):
        p, emin = quantize.FORMATS[fmt]
        v = np.asarray(v, dtype=np.float64)
        out = np.zeros_like(v)
        nz = v > 0
        _, E = np.frexp(v[nz])
        qe = np.maximum(E.astype(np.int64) - 1, emin) - (p - 1)
        n = np.ldexp(v[nz], -qe)
        out[nz] = np.ldexp(how(n), qe)
        return out
    return f


def test_truncating_quantiser_is_caught(monkeypatch):
    from oracle import quantize
    import test_oracle_quantize as T
    monkeypatch.setattr(quantize, "round_to_format", _round_variant(np.floor))
    try:
        T.test_bf16_matches_torch_conversion()
    except AssertionError:
        return
    raise AssertionError("truncation not caught")


def test_ties_away_from_zero_is_caught(monkeypatch):
    from oracle import quantize
    import test_oracle_quantize as T
    monkeypatch.setattr(quantize, "round_to_format", _round_variant(lambda n: np.floor(n + 0.5)))
    try:
        T.test_ties_go_to_even()
    except AssertionError:
        return
    raise AssertionError("ties away from zero not caught")


def test_wrong_exponent_offset_is_caught(monkeypatch):
    """One significand bit too many (quantum off by a factor two)."""
    from oracle import quantize
    import test_oracle_quantize as T
    monkeypatch.setitem(quantize.FORMATS, "f16", (12, -14))
    try:
        T.test_f16_matches_numpy_conversion()
    except (AssertionError, ValueError):
        return
    raise AssertionError("wrong precision not caught")


def test_sum_instead_of_max_scale_is_caught(monkeypatch):
    from oracle import quantize
    import test_oracle_quantize as T

    def col_sums(D):
        C = sp.csc_matrix(D)
        s = np.asarray(C.sum(axis=0)).ravel().astype(np.float32)
        s[s == 0] = 1.0
        return s
    monkeypatch.setattr(quantize, "column_scales", col_sums)
    try:
        T.test_stored_form_properties("bf16")
    except AssertionError:
        return
    raise AssertionError("sum scale not caught")


def _coarse_pins_fail():
    """Run the coarse-layout pins; return True if any of them fails."""
    import pytest as _pytest
    import test_oracle_coarse as C
    from workloads import TINY_COARSE
    try:
        C.test_layout_block_by_block(C.EVEN)
        C.test_coarse_centres_are_exact_block_means(TINY_COARSE)
        C.test_rows_against_the_uniform_and_the_doubled_grid(C.EVEN)
    except (AssertionError, _pytest.fail.Exception):
        return True
    return False


def test_coarse_pins_hold_without_mistakes():
    assert not _coarse_pins_fail()


def test_coarse_centre_off_by_half_a_voxel_is_caught(monkeypatch):
    """Coarse centres at 2 b h - n h / 2 (the block's corner voxel instead of
    the block's middle) fail the block-mean and doubled-grid pins."""
    real = phantom.coarse_centres

    def shifted(spec, blocks):
        x, y, z = real(spec, blocks)
        return x - spec.h / 2, y - spec.h / 2, z - spec.h / 2
    monkeypatch.setattr(phantom, "coarse_centres", shifted)
    assert _coarse_pins_fail()


def test_coarse_minima_over_the_layout_are_caught(monkeypatch):
    """Truncating against the minimum over the layout's voxels (instead of
    the full grid) changes kept entries, which the uniform-phantom rows
    catch."""
    real = phantom.kept_entries
    monkeypatch.setattr(phantom, "kept_entries", lambda spec, e, emin: real(spec, e, e.min()))
    assert _coarse_pins_fail()


def test_coarse_blocks_with_an_organ_voxel_are_caught(monkeypatch):
    """Merging blocks with up to one non-normal voxel fails the block scan."""
    def loose(spec):
        cx, cy, cz = spec.nx // 2, spec.ny // 2, spec.nz // 2
        sid = phantom.grid_structure_ids(spec).reshape(spec.nz, spec.ny, spec.nx)
        sub = sid[:2 * cz, :2 * cy, :2 * cx].reshape(cz, 2, cy, 2, cx, 2)
        ok = np.sum(sub != 0, axis=(1, 3, 5)) <= 1
        return np.nonzero(ok.ravel())[0].astype(np.int64)
    monkeypatch.setattr(phantom, "coarse_blocks", loose)
    assert _coarse_pins_fail()
