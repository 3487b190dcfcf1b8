"""Pins of the oracle's phantom and dose-deposition matrix (CPU only).

Each check compares the oracle against something other than itself: exact
integer or rational geometry, closed forms of special beam directions, the
truncation rule restated in the dose domain, and transposition invariants.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import phantom
from workloads import BLADDER, NORMAL, PTV, RECTUM, SMALL, TINY, PAPER_SCALE, PhantomSpec


def _scaled_int(v: float, scale: int) -> int:
    f = Fraction(v) * scale
    assert f.denominator == 1, (v, scale)
    return int(f)


def _structures_integer(spec: PhantomSpec) -> np.ndarray:
    """Structure ids in exact int64 arithmetic on a lattice scaled by 4.

    4 * ((i + 1/2) h - n h / 2) = 2 h (2 i + 1 - n); with h and every radius a
    multiple of 1/4 mm all tests become integer comparisons.
    """
    S = 4
    factor = Fraction(spec.h) * S / 2          # S * h / 2
    assert factor.denominator == 1
    def coord(n):
        k = 2 * np.arange(n, dtype=np.int64) + 1 - n
        return k * int(factor)                 # = S * ((i + 1/2) h - n h / 2)
    X = coord(spec.nx)[None, None, :]
    Y = coord(spec.ny)[None, :, None]
    Z = coord(spec.nz)[:, None, None]
    R = _scaled_int(spec.r_ptv, S)
    rr = _scaled_int(spec.r_rectum, S)
    rb = _scaled_int(spec.r_bladder, S)
    cy_r = -(R + rr)
    cy_b = R + rb
    sid = np.full((spec.nz, spec.ny, spec.nx), NORMAL, dtype=np.uint8)
    bladder = X * X + (Y - cy_b) ** 2 + Z * Z <= rb * rb
    rectum = (X * X + (Y - cy_r) ** 2 + 0 * Z) <= rr * rr
    ptv = X * X + Y * Y + Z * Z <= R * R
    sid[np.broadcast_to(bladder, sid.shape)] = BLADDER
    sid[np.broadcast_to(rectum, sid.shape)] = RECTUM
    sid[np.broadcast_to(ptv, sid.shape)] = PTV
    return sid.ravel()


@pytest.mark.parametrize("spec", [TINY, SMALL, PAPER_SCALE], ids=lambda s: s.name)
def test_structure_ids_exact_lattice(spec):
    got = phantom.structure_ids(spec)
    want = _structures_integer(spec)
    assert got.dtype == np.uint8 and got.shape == (spec.nv,)
    assert np.array_equal(got, want)
    # every structure is present and the PTV is mirror-symmetric in x and z
    assert set(np.unique(got)) == {NORMAL, PTV, RECTUM, BLADDER}
    g3 = got.reshape(spec.nz, spec.ny, spec.nx)
    assert np.array_equal(g3, g3[:, :, ::-1]) and np.array_equal(g3, g3[::-1, :, :])


def test_structure_ids_rational_brute_force_tiny():
    """Pure-Python exact rational classification of every tiny-phantom voxel."""
    spec = TINY
    h = Fraction(spec.h)
    R, rr, rb = Fraction(spec.r_ptv), Fraction(spec.r_rectum), Fraction(spec.r_bladder)
    got = phantom.structure_ids(spec)
    j = 0
    for iz in range(spec.nz):
        z = (iz + Fraction(1, 2)) * h - spec.nz * h / 2
        for iy in range(spec.ny):
            y = (iy + Fraction(1, 2)) * h - spec.ny * h / 2
            for ix in range(spec.nx):
                x = (ix + Fraction(1, 2)) * h - spec.nx * h / 2
                if x * x + y * y + z * z <= R * R:
                    want = PTV
                elif x * x + (y + R + rr) ** 2 <= rr * rr:
                    want = RECTUM
                elif x * x + (y - R - rb) ** 2 + z * z <= rb * rb:
                    want = BLADDER
                else:
                    want = NORMAL
                assert got[j] == want, (ix, iy, iz)
                j += 1


@pytest.mark.parametrize("spec", [TINY, SMALL, PAPER_SCALE], ids=lambda s: s.name)
def test_beamlet_set_integer(spec):
    """Beamlets = integer squares whose closest point to the axis is within reach."""
    S = 4
    w = _scaled_int(spec.beamlet, S)
    reach = _scaled_int(spec.r_ptv + spec.margin, S)
    per_beam = []
    for m in range(-200, 200):
        cu = 0 if m * w <= 0 <= (m + 1) * w else min(abs(m * w), abs((m + 1) * w))
        for n in range(-200, 200):
            cv = 0 if n * w <= 0 <= (n + 1) * w else min(abs(n * w), abs((n + 1) * w))
            if cu * cu + cv * cv <= reach * reach:
                per_beam.append((m, n))
    bls = phantom.beamlets(spec)
    got = [(b.beam, b.m, b.n) for b in bls]
    want = [(b, m, n) for b in range(spec.n_beams) for (m, n) in per_beam]
    assert got == want
    # four-fold symmetry of the footprint about the beam axis
    s = set(per_beam)
    assert all((-1 - m, n) in s and (m, -1 - n) in s for (m, n) in s)
    for b in bls:
        assert b.u_c == (b.m + 0.5) * spec.beamlet and b.v_c == (b.n + 0.5) * spec.beamlet


def test_paper_scale_beamlet_count():
    # 9 fields of 5 mm beamlets over a 40 mm reach: 232 beamlets per field
    assert len(phantom.beamlets(PAPER_SCALE)) == 9 * 232
    assert len(phantom.beamlets(TINY)) == 5 * 32


def test_depth_closed_forms():
    """Depth for 0, 90 and 45 degree beams against the entry-face distance."""
    spec = PhantomSpec(name="sq", nx=12, ny=12, nz=3, h=5.0, r_ptv=10.0, r_rectum=3.0,
                       r_bladder=5.0, n_beams=8, beamlet=5.0, sigma=3.0, tau=0.01)
    x, y, z = phantom.voxel_centres(spec)
    hx = spec.nx * spec.h / 2
    hy = spec.ny * spec.h / 2
    dirs = phantom.beam_directions(spec)
    d0, u0 = phantom.beam_depth_and_u(spec, x, y, *dirs[0])
    assert np.array_equal(d0, x + hx) and np.array_equal(u0, y)
    d2, u2 = phantom.beam_depth_and_u(spec, x, y, *dirs[2])          # 90 degrees
    np.testing.assert_allclose(d2, y + hy, rtol=0, atol=1e-12)
    np.testing.assert_allclose(u2, -x, rtol=0, atol=1e-12)
    d1, u1 = phantom.beam_depth_and_u(spec, x, y, *dirs[1])          # 45 degrees
    c = math.sqrt(0.5)
    np.testing.assert_allclose(d1, np.minimum(x + hx, y + hy) / c, rtol=1e-13)
    np.testing.assert_allclose(u1, (y - x) * c, rtol=0, atol=1e-12)
    d4, _ = phantom.beam_depth_and_u(spec, x, y, *dirs[4])          # 180 degrees
    np.testing.assert_allclose(d4, hx - x, rtol=0, atol=1e-12)
    assert np.all(d0 >= 0) and np.all(d1 >= 0) and np.all(d4 >= 0)


def test_beam0_columns_closed_form_and_truncation():
    """For the 0-degree beam, D_ij = exp(-(mu (x + L/2) + ((y-u_c)^2 + (z-v_c)^2)/(2 s^2)))
    and the kept set is {D_ij >= tau * max_j D_ij} (stated in the dose domain)."""
    spec = TINY
    bls, cols = phantom.build_columns(spec)
    x, y, z = phantom.voxel_centres(spec)
    hx = spec.nx * spec.h / 2
    n0 = sum(1 for b in bls if b.beam == 0)
    for i in range(n0):
        b = bls[i]
        dense = np.exp(-(spec.mu * (x + hx) + ((y - b.u_c) ** 2 + (z - b.v_c) ** 2)
                         / (2 * spec.sigma ** 2)))
        rel = dense / (spec.tau * dense.max())
        assert not np.any(np.abs(rel - 1.0) < 1e-9), "ambiguous truncation tie"
        want_rows = np.nonzero(rel >= 1.0)[0]
        rows, vals = cols[i]
        assert np.array_equal(rows, want_rows)
        np.testing.assert_allclose(vals, dense[rows].astype(np.float32), rtol=2.5e-7, atol=0)


def test_csr_csc_are_transposes_and_sorted():
    D = phantom.build_dose_matrix(TINY)
    assert D.nv == TINY.nv and D.nb == 160 and D.nnz == 115456
    csr, csc = D.csr, D.csc
    assert csr.indptr.dtype == np.int32 and csr.indices.dtype == np.int32
    assert csr.data.dtype == np.float32 and csc.data.dtype == np.float32
    for j in range(0, D.nv, 97):
        c = csr.indices[csr.indptr[j]:csr.indptr[j + 1]]
        assert np.all(np.diff(c) > 0)
    for i in range(D.nb):
        r = csc.indices[csc.indptr[i]:csc.indptr[i + 1]]
        assert np.all(np.diff(r) > 0)
    dense_r = csr.toarray()
    dense_c = csc.toarray()
    assert np.array_equal(dense_r, dense_c)
    assert np.all(dense_r >= 0) and np.all(dense_r <= 1)
    # each column's largest entry is the beamlet maximum exp(-e_min) <= 1
    assert np.all(dense_c.max(axis=0) > 0.2)


def test_tiny_shape_statistics():
    """Row/column statistics of the tiny phantom (a regression fingerprint)."""
    D = phantom.build_dose_matrix(TINY)
    lens = np.diff(D.csr.indptr)
    assert int(lens.max()) == 22
    assert abs((lens > 0).mean() - 0.682) < 0.001
    cl = np.diff(D.csc.indptr)
    assert int(cl.min()) == 640 and int(cl.max()) == 806


# An odd-sized grid with an odd number of beams (three: 0, 120, 240 degrees),
# so that no beam is axis-aligned but the first.
ODD = PhantomSpec(name="odd_17x13x9_5mm_3field", nx=17, ny=13, nz=9, h=5.0, r_ptv=12.5,
                  r_rectum=5.0, r_bladder=7.5, n_beams=3, beamlet=5.0, sigma=3.0, tau=0.01)


@pytest.mark.parametrize("spec", [TINY, SMALL, ODD], ids=lambda s: s.name)
def test_dose_rows_equal_the_matrix_rows(spec):
    """dose_rows (rows of D evaluated voxel by voxel, given every beamlet's
    e_min) gives exactly the rows of the column-built matrix, for every row:
    the same kept beamlets and bit-identical float32 values."""
    D = phantom.build_dose_matrix(spec)
    emin = phantom.column_minima(spec)
    rows = phantom.dose_rows(spec, np.arange(spec.nv), emin)
    csr = D.csr
    for j, (cols, vals) in enumerate(rows):
        lo, hi = csr.indptr[j], csr.indptr[j + 1]
        assert np.array_equal(cols, csr.indices[lo:hi]), j
        assert vals.dtype == np.float32 and np.array_equal(vals, csr.data[lo:hi]), j


@pytest.mark.parametrize("spec", [TINY, SMALL, ODD], ids=lambda s: s.name)
def test_column_minima_give_the_column_maxima(spec):
    """exp(-e_min) rounded to float32 is each column's largest entry (every
    column keeps its own minimum-exponent voxel), and e_min is the smallest
    exponent of the column: no voxel of the grid has a smaller one."""
    D = phantom.build_dose_matrix(spec)
    emin = phantom.column_minima(spec)
    assert emin.shape == (D.nb,) and np.all(np.isfinite(emin)) and np.all(emin >= 0)
    colmax = np.array([D.csc.data[D.csc.indptr[i]:D.csc.indptr[i + 1]].max() for i in range(D.nb)])
    assert np.array_equal(np.exp(-emin).astype(np.float32), colmax)
    # brute force over the grid for a few beamlets, one formula at a time
    x, y, z = phantom.voxel_centres(spec)
    bls = phantom.beamlets(spec)
    for i in range(0, D.nb, max(1, D.nb // 7)):
        b = bls[i]
        th = (2.0 * math.pi * b.beam) / spec.n_beams
        c, s = math.cos(th), math.sin(th)
        depth, u = phantom.beam_depth_and_u(spec, x, y, c, s)
        e = (spec.mu * depth) + (((u - b.u_c) ** 2 + (z - b.v_c) ** 2) / ((2.0 * spec.sigma) * spec.sigma))
        assert abs(e.min() - emin[i]) <= 1e-12 * max(1.0, emin[i])


def test_process_pool_build_equals_serial():
    """The process-pool build gives the serial build's arrays, element for
    element (the paper-scale fixtures are written with a pool)."""
    a = phantom.build_dose_matrix(SMALL)
    b = phantom.build_dose_matrix(SMALL, workers=3)
    for p, q in ((a.csr, b.csr), (a.csc, b.csc)):
        assert np.array_equal(p.indptr, q.indptr) and np.array_equal(p.indices, q.indices)
        assert p.data.dtype == q.data.dtype and np.array_equal(p.data, q.data)
    assert np.array_equal(a.struct_id, b.struct_id)
    assert [(t.beam, t.m, t.n) for t in a.beamlets] == [(t.beam, t.m, t.n) for t in b.beamlets]
