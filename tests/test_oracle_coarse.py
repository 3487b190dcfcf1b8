"""Pins of the oracle's coarse unspecified-tissue layout (Section 3.1:
voxels outside the target and organs at twice the size in each dimension),
CPU only.

The layout is checked against exact integer structures and a block-by-block
scan; coarse voxel centres against the exact mean of their eight grid
voxels; rows of D against two independent evaluations: the voxels at the
grid spacing must keep their rows of the uniform phantom, and each coarse
voxel must have the row of the matching voxel of a grid at twice the spacing
over the same box (both with the full grid's e_min)."""
import dataclasses
from fractions import Fraction

import numpy as np
import pytest

from oracle import phantom
from test_oracle_phantom import _structures_integer
from workloads import NORMAL, SMALL_COARSE, TINY_COARSE, PhantomSpec

# an even grid small enough for full scans, with every structure present
EVEN = PhantomSpec(name="even_24x20x10_4mm_5field_coarse", nx=24, ny=20, nz=10, h=4.0, r_ptv=12.0,
                   r_rectum=5.0, r_bladder=7.5, n_beams=5, beamlet=5.0, sigma=3.0, tau=0.01,
                   coarse_normal=True)


def _uniform(spec):
    return dataclasses.replace(spec, coarse_normal=False)


@pytest.mark.parametrize("spec", [TINY_COARSE, SMALL_COARSE, EVEN], ids=lambda s: s.name)
def test_layout_block_by_block(spec):
    """A block is coarse exactly when it is aligned, lies wholly inside the
    grid and its eight voxels are normal tissue (exact integer structures);
    the fine voxels are the grid voxels of no coarse block."""
    sid = _structures_integer(spec).reshape(spec.nz, spec.ny, spec.nx)
    want = []
    cx, cy = spec.nx // 2, spec.ny // 2
    for bz in range((spec.nz + 1) // 2):
        for by in range((spec.ny + 1) // 2):
            for bx in range((spec.nx + 1) // 2):
                if 2 * bx + 1 >= spec.nx or 2 * by + 1 >= spec.ny or 2 * bz + 1 >= spec.nz:
                    continue            # incomplete block at an upper face
                cube = sid[2 * bz:2 * bz + 2, 2 * by:2 * by + 2, 2 * bx:2 * bx + 2]
                if np.all(cube == NORMAL):
                    want.append(bx + cx * (by + cy * bz))
    fine, blocks = phantom.voxel_layout(spec)
    assert blocks.tolist() == want
    assert 0 < len(blocks) and len(fine) < spec.grid_voxels
    in_block = set()
    for b in want:
        bx, by, bz = b % cx, (b // cx) % cy, b // (cx * cy)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    in_block.add((2 * bx + dx) + spec.nx * ((2 * by + dy) + spec.ny * (2 * bz + dz)))
    assert fine.tolist() == [j for j in range(spec.grid_voxels) if j not in in_block]
    assert len(fine) + 8 * len(blocks) == spec.grid_voxels
    assert phantom.voxel_count(spec) == len(fine) + len(blocks)
    # structure ids: the grid voxel's own, normal for coarse voxels
    got = phantom.structure_ids(spec)
    assert np.array_equal(got[:len(fine)], sid.ravel()[fine])
    assert np.all(got[len(fine):] == NORMAL)
    with pytest.raises(ValueError):
        _ = spec.nv


def test_odd_grid_keeps_incomplete_blocks_fine():
    """SMALL's odd sizes: no coarse voxel touches the last x, y or z layer."""
    fine, blocks = phantom.voxel_layout(SMALL_COARSE)
    bx, by, bz = phantom.block_axes(SMALL_COARSE, blocks)
    assert np.all(2 * bx + 1 < SMALL_COARSE.nx - 1) and np.all(2 * by + 1 < SMALL_COARSE.ny - 1)
    assert np.all(2 * bz + 1 < SMALL_COARSE.nz - 1)
    last = [j for j in range(SMALL_COARSE.grid_voxels) if j % SMALL_COARSE.nx == SMALL_COARSE.nx - 1]
    assert set(last) <= set(fine.tolist())


@pytest.mark.parametrize("spec", [TINY_COARSE, SMALL_COARSE], ids=lambda s: s.name)
def test_coarse_centres_are_exact_block_means(spec):
    fine, blocks = phantom.voxel_layout(spec)
    x, y, z = phantom.voxel_centres(spec)
    gx, gy, gz = phantom.grid_centres(spec)
    assert np.array_equal(x[:len(fine)], gx[fine]) and np.array_equal(z[:len(fine)], gz[fine])
    cx, cy = spec.nx // 2, spec.ny // 2
    for k in range(0, len(blocks), max(1, len(blocks) // 50)):
        b = int(blocks[k])
        bx, by, bz = b % cx, (b // cx) % cy, b // (cx * cy)
        js = [(2 * bx + dx) + spec.nx * ((2 * by + dy) + spec.ny * (2 * bz + dz))
              for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        for got, grid in ((x, gx), (y, gy), (z, gz)):
            mean = sum(Fraction(float(grid[j])) for j in js) / 8
            assert Fraction(float(got[len(fine) + k])) == mean


@pytest.mark.parametrize("spec", [TINY_COARSE, EVEN], ids=lambda s: s.name)
def test_rows_against_the_uniform_and_the_doubled_grid(spec):
    """Fine rows equal the uniform phantom's rows at those voxels; coarse
    rows equal the rows of the grid at spacing 2h over the same box, all
    with the full grid's e_min (bit-identical indices and float32 values)."""
    D = phantom.build_dose_matrix(spec)
    fine, blocks = phantom.voxel_layout(spec)
    U = phantom.build_dose_matrix(_uniform(spec))
    assert D.nv == len(fine) + len(blocks) and D.nb == U.nb
    emin = phantom.column_minima(spec)
    assert np.array_equal(emin, phantom.column_minima(_uniform(spec)))
    for r, j in enumerate(fine):
        a = slice(D.csr.indptr[r], D.csr.indptr[r + 1])
        b = slice(U.csr.indptr[j], U.csr.indptr[j + 1])
        assert np.array_equal(D.csr.indices[a], U.csr.indices[b]) and np.array_equal(D.csr.data[a], U.csr.data[b])
    assert spec.nx % 2 == 0 and spec.ny % 2 == 0 and spec.nz % 2 == 0
    doubled = dataclasses.replace(_uniform(spec), nx=spec.nx // 2, ny=spec.ny // 2, nz=spec.nz // 2, h=2 * spec.h)
    rows = phantom.dose_rows(doubled, blocks, emin)     # block index = the doubled grid's voxel index
    for k, (cols, vals) in enumerate(rows):
        r = len(fine) + k
        sl = slice(D.csr.indptr[r], D.csr.indptr[r + 1])
        assert np.array_equal(D.csr.indices[sl], cols) and np.array_equal(D.csr.data[sl], vals), k
    # the coarse layout is smaller in rows and nonzeros
    assert D.nnz < U.nnz


def test_coarse_matrix_transposes():
    D = phantom.build_dose_matrix(SMALL_COARSE)
    assert (D.csr != D.csc.tocsr()).nnz == 0
    assert D.struct_id.shape == (D.nv,)
