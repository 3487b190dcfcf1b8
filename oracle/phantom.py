"""FP64 oracle: phantom structures and the dose-deposition matrix D.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.

The paper takes D from a clinical dose engine (Section 2.1: D_ij is the dose
to voxel j from beamlet i of unit intensity; Section 2.3 stores it in CSR).
Here D comes from a synthetic pencil-beam model, evaluated by brute force over
every (voxel, beamlet) pair in float64, with every arithmetic expression
written in one fixed order so that an independent implementation that follows
the same formulas (IEEE float64, no fused multiply-add) reproduces the
sparsity pattern bit for bit:

  voxel centre   p_a = (i_a + 0.5)*h - (n_a*h)/2         (a = x, y, z)
  beam b         theta = (2*pi*b)/B, c = cos(theta), s = sin(theta)
                 (host libm cos/sin, computed once per beam)
  depth          t_a = min((lo_a - p_a)/dir_a, (hi_a - p_a)/dir_a) for the
                 in-plane axes with dir_a != 0, dir = (c, s); depth = -max t_a
  lateral        u = (-s)*x + c*y,  v = z
  beamlet (m,n)  centre (u_c, v_c) = ((m+0.5)*w, (n+0.5)*w)
  exponent       e = (mu*depth) + (r2/((2*sigma)*sigma)),
                 r2 = (u-u_c)*(u-u_c) + (v-v_c)*(v-v_c)
  keep           e <= e_min + L,  L = log(1/tau),  e_min = min over voxels
                 (equivalent to D >= tau * max_j D, with no exp in the test)
  value          D = float32(exp(-e))

Voxel j = ix + nx*(iy + ny*iz).  Beamlets are beam-major, then m ascending,
then n ascending; a beamlet exists if the point of its square closest to the
beam axis lies within r_ptv + margin.

With coarse unspecified tissue (Section 3.1: twice the voxel size in each
dimension outside the target and organs), every aligned, complete block of
2x2x2 grid voxels that are all normal tissue is one voxel centred at
  c_a = (2*b_a + 1)*h - (n_a*h)/2                      (a = x, y, z)
of structure "normal"; the voxel order is then the remaining grid voxels
(j ascending) followed by the coarse voxels (b = bx + cx*(by + cy*bz)
ascending, cx = nx//2, cy = ny//2).  e_min stays the minimum over the full
grid (the beamlet's maximum dose at full resolution), so the voxels at the
grid spacing keep exactly the rows they have in the uniform phantom.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp

from workloads import BLADDER, NORMAL, PTV, RECTUM, PhantomSpec


def grid_centres(spec: PhantomSpec):
    """Centre coordinates (x, y, z) in mm, float64, of every grid voxel j."""
    def axis(n):
        i = np.arange(n, dtype=np.float64)
        return (i + 0.5) * spec.h - (n * spec.h) / 2.0
    ax, ay, az = axis(spec.nx), axis(spec.ny), axis(spec.nz)
    z, y, x = np.meshgrid(az, ay, ax, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def grid_structure_ids(spec: PhantomSpec) -> np.ndarray:
    """Structure id of every grid voxel (uint8), priority PTV > rectum > bladder > normal.

    A voxel belongs to a structure when its centre lies inside or on it:
    PTV sphere at the origin, rectum cylinder along z centred at
    (0, -(r_ptv + r_rectum)), bladder sphere centred at (0, r_ptv + r_bladder, 0).
    """
    return _structure_at(spec, *grid_centres(spec))


def coarse_blocks(spec: PhantomSpec) -> np.ndarray:
    """Indices b = bx + cx*(by + cy*bz) of the coarse voxels: the aligned,
    complete 2x2x2 blocks of grid voxels that are all normal tissue (none
    for a uniform grid)."""
    if not spec.coarse_normal:
        return np.zeros(0, dtype=np.int64)
    cx, cy, cz = spec.nx // 2, spec.ny // 2, spec.nz // 2
    sid = grid_structure_ids(spec).reshape(spec.nz, spec.ny, spec.nx)
    sub = sid[:2 * cz, :2 * cy, :2 * cx].reshape(cz, 2, cy, 2, cx, 2)
    normal = np.all(sub == NORMAL, axis=(1, 3, 5))
    return np.nonzero(normal.ravel())[0].astype(np.int64)


def block_axes(spec: PhantomSpec, blocks: np.ndarray):
    """(bx, by, bz) of coarse block indices."""
    cx, cy = spec.nx // 2, spec.ny // 2
    return blocks % cx, (blocks // cx) % cy, blocks // (cx * cy)


def voxel_layout(spec: PhantomSpec):
    """(fine, blocks): grid indices of the voxels kept at the grid spacing
    (ascending) and the coarse voxels' block indices (ascending).  The
    voxel order of D is fine first, then blocks."""
    n = spec.grid_voxels
    blocks = coarse_blocks(spec)
    if len(blocks) == 0:
        return np.arange(n, dtype=np.int64), blocks
    bx, by, bz = block_axes(spec, blocks)
    covered = np.zeros(n, dtype=bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                covered[(2 * bx + dx) + spec.nx * ((2 * by + dy) + spec.ny * (2 * bz + dz))] = True
    return np.nonzero(~covered)[0].astype(np.int64), blocks


def coarse_centres(spec: PhantomSpec, blocks: np.ndarray):
    """Centres (x, y, z) of coarse voxels: c_a = (2 b_a + 1) h - (n_a h)/2."""
    bx, by, bz = block_axes(spec, blocks)

    def axis(b, n):
        return (2.0 * b.astype(np.float64) + 1.0) * spec.h - (n * spec.h) / 2.0
    return axis(bx, spec.nx), axis(by, spec.ny), axis(bz, spec.nz)


def voxel_count(spec: PhantomSpec) -> int:
    """Rows of D: grid voxels, or fine plus coarse voxels of a coarse layout."""
    fine, blocks = voxel_layout(spec)
    return len(fine) + len(blocks)


def voxel_centres(spec: PhantomSpec):
    """Centre coordinates (x, y, z) in mm, float64, of every voxel in D's row
    order (the grid's voxels for a uniform grid)."""
    x, y, z = grid_centres(spec)
    fine, blocks = voxel_layout(spec)
    if len(blocks) == 0:
        return x, y, z
    cx, cy, cz = coarse_centres(spec, blocks)
    return (np.concatenate([x[fine], cx]), np.concatenate([y[fine], cy]), np.concatenate([z[fine], cz]))


def structure_ids(spec: PhantomSpec) -> np.ndarray:
    """Structure id of every voxel of D's row order (uint8): the grid voxel's
    own for voxels at the grid spacing, normal tissue for coarse voxels."""
    fine, blocks = voxel_layout(spec)
    sid = grid_structure_ids(spec)
    if len(blocks) == 0:
        return sid
    return np.concatenate([sid[fine], np.full(len(blocks), NORMAL, dtype=np.uint8)])


def _structure_at(spec: PhantomSpec, x, y, z) -> np.ndarray:
    sid = np.full(x.shape, NORMAL, dtype=np.uint8)
    cb = spec.r_ptv + spec.r_bladder
    dyb = y - cb
    in_bladder = (x * x + dyb * dyb) + z * z <= spec.r_bladder * spec.r_bladder
    cr = -(spec.r_ptv + spec.r_rectum)
    dyr = y - cr
    in_rectum = x * x + dyr * dyr <= spec.r_rectum * spec.r_rectum
    in_ptv = (x * x + y * y) + z * z <= spec.r_ptv * spec.r_ptv
    sid[in_bladder] = BLADDER
    sid[in_rectum] = RECTUM
    sid[in_ptv] = PTV
    return sid


@dataclass
class Beamlet:
    beam: int
    m: int
    n: int
    u_c: float
    v_c: float


def beam_directions(spec: PhantomSpec):
    """(cos, sin) of each beam angle 2*pi*b/B, via the host math library."""
    out = []
    for b in range(spec.n_beams):
        theta = (2.0 * math.pi * b) / spec.n_beams
        out.append((math.cos(theta), math.sin(theta)))
    return out


def beamlets(spec: PhantomSpec) -> List[Beamlet]:
    """Beamlets covering the PTV projection plus the margin, in column order."""
    w = spec.beamlet
    reach = spec.r_ptv + spec.margin
    kmax = int(math.ceil(reach / w)) + 1
    out = []
    for b in range(spec.n_beams):
        for m in range(-kmax, kmax):
            lo_u, hi_u = m * w, (m + 1) * w
            cu = min(max(0.0, lo_u), hi_u)
            for n in range(-kmax, kmax):
                lo_v, hi_v = n * w, (n + 1) * w
                cv = min(max(0.0, lo_v), hi_v)
                if cu * cu + cv * cv <= reach * reach:
                    out.append(Beamlet(b, m, n, (m + 0.5) * w, (n + 0.5) * w))
    return out


def beam_depth_and_u(spec: PhantomSpec, x, y, cos_t: float, sin_t: float):
    """Depth below the box entry point along the beam, and the lateral u."""
    hx, hy = (spec.nx * spec.h) / 2.0, (spec.ny * spec.h) / 2.0
    ts = []
    if cos_t != 0.0:
        ts.append(np.minimum((-hx - x) / cos_t, (hx - x) / cos_t))
    if sin_t != 0.0:
        ts.append(np.minimum((-hy - y) / sin_t, (hy - y) / sin_t))
    t_entry = ts[0] if len(ts) == 1 else np.maximum(ts[0], ts[1])
    depth = -t_entry
    u = (-sin_t) * x + cos_t * y
    return depth, u


def beamlet_exponent(spec: PhantomSpec, depth, u, z, bl: Beamlet):
    """Exponent e = mu*depth + r^2/(2 sigma^2) of one beamlet at every voxel."""
    du = u - bl.u_c
    dv = z - bl.v_c
    r2 = du * du + dv * dv
    return (spec.mu * depth) + (r2 / ((2.0 * spec.sigma) * spec.sigma))


@dataclass
class DoseMatrix:
    """D (nv x nb) as scipy CSR and CSC, float32 values, int32 indices."""
    nv: int
    nb: int
    csr: sp.csr_matrix
    csc: sp.csc_matrix
    struct_id: np.ndarray
    beamlets: List[Beamlet]

    @property
    def nnz(self) -> int:
        return int(self.csr.nnz)


def kept_entries(spec: PhantomSpec, e: np.ndarray, emin: float):
    """Kept voxel indices (ascending) and float32 values of one beamlet, from
    its exponents e at the voxels and its minimum emin over the grid."""
    keep_limit = emin + math.log(1.0 / spec.tau)
    rows = np.nonzero(e <= keep_limit)[0].astype(np.int32)
    vals = np.exp(-e[rows]).astype(np.float32)
    return rows, vals


def build_columns(spec: PhantomSpec, which=None):
    """Columns of D for the beamlet indices ``which`` (all when None).

    Returns (list of beamlets, list of (rows, vals)) in the requested order.
    The exponents are evaluated on the whole grid (for e_min); a coarse
    layout keeps its fine voxels' values and adds the coarse voxels'.
    """
    bls = beamlets(spec)
    dirs = beam_directions(spec)
    x, y, z = grid_centres(spec)
    fine, blocks = voxel_layout(spec)
    coarse = len(blocks) > 0
    if coarse:
        xc, yc, zc = coarse_centres(spec, blocks)
    idx = range(len(bls)) if which is None else which
    cache = {}
    cols = []
    for i in idx:
        bl = bls[i]
        if bl.beam not in cache:
            cache.clear()
            cache[bl.beam] = (beam_depth_and_u(spec, x, y, *dirs[bl.beam]),
                              beam_depth_and_u(spec, xc, yc, *dirs[bl.beam]) if coarse else None)
        (depth, u), cdu = cache[bl.beam]
        e = beamlet_exponent(spec, depth, u, z, bl)
        emin = e.min()
        if coarse:
            e = np.concatenate([e[fine], beamlet_exponent(spec, cdu[0], cdu[1], zc, bl)])
        cols.append(kept_entries(spec, e, emin))
    return bls, cols


def _columns_of_beam(args):
    spec, beam = args
    bls = beamlets(spec)
    which = [i for i, b in enumerate(bls) if b.beam == beam]
    return build_columns(spec, which)[1]


def build_dose_matrix(spec: PhantomSpec, workers: int = 1) -> DoseMatrix:
    """Brute-force D for the whole phantom, in CSC then CSR (indices sorted).

    ``workers`` > 1 evaluates the beams in separate processes; each column is
    computed by the same code either way.  The workers are fresh interpreters
    (the "spawn" start method), never forks: a fork of a process that holds a
    GPU runtime can inherit a lock held by one of its threads and never
    finish, so the pool must not copy the caller's state.
    """
    if workers > 1 and spec.n_beams > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(min(workers, spec.n_beams)) as pool:
            per_beam = pool.map(_columns_of_beam, [(spec, b) for b in range(spec.n_beams)])
        bls = beamlets(spec)
        cols = [c for group in per_beam for c in group]
    else:
        bls, cols = build_columns(spec)
    nv, nb = voxel_count(spec), len(bls)
    lens = np.array([len(r) for r, _ in cols], dtype=np.int64)
    col_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(lens, out=col_ptr[1:])
    row_idx = np.concatenate([r for r, _ in cols]) if nb else np.zeros(0, np.int32)
    vals = np.concatenate([v for _, v in cols]) if nb else np.zeros(0, np.float32)
    csc = sp.csc_matrix((vals, row_idx, col_ptr), shape=(nv, nb))
    csc.has_sorted_indices = True
    csr = csc.tocsr()
    csr.sort_indices()
    return DoseMatrix(nv, nb, csr, csc, structure_ids(spec), bls)


def column_minima(spec: PhantomSpec, workers: int = 1) -> np.ndarray:
    """e_min of every beamlet (float64), by brute force over all grid voxels."""
    bls = beamlets(spec)
    dirs = beam_directions(spec)
    x, y, z = grid_centres(spec)
    out = np.empty(len(bls))
    cache = {}
    for i, bl in enumerate(bls):
        if bl.beam not in cache:
            cache.clear()
            cache[bl.beam] = beam_depth_and_u(spec, x, y, *dirs[bl.beam])
        depth, u = cache[bl.beam]
        out[i] = beamlet_exponent(spec, depth, u, z, bl).min()
    return out


def dose_rows(spec: PhantomSpec, rows, emin: np.ndarray):
    """Rows of D (kept beamlet indices ascending, float32 values) for the voxel
    indices ``rows`` (D's row order), given every beamlet's e_min over the
    grid; same formulas as the columns."""
    bls = beamlets(spec)
    dirs = beam_directions(spec)
    x, y, z = voxel_centres(spec)
    rows = np.asarray(rows, dtype=np.int64)
    xs, ys, zs = x[rows], y[rows], z[rows]
    L = math.log(1.0 / spec.tau)
    out = []
    per_beam = [beam_depth_and_u(spec, xs, ys, *dirs[b]) for b in range(spec.n_beams)]
    e = np.empty((len(rows), len(bls)))
    for i, bl in enumerate(bls):
        depth, u = per_beam[bl.beam]
        e[:, i] = beamlet_exponent(spec, depth, u, zs, bl)
    for r in range(len(rows)):
        keep = np.nonzero(e[r] <= emin + L)[0].astype(np.int32)
        out.append((keep, np.exp(-e[r, keep]).astype(np.float32)))
    return out
