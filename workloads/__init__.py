"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only describes workloads: phantom geometry parameters, penalty
tables, solver settings and seeded random draws (batch geometries, start
vectors, random sparse test matrices).  It holds none of the optimisation
method's arithmetic: no dose, objective, gradient, projection or line search,
and no dose-deposition kernel.  Both the FP64 oracle and the HIP library read
the same specification and build their inputs independently.

The clinical prostate case of the paper (Section 3.1, Table 1) is not public;
the phantoms below are prostate-shaped stand-ins with the paper's shape
features: nine (or five) coplanar equispaced fields, 5x5 mm (or 10x10 mm)
beamlets, 2.5 mm (or 4/5 mm) voxels, a spherical target with a posterior
rectum and an anterior bladder.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

# Structure ids used in every phantom (uint8 per voxel).
NORMAL, PTV, RECTUM, BLADDER = 0, 1, 2, 3
STRUCTURE_NAMES = ("normal", "ptv", "rectum", "bladder")


@dataclass(frozen=True)
class Penalty:
    """One-sided quadratic penalty parameters of one structure (Eq. (1)).

    Under-dose term weight ``w_under`` below ``T_under``; over-dose term
    weight ``w_over`` above ``T_over``.  The paper's model is the special case
    w = 1 and T_under = T_over = T_j, with no under-dose term off-target.
    """
    T_under: float
    T_over: float
    w_under: float
    w_over: float


# Penalties of the prostate-shaped phantoms: target 70 Gy with under/over
# weights 1.0/0.5; rectum above 40 Gy (0.3); bladder above 45 Gy (0.2);
# normal tissue above 30 Gy (0.05).  Indexed by structure id.
PROSTATE_PENALTIES: Tuple[Penalty, ...] = (
    Penalty(0.0, 30.0, 0.0, 0.05),   # normal
    Penalty(70.0, 70.0, 1.0, 0.5),   # PTV
    Penalty(0.0, 40.0, 0.0, 0.3),    # rectum
    Penalty(0.0, 45.0, 0.0, 0.2),    # bladder
)


@dataclass(frozen=True)
class PhantomSpec:
    """Geometry of a water box phantom with coplanar parallel pencil beams.

    Voxel grid ``nx*ny*nz`` at spacing ``h`` mm, centred on the isocentre.
    Structures: PTV sphere of radius ``r_ptv`` at the origin; rectum cylinder
    along z of radius ``r_rectum`` tangent to the PTV at -y; bladder sphere of
    radius ``r_bladder`` tangent to the PTV at +y.  ``n_beams`` coplanar beams
    at angles 2*pi*b/n_beams; square beamlets of side ``beamlet`` mm cover the
    PTV projection plus ``margin`` mm.  Dose kernel exp(-(mu*depth + r^2 /
    (2 sigma^2))), truncated below ``tau`` times the beamlet maximum.

    ``coarse_normal``: unspecified tissue at twice the voxel size in each
    dimension (Section 3.1).  Every aligned, complete 2x2x2 block of grid
    voxels that are all normal tissue becomes one voxel of side 2h at the
    block's centre; the other voxels keep the grid spacing.  The voxel count
    then depends on the structures, which each phantom builder evaluates
    itself, so ``nv`` is defined for uniform grids only.
    """
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    r_ptv: float
    r_rectum: float
    r_bladder: float
    n_beams: int
    beamlet: float
    sigma: float
    tau: float
    mu: float = 0.005
    margin: float = 5.0
    penalties: Tuple[Penalty, ...] = PROSTATE_PENALTIES
    seed: int = 0
    coarse_normal: bool = False

    @property
    def grid_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nv(self) -> int:
        if self.coarse_normal:
            raise ValueError(f"{self.name}: the voxel count of a layout with coarse unspecified tissue "
                             "comes from its phantom builder")
        return self.grid_voxels

    def as_dict(self) -> dict:
        d = dataclasses.asdict(self)
        d["penalties"] = [dataclasses.asdict(p) for p in self.penalties]
        return d


@dataclass(frozen=True)
class SolveSettings:
    """Armijo gradient-projection settings (Section 2.2).

    ``eps`` and ``alpha`` are the two Armijo parameters (0 < eps < 1,
    alpha > 1); ``delta`` the relative-change stopping tolerance;
    ``fixed_iters`` runs exactly ``max_iter`` accepted iterations with the
    stopping test off.
    """
    eps: float = 1e-4
    alpha: float = 2.0
    delta: float = 1e-5
    max_iter: int = 20000
    max_backtracks: int = 60
    fixed_iters: bool = False
    x0: float = 1.0
    power_iters: int = 50


# Tiny phantom: 40x40x20 voxels at 5 mm, 5 beams at 0/72/144/216/288 deg,
# 10 mm beamlets, sigma 4 mm, 1 % truncation; 200 fixed iterations.
TINY = PhantomSpec(name="tiny_40x40x20_5mm_5field", nx=40, ny=40, nz=20, h=5.0,
                   r_ptv=20.0, r_rectum=8.0, r_bladder=15.0, n_beams=5,
                   beamlet=10.0, sigma=4.0, tau=0.01, seed=0)
TINY_SETTINGS = SolveSettings(max_iter=200, fixed_iters=True)

# Paper-scale single plan: 160x104x80 voxels at 2.5 mm (400x260x200 mm box),
# 9 equispaced fields, 5 mm beamlets, sigma 3 mm, 0.5 % truncation, structures
# scaled by 1.75 to prostate dimensions; run to relative change < 1e-5.
PAPER_SCALE = PhantomSpec(name="prostate_160x104x80_2.5mm_9field", nx=160, ny=104, nz=80,
                          h=2.5, r_ptv=35.0, r_rectum=14.0, r_bladder=26.25, n_beams=9,
                          beamlet=5.0, sigma=3.0, tau=0.005, seed=1)
PAPER_SCALE_SETTINGS = SolveSettings(delta=1e-5, max_iter=20000)

# A small ragged case used by parity tests: several row blocks and column
# chunks, odd sizes, two beam families.
SMALL = PhantomSpec(name="small_33x27x11_4mm_7field", nx=33, ny=27, nz=11, h=4.0,
                    r_ptv=15.0, r_rectum=6.0, r_bladder=11.25, n_beams=7,
                    beamlet=5.0, sigma=3.0, tau=0.005, seed=2)

# The shape of the paper's largest scenario (Table 1, scenario 3: 9 fields,
# 5 mm beamlets, 6,453 beamlets, 143,329 voxels, 43.3 M nonzeros, about 300
# per voxel) on a uniform 4 mm grid with wide beamlet kernels: 6,444
# beamlets, 142,560 voxels, about 41 M nonzeros.  Its CSR and CSC (about
# 0.6 GB) exceed the 256 MB last-level cache, so its passes stream from HBM.
SCENARIO3_SHAPE = PhantomSpec(name="scenario3_shape_66x54x40_4mm_9field", nx=66, ny=54, nz=40, h=4.0,
                              r_ptv=67.0, r_rectum=26.8, r_bladder=50.25, n_beams=9, beamlet=5.0,
                              sigma=7.5, tau=0.005, seed=4)

# A small phantom with the same wide kernels (rows of up to 656 nonzeros,
# most columns reaching a sixth of the voxels) for parity tests.
WIDE = PhantomSpec(name="wide_30x26x16_4mm_9field", nx=30, ny=26, nz=16, h=4.0, r_ptv=40.0,
                   r_rectum=16.0, r_bladder=30.0, n_beams=9, beamlet=5.0, sigma=7.5, tau=0.005, seed=5)

# The same phantoms with unspecified tissue at twice the voxel size (the
# paper's reduction of the problem size, Section 3.1).  SMALL's odd grid
# leaves incomplete blocks at its upper faces, which keep the grid spacing.
TINY_COARSE = dataclasses.replace(TINY, name="tiny_40x40x20_5mm_5field_coarse", coarse_normal=True)
SMALL_COARSE = dataclasses.replace(SMALL, name="small_33x27x11_4mm_7field_coarse", coarse_normal=True)
PAPER_SCALE_COARSE = dataclasses.replace(PAPER_SCALE, name="prostate_160x104x80_2.5mm_9field_coarse",
                                         coarse_normal=True)

NAMED = {"tiny": TINY, "paper": PAPER_SCALE, "small": SMALL, "scenario3": SCENARIO3_SHAPE,
         "paper_coarse": PAPER_SCALE_COARSE}

# Fixed box of the batched / served instances (mm) and the grids it gives.
_BOX_GRIDS = {2.5: (160, 104, 80), 4.0: (100, 65, 50), 5.0: (80, 52, 40)}


def draw_batch_instance(seed: int) -> PhantomSpec:
    """Random uneven re-plan geometry drawn from ``seed``.

    Draw order with ``numpy.random.default_rng(seed)``: beam count from
    {5, 7, 9}; beamlet size from {5, 10} mm; voxel size from {2.5, 4, 5} mm;
    PTV radius uniform in [15, 30) mm.  Organs at risk scale with
    r_ptv / 20 from the tiny phantom's 8 mm rectum and 15 mm bladder.  5 mm
    beamlets use sigma 3 mm and 0.5 % truncation, 10 mm beamlets sigma 4 mm
    and 1 %.
    """
    rng = np.random.default_rng(seed)
    n_beams = int(rng.choice([5, 7, 9]))
    beamlet = float(rng.choice([5.0, 10.0]))
    h = float(rng.choice([2.5, 4.0, 5.0]))
    r_ptv = float(rng.uniform(15.0, 30.0))
    nx, ny, nz = _BOX_GRIDS[h]
    sigma, tau = (3.0, 0.005) if beamlet == 5.0 else (4.0, 0.01)
    scale = r_ptv / 20.0
    return PhantomSpec(name=f"batch_seed{seed}", nx=nx, ny=ny, nz=nz, h=h, r_ptv=r_ptv,
                       r_rectum=8.0 * scale, r_bladder=15.0 * scale, n_beams=n_beams,
                       beamlet=beamlet, sigma=sigma, tau=tau, seed=seed)


def batch_instances(first_seed: int = 100, count: int = 32) -> List[PhantomSpec]:
    """The batched re-plan workload: ``count`` instances, seeds first_seed.. ."""
    return [draw_batch_instance(first_seed + i) for i in range(count)]


def replan_penalty_table(spec: PhantomSpec, rng: np.random.Generator) -> np.ndarray:
    """New thresholds for a re-plan of a resident patient: the PTV's under- and
    overdose thresholds both drawn uniform in [66, 74) Gy, each other
    structure's overdose threshold scaled by a factor uniform in [0.9, 1.1)."""
    t = penalty_table(spec).copy()
    t[PTV, 0] = t[PTV, 1] = rng.uniform(66.0, 74.0)
    others = [s for s in range(len(t)) if s != PTV]     # rows are structure ids
    t[others, 1] *= rng.uniform(0.9, 1.1, len(others))
    return t


@dataclass
class ServedRequest:
    """One request of the served re-plan workload."""
    arrival_s: float           # seconds after the start of the stream
    patient: int
    spec: PhantomSpec          # the patient's geometry (seed 1000 + first request index)
    table: np.ndarray          # (nstruct, 4) penalties
    replan: bool               # True: a resident patient with new thresholds


def served_requests(rate: float, count: int, seed: int = 0, reuse: float = 0.3) -> List[ServedRequest]:
    """Poisson stream of ``count`` requests at ``rate`` per second.

    Request i is, with probability ``reuse`` (once a patient exists), a re-plan
    of an earlier request's patient chosen uniformly with thresholds from
    ``replan_penalty_table``; otherwise a new patient whose geometry is
    ``draw_batch_instance(1000 + i)`` with the standard penalties.  One
    generator ``default_rng(seed)`` draws, per request in order: the
    exponential gap, the reuse coin, then the patient choice and thresholds.
    """
    rng = np.random.default_rng(seed)
    out: List[ServedRequest] = []
    patients: List[Tuple[int, PhantomSpec]] = []
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        if patients and rng.random() < reuse:
            pid, spec = patients[int(rng.integers(len(patients)))]
            out.append(ServedRequest(t, pid, spec, replan_penalty_table(spec, rng), True))
        else:
            spec = draw_batch_instance(1000 + i)
            patients.append((i, spec))
            out.append(ServedRequest(t, i, spec, penalty_table(spec), False))
    return out


def day_geometry(spec: PhantomSpec, ptv_scale: float = 0.95, rectum_scale: float = 0.9,
                 bladder_scale: float = 1.2) -> PhantomSpec:
    """The patient's anatomy on a treatment day, for re-optimisation towards
    the original plan's dose: the target shrinks and the bladder fills (its
    radius grows), the rectum empties; the organs stay in contact with the
    target, so they move with it.  Same grid, beams and beamlet model; the
    beamlets are those covering the new target."""
    return dataclasses.replace(spec, name=f"{spec.name}_day", r_ptv=spec.r_ptv * ptv_scale,
                               r_rectum=spec.r_rectum * rectum_scale,
                               r_bladder=spec.r_bladder * bladder_scale)


def power_start_vector(nb: int, seed: int) -> np.ndarray:
    """Seeded positive start vector (float64) for the step-size power iteration."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, size=nb)


def start_point(nb: int, settings: SolveSettings) -> np.ndarray:
    """The initial fluence x_1 (all beamlets at ``settings.x0``)."""
    return np.full(nb, settings.x0, dtype=np.float64)


def penalty_table(spec_or_penalties) -> np.ndarray:
    """(nstruct, 4) float64 table [T_under, T_over, w_under, w_over]."""
    pens = spec_or_penalties.penalties if isinstance(spec_or_penalties, PhantomSpec) else spec_or_penalties
    return np.array([[p.T_under, p.T_over, p.w_under, p.w_over] for p in pens], dtype=np.float64)


@dataclass
class RandomCSR:
    """A random nonnegative sparse matrix in CSR form (float32 values)."""
    nv: int
    nb: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    struct_id: np.ndarray = field(default=None)


def random_csr(nv: int, nb: int, mean_row: float, seed: int, empty_frac: float = 0.3,
               long_rows: int = 0, long_len: int = 0, nstruct: int = 4) -> RandomCSR:
    """Seeded random CSR test matrix with ragged rows.

    A fraction ``empty_frac`` of rows is empty; the other row lengths are
    geometric with mean ``mean_row`` (capped at nb); ``long_rows`` rows get
    ``long_len`` entries.  Columns are distinct and ascending within a row;
    values are float32 in (0, 1].  Structure ids are uniform in [0, nstruct).
    """
    rng = np.random.default_rng(seed)
    lens = rng.geometric(1.0 / max(mean_row, 1.0), size=nv)
    lens = np.minimum(lens, nb)
    lens[rng.random(nv) < empty_frac] = 0
    if long_rows:
        idx = rng.choice(nv, size=min(long_rows, nv), replace=False)
        lens[idx] = min(long_len, nb)
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    cols = np.empty(int(row_ptr[-1]), dtype=np.int32)
    for j in range(nv):
        n = int(lens[j])
        if n:
            cols[row_ptr[j]:row_ptr[j + 1]] = np.sort(rng.choice(nb, size=n, replace=False))
    val = (1.0 - rng.random(int(row_ptr[-1]))).astype(np.float32)
    sid = rng.integers(0, nstruct, size=nv).astype(np.uint8)
    return RandomCSR(nv, nb, row_ptr.astype(np.int32), cols, val, sid)


def random_penalties(nstruct: int, seed: int, scale: float = 1.0) -> Tuple[Penalty, ...]:
    """Seeded penalty table with mixed one- and two-sided structures."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(nstruct):
        tu = float(rng.uniform(0.2, 1.0) * scale)
        to = tu + float(rng.uniform(0.0, 0.5) * scale)
        wu = float(rng.uniform(0.5, 2.0)) if s % 2 == 1 else 0.0
        wo = float(rng.uniform(0.05, 1.0))
        out.append(Penalty(tu, to, wu, wo))
    return tuple(out)
