"""FP64 oracle: the fluence-map model of Section 2.1 and its derivatives.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.

Every function is a plain float64 evaluation of a definition:

  dose        z = D x                                     (Section 2.1)
  penalties   F_j = w_u*min(z_j - T_u,j, 0)^2 + w_o*max(z_j - T_o,j, 0)^2
              -- Eq. (1) with per-voxel weights and separate under/over
              thresholds; the paper's model is w = 1, T_u = T_o = T_j with the
              under-dose term only on target voxels.  The paper joins the two
              one-sided terms with a union sign; for T_u <= T_o at most one is
              non-zero, so the union is their sum.
  objective   G(x) = sum_j F_j((D x)_j)                   (Eqs. (2)-(4))
  gradient    grad G(x) = 2 D^T r,  r_j = w_u*min(z_j - T_u,j, 0)
                                         + w_o*max(z_j - T_o,j, 0)
              -- the paper names the gradient but prints no formula; this is
              the derivative of the squared one-sided terms.
  projection  P(y) = argmin_{x >= 0} ||y - x|| = max(0, y) (Section 2.2)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class VoxelPenalties:
    """Per-voxel penalty parameters (float64 arrays of length nv)."""
    T_under: np.ndarray
    T_over: np.ndarray
    w_under: np.ndarray
    w_over: np.ndarray

    @staticmethod
    def from_structures(struct_id: np.ndarray, table: np.ndarray) -> "VoxelPenalties":
        """Expand a (nstruct, 4) [T_u, T_o, w_u, w_o] table over structure ids."""
        t = np.asarray(table, dtype=np.float64)[np.asarray(struct_id, dtype=np.int64)]
        return VoxelPenalties(t[:, 0].copy(), t[:, 1].copy(), t[:, 2].copy(), t[:, 3].copy())

    def with_targets(self, T_under: np.ndarray, T_over: np.ndarray) -> "VoxelPenalties":
        """Same weights, per-voxel thresholds (the paper's T_j of an original plan)."""
        return VoxelPenalties(np.asarray(T_under, np.float64), np.asarray(T_over, np.float64),
                              self.w_under, self.w_over)


def as_f64_matrix(D):
    """D with its float32 values promoted exactly to float64."""
    return D.astype(np.float64)


def dose(D, x: np.ndarray) -> np.ndarray:
    """Voxel dose z_j = sum_i D_ij x_i."""
    return as_f64_matrix(D) @ np.asarray(x, dtype=np.float64)


def under_over(z: np.ndarray, pen: VoxelPenalties):
    """The two one-sided deviations min(z - T_u, 0) and max(z - T_o, 0)."""
    return np.minimum(z - pen.T_under, 0.0), np.maximum(z - pen.T_over, 0.0)


def voxel_objective(z: np.ndarray, pen: VoxelPenalties) -> np.ndarray:
    """F_j(z_j) for every voxel."""
    under, over = under_over(z, pen)
    return pen.w_under * under * under + pen.w_over * over * over


def objective_from_dose(z: np.ndarray, pen: VoxelPenalties) -> float:
    """G = sum over voxels of F_j(z_j)."""
    return float(np.sum(voxel_objective(z, pen)))


def objective(D, x: np.ndarray, pen: VoxelPenalties) -> float:
    """G(x) = sum_j F_j((D x)_j)."""
    return objective_from_dose(dose(D, x), pen)


def residual(z: np.ndarray, pen: VoxelPenalties) -> np.ndarray:
    """r_j = w_u*min(z_j - T_u, 0) + w_o*max(z_j - T_o, 0) = F_j'(z_j) / 2."""
    under, over = under_over(z, pen)
    return pen.w_under * under + pen.w_over * over


def adjoint(D, r: np.ndarray) -> np.ndarray:
    """D^T r."""
    return as_f64_matrix(D).T @ np.asarray(r, dtype=np.float64)


def gradient_from_dose(D, z: np.ndarray, pen: VoxelPenalties) -> np.ndarray:
    """grad G = 2 D^T r(z)."""
    return 2.0 * adjoint(D, residual(z, pen))


def gradient(D, x: np.ndarray, pen: VoxelPenalties) -> np.ndarray:
    """grad G(x) = 2 D^T r(D x)."""
    return gradient_from_dose(D, dose(D, x), pen)


def project(y: np.ndarray) -> np.ndarray:
    """Projection onto the nonnegative orthant, max(0, y)."""
    return np.maximum(0.0, np.asarray(y, dtype=np.float64))
