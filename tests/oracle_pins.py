"""Shared checkers used by the oracle pin tests and by the planted-mistake tests.

Each checker measures the oracle against a reference that does not come from
the oracle itself (finite differences, dense linear algebra, exact rational
arithmetic, hand-worked numbers, library solvers).
"""
import os

import numpy as np
import scipy.sparse as sp

from oracle import model, solver

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line or "=" not in line:
                continue
            key, val = (s.strip() for s in line.split("=", 1))
            out[key] = val
    return out


def floats(s):
    return np.array([float(t) for t in s.split()], dtype=np.float64)


def worked_example():
    g = read_golden("worked_example_armijo.txt")
    nr, nc = int(g["D_rows"]), int(g["D_cols"])
    D = sp.csr_matrix(floats(g["D"]).reshape(nr, nc).astype(np.float32))
    pen = model.VoxelPenalties(floats(g["T_under"]), floats(g["T_over"]),
                               floats(g["w_under"]), floats(g["w_over"]))
    return g, D, pen


def fd_gradient_error(D, pen, x, coords, rel_h=1e-5):
    """max_i |central FD_i - grad_i| / ||grad||_inf over coordinates whose
    +-h step moves no voxel dose across a penalty threshold (where G is an
    exact quadratic along the coordinate, so central differences are exact up
    to rounding)."""
    Dd = D.toarray().astype(np.float64) if sp.issparse(D) else np.asarray(D, np.float64)
    g = model.gradient(D, x, pen)
    z = Dd @ x
    scale = max(np.max(np.abs(g)), 1e-300)
    worst, used = 0.0, 0
    for i in coords:
        h = rel_h * (1.0 + abs(x[i]))
        col = Dd[:, i]
        nz = col != 0
        reach = h * col[nz]
        if np.any(np.abs(z[nz] - pen.T_under[nz]) <= reach) or np.any(np.abs(z[nz] - pen.T_over[nz]) <= reach):
            continue
        xp = x.copy(); xp[i] += h
        xm = x.copy(); xm[i] -= h
        fd = (model.objective(D, xp, pen) - model.objective(D, xm, pen)) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / scale)
        used += 1
    return worst, used


def armijo_trace_errors(D, pen, x1, res, eps, alpha, lambda0):
    """Replay a solve: return a list of violations of the Armijo rule
    (each accepted lambda = lambda0 alpha^-m, every smaller m fails the test,
    the accepted one passes, G strictly decreases)."""
    bad = []
    x = np.asarray(x1, np.float64)
    G = model.objective(D, x, pen)
    for e in res.trace:
        g = model.gradient(D, x, pen)
        lam = lambda0
        for m in range(e.backtracks + 1):
            xt = np.maximum(0.0, x - lam * g)
            s = float(np.sum((xt - x) ** 2))
            Gt = model.objective(D, xt, pen)
            C = G - (eps / lam) * s
            if m < e.backtracks and Gt < C:
                bad.append((e.k, m, "smaller backtrack count would pass"))
            if m == e.backtracks:
                if not Gt < C:
                    bad.append((e.k, m, "accepted trial fails"))
                if lam != e.lam:
                    bad.append((e.k, m, "lambda mismatch"))
            if m < e.backtracks:
                lam = lam / alpha
        if not e.G < G:
            bad.append((e.k, -1, "G not decreasing"))
        x, G = xt, Gt
    return bad


def kkt_closed_form_errors():
    """The projected-gradient residual |x - max(0, x - grad G(x))| of one-voxel,
    one-beamlet problems against its value worked by hand.

    With D = [d], G(x) = w_u min(dx - T_u, 0)^2 + w_o max(dx - T_o, 0)^2 and
    grad G = 2 d r.  Cases (d, T_u, T_o, w_u, w_o, x, residual):
      under-dosed at 0: r = -2, g = -4, max(0, 4) = 4          -> 4
      over-dosed at 3:  r = 1,  g = 2,  max(0, 1) = 1          -> 2
      over-only at 0.5: g = 2 * 0.5 = 1, max(0, -0.5) = 0      -> 0.5
      inside [T_u, T_o] at 2.5 (d = 2: dose 5 in [4, 6]): g = 0 -> 0
      d = 0.5, two-sided T = 1, w = 2, x = 1: dose 0.5, r = -1,
      g = -1, max(0, 2) = 2                                    -> 1
    Returns the cases whose residual differs by more than 1e-15."""
    cases = [(1.0, 2.0, 2.0, 1.0, 1.0, 0.0, 4.0),
             (1.0, 2.0, 2.0, 1.0, 1.0, 3.0, 2.0),
             (1.0, 0.0, 0.0, 0.0, 1.0, 0.5, 0.5),
             (2.0, 4.0, 6.0, 1.0, 1.0, 2.5, 0.0),
             (0.5, 1.0, 1.0, 2.0, 2.0, 1.0, 1.0)]
    bad = []
    for d, Tu, To, wu, wo, x, want in cases:
        D = sp.csr_matrix(np.array([[d]], np.float32))
        pen = model.VoxelPenalties(np.array([Tu]), np.array([To]), np.array([wu]), np.array([wo]))
        got = solver.kkt_residual(D, pen, np.array([x]))
        if abs(got - want) > 1e-15:
            bad.append((d, Tu, To, wu, wo, x, got, want))
    return bad
