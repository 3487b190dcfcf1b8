"""Write the oracle's fingerprint of the paper-scale phantom and its full
Armijo trajectory (tests/golden/paper_scale_oracle.json; with --coarse, of
the same phantom with unspecified tissue at twice the voxel size, to
tests/golden/paper_scale_coarse_oracle.json).

Calls only the FP64 oracle and the workload specification.  Run from the
repository root:  python tests/golden/make_paper_scale_fixture.py [--coarse]
(about two minutes on one core plus the parallel matrix build).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import model, phantom, solver  # noqa: E402
from workloads import (PAPER_SCALE, PAPER_SCALE_COARSE, PAPER_SCALE_SETTINGS, penalty_table,  # noqa: E402
                       power_start_vector, start_point)


EXTRA = 40   # iterations stored beyond the oracle's stop


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def main():
    coarse = "--coarse" in sys.argv[1:]
    spec, st = (PAPER_SCALE_COARSE if coarse else PAPER_SCALE), PAPER_SCALE_SETTINGS
    name = "paper_scale_coarse_oracle.json" if coarse else "paper_scale_oracle.json"
    t0 = time.time()
    D = phantom.build_dose_matrix(spec, workers=9)
    emin = phantom.column_minima(spec)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(spec))
    lam0, sigma = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, spec.seed),
                                                      st.power_iters)
    res = solver.solve(D.csr, pen, start_point(D.nb, st), eps=st.eps, alpha=st.alpha, lambda0=lam0,
                       delta=st.delta, max_iter=st.max_iter, max_backtracks=st.max_backtracks,
                       fixed_iters=st.fixed_iters)
    # the same trajectory continued past the stop, so that a run which stops
    # a little later can be compared at its own stop index
    ext = solver.solve(D.csr, pen, start_point(D.nb, st), eps=st.eps, alpha=st.alpha, lambda0=lam0,
                       max_iter=res.iterations + EXTRA, max_backtracks=st.max_backtracks, fixed_iters=True)
    assert [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in ext.trace[:res.iterations]] == \
        [(e.k, e.lam, e.backtracks, e.step_sq, e.G) for e in res.trace]
    out = {
        "workload": spec.name,
        "nv": D.nv, "nb": D.nb, "nnz": D.nnz,
        "sha256_row_ptr": sha(D.csr.indptr, "<i4"), "sha256_col_idx": sha(D.csr.indices, "<i4"),
        "sha256_col_ptr": sha(D.csc.indptr, "<i4"), "sha256_row_idx": sha(D.csc.indices, "<i4"),
        "sha256_struct_id": sha(D.struct_id, "u1"),
        "val_sum": float(D.csr.data.astype(np.float64).sum()),
        "val_sumsq": float((D.csr.data.astype(np.float64) ** 2).sum()),
        "col_counts": np.diff(D.csc.indptr).astype(int).tolist(),
        "emin": emin.tolist(),
        "lambda0": lam0, "sigma": sigma,
        "G_initial": res.G_initial, "status": res.status, "iterations": res.iterations,
        "trace": [[e.k, e.lam, e.backtracks, e.step_sq, e.G] for e in ext.trace],
        "trace_note": f"the stopped trajectory's {res.iterations} iterations, then {EXTRA} more (stopping test off)",
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)
    print("wrote", name, res.iterations, res.G, time.time() - t0)


if __name__ == "__main__":
    main()
