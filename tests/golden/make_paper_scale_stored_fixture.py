"""Write the oracle's fingerprint and Armijo trajectory of the paper-scale
phantom with D stored as bfloat16 and as binary16 codes with per-beamlet
scales (tests/golden/paper_scale_stored_oracle.json).

Calls only the FP64 oracle and the workload specification.  Run from the
repository root:  python tests/golden/make_paper_scale_stored_fixture.py
(a few minutes on one core per format plus the parallel matrix build).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import model, phantom, quantize, solver  # noqa: E402
from workloads import PAPER_SCALE, PAPER_SCALE_SETTINGS, penalty_table, power_start_vector, start_point  # noqa: E402


EXTRA = 40   # iterations stored beyond the oracle's stop


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def main():
    spec, st = PAPER_SCALE, PAPER_SCALE_SETTINGS
    t0 = time.time()
    D = phantom.build_dose_matrix(spec, workers=9)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(spec))
    out = {"workload": spec.name, "nv": D.nv, "nb": D.nb, "nnz": D.nnz, "forms": {}}
    for fmt in ("bf16", "f16"):
        S = quantize.store(D.csr, fmt)
        lam0, sigma = solver.lambda0_from_power_iteration(S.Dq, pen, power_start_vector(D.nb, spec.seed),
                                                          st.power_iters)
        res = solver.solve(S.Dq, pen, start_point(D.nb, st), eps=st.eps, alpha=st.alpha, lambda0=lam0,
                           delta=st.delta, max_iter=st.max_iter, max_backtracks=st.max_backtracks,
                           fixed_iters=st.fixed_iters)
        # continued past the stop (stopping test off), for runs that stop later
        ext = solver.solve(S.Dq, pen, start_point(D.nb, st), eps=st.eps, alpha=st.alpha, lambda0=lam0,
                           max_iter=res.iterations + EXTRA, max_backtracks=st.max_backtracks, fixed_iters=True)
        assert [e.G for e in ext.trace[:res.iterations]] == [e.G for e in res.trace]
        out["forms"][fmt] = {
            "sha256_scale": sha(S.scale, "<f4"),
            "sha256_q_csr": sha(S.q_csr, "<u2"),
            "sha256_q_csc": sha(S.q_csc, "<u2"),
            "lambda0": lam0, "sigma": sigma,
            "G_initial": res.G_initial, "status": res.status, "iterations": res.iterations,
            "trace": [[e.k, e.lam, e.backtracks, e.step_sq, e.G] for e in ext.trace],
        }
        print(fmt, res.iterations, res.G, time.time() - t0, flush=True)
    out["seconds"] = time.time() - t0
    with open(os.path.join(HERE, "paper_scale_stored_oracle.json"), "w") as f:
        json.dump(out, f)
    print("wrote paper_scale_stored_oracle.json", time.time() - t0)


if __name__ == "__main__":
    main()
