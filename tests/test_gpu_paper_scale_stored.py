"""Paper-scale phantom with D stored as bfloat16 / binary16 codes, in the
launch configuration the benchmark times, against the oracle's stored
fingerprint and trajectories (tests/golden/paper_scale_stored_oracle.json,
written by make_paper_scale_stored_fixture.py from the oracle alone)."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_util import banner, check_trajectory, to_dev, to_host
from oracle import phantom, quantize
from workloads import PAPER_SCALE, PAPER_SCALE_SETTINGS, penalty_table, power_start_vector, start_point

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def fx():
    with open(os.path.join(HERE, "golden", "paper_scale_stored_oracle.json")) as f:
        stored = json.load(f)
    with open(os.path.join(HERE, "golden", "paper_scale_oracle.json")) as f:
        plain = json.load(f)
    return stored, plain


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_stored_paper_scale_against_oracle(ctx, fx, fmt):
    from paper_0908_4421_amd.imrt import Dose, Plan
    import torch
    stored, plain = fx
    ref = stored["forms"][fmt]
    banner(f"paper-scale {fmt} build")
    dose = Dose.from_geometry(ctx, PAPER_SCALE, storage=fmt)
    assert (dose.nv, dose.nb, dose.nnz) == (stored["nv"], stored["nb"], stored["nnz"])
    codes = dose.export_codes()
    # scales and codes bit-exact (hashes of the oracle's arrays)
    assert sha(codes["col_scale"], "<f4") == ref["sha256_scale"]
    assert sha(codes["val_code"], "<u2") == ref["sha256_q_csr"]
    assert sha(codes["cval_code"], "<u2") == ref["sha256_q_csc"]
    plan = Plan(ctx, dose)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(PAPER_SCALE))
    st = PAPER_SCALE_SETTINGS
    lam, sig = plan.lambda0(to_dev(power_start_vector(dose.nb, PAPER_SCALE.seed).astype(np.float32)),
                            st.power_iters)
    assert lam == ref["lambda0"] and abs(sig - ref["sigma"]) <= 1e-5 * ref["sigma"]
    banner(f"paper-scale {fmt} solve")
    x = to_dev(start_point(dose.nb, st).astype(np.float32))
    res, tr = plan.solve(x, eps=st.eps, alpha=st.alpha, lambda0=lam, delta=st.delta, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks, trace=True)
    assert res.status == 0
    # every iteration and the final G at the GPU's own stop index against the
    # oracle run on D~ (stored 40 iterations past its stop)
    worst, K, Ko = check_trajectory(tr, res, ref["trace"], ref["G_initial"], ref["iterations"], delta=st.delta)
    banner(f"paper-scale {fmt}: stop {K} (oracle {Ko}), worst G error {worst:.2e}")
    # dose at sampled voxels against the oracle's rows of D~ (float32 values of
    # the oracle's rows, coded with the scales just proven equal to the oracle's)
    d = torch.empty(dose.nv, dtype=torch.float32, device="cuda")
    assert plan.objective(x, d) == res.G_final
    d = to_host(d)
    xg = to_host(x).astype(np.float64)
    s = codes["col_scale"].astype(np.float64)
    ex = dose.export()
    lens = np.diff(ex["row_ptr"])
    rng = np.random.default_rng(17)
    rows = rng.choice(np.nonzero(lens > 0)[0], 200, replace=False)
    err = 0.0
    for j, (c, v) in zip(rows, phantom.dose_rows(PAPER_SCALE, rows, np.array(plain["emin"]))):
        q = quantize.round_to_format(v.astype(np.float64) / s[c], fmt)
        z = float((s[c] * q) @ xg[c])
        err = max(err, abs(d[j] - z) / max(abs(z), 1e-30))
    assert err <= 1e-5
    # the stated error of the stored form: its final G against the float32
    # oracle's final G (printed; bounded by the code's precision)
    G32 = plain["trace"][plain["iterations"] - 1][4]
    banner(f"paper-scale {fmt}: {res.iterations} iterations, G {res.G_final:.9g} vs float32 oracle {G32:.9g} "
           f"({abs(res.G_final - G32) / G32:.2e} relative)")
    p, _ = quantize.FORMATS[fmt]
    assert abs(res.G_final - G32) / G32 <= 2.0 ** -p
