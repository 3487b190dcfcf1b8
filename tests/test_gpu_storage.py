"""16-bit storage of D (bfloat16 / binary16 codes with per-beamlet scales) on
the GPU against the FP64 oracle: the codes and scales bit-exact, both sparse
products and the full solve against the oracle run on the dequantised matrix
D~ = s q, and the error of the stored form against the float32 D stated."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import banner, csr_of, rel_normwise, to_dev, to_host
from oracle import model, phantom, quantize, solver
from workloads import (PAPER_SCALE, TINY, TINY_SETTINGS, penalty_table, power_start_vector, random_csr)

pytestmark = pytest.mark.gpu

FORMATS = ["bf16", "f16"]


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


@pytest.fixture(scope="module")
def tiny_oracle():
    D = phantom.build_dose_matrix(TINY)
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(TINY))
    return D, pen


def _codes_csc_match(ex_codes, S, D):
    """The library's codes in CSC order and scales equal the oracle's."""
    assert np.array_equal(ex_codes["col_scale"], S.scale)
    assert np.array_equal(ex_codes["val_code"], S.q_csr)
    assert np.array_equal(ex_codes["cval_code"], S.q_csc)


@pytest.mark.parametrize("fmt", FORMATS)
def test_tiny_phantom_codes_bit_exact(ctx, tiny_oracle, fmt):
    from paper_0908_4421_amd.imrt import Dose
    banner(f"tiny codes {fmt}")
    D, _ = tiny_oracle
    lib = Dose.from_geometry(ctx, TINY, storage=fmt)
    S = quantize.store(D.csr, fmt)
    ex = lib.export()
    assert np.array_equal(ex["row_ptr"], D.csr.indptr) and np.array_equal(ex["col_idx"], D.csr.indices)
    _codes_csc_match(lib.export_codes(), S, D)
    # exported float32 values are the float32 rounding of s q
    assert np.array_equal(ex["val"], S.Dq.data.astype(np.float32))


@pytest.mark.parametrize("fmt", FORMATS)
def test_paper_scale_sampled_columns_codes(ctx, fmt):
    """Paper-scale phantom: scales and codes of sampled beamlets, from the
    oracle's own columns."""
    from paper_0908_4421_amd.imrt import Dose
    banner(f"paper-scale codes {fmt}")
    lib = Dose.from_geometry(ctx, PAPER_SCALE, storage=fmt)
    ex = lib.export()
    codes = lib.export_codes()
    rng = np.random.default_rng(11)
    cols = sorted(rng.choice(lib.nb, size=8, replace=False).tolist())
    _, oc = phantom.build_columns(PAPER_SCALE, cols)
    for i, (rows, vals) in zip(cols, oc):
        s = np.float32(vals.max())
        assert codes["col_scale"][i] == s
        q = quantize.to_bits(quantize.round_to_format(vals.astype(np.float64) / np.float64(s), fmt), fmt)
        a, b = ex["col_ptr"][i], ex["col_ptr"][i + 1]
        assert np.array_equal(ex["row_idx"][a:b], rows)
        assert np.array_equal(codes["cval_code"][a:b], q)


CASES = {
    # name: (nv, nb, mean_row, seed, empty_frac, long_rows, long_len)
    "ragged": (5003, 211, 12.0, 1, 0.5, 0, 0),
    "long_rows": (700, 6000, 8.0, 2, 0.2, 4, 4500),
    "dense_cols": (3000, 7, 5.0, 4, 0.0, 0, 0),
    "one_row": (1, 300, 200.0, 6, 0.0, 0, 0),
    "one_col": (4097, 1, 1.0, 7, 0.3, 0, 0),
}


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("name", list(CASES))
def test_products_against_dequantised_oracle(ctx, fmt, name):
    from paper_0908_4421_amd.imrt import Dose
    nv, nb, mean, seed, empty, nlong, llen = CASES[name]
    banner(f"16-bit products {fmt} {name}")
    A = random_csr(nv, nb, mean, seed, empty_frac=empty, long_rows=nlong, long_len=llen)
    D = csr_of(A)
    S = quantize.store(D, fmt)
    lib = Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val, storage=fmt)
    _codes_csc_match(lib.export_codes(), S, D)
    rng = np.random.default_rng(seed + 200)
    x = rng.uniform(0.0, 2.0, nb).astype(np.float32)
    r = rng.standard_normal(nv).astype(np.float32)
    d = to_host(lib.apply(to_dev(x)))
    y = to_host(lib.apply_transpose(to_dev(r)))
    d_ref = model.dose(S.Dq, x.astype(np.float64))
    y_ref = model.adjoint(S.Dq, r.astype(np.float64))
    assert np.all(np.abs(d - d_ref) <= 1e-5 * np.abs(d_ref) + 1e-30)
    scale = abs(S.Dq).T @ np.abs(r.astype(np.float64))
    assert np.all(np.abs(y - y_ref) <= 1e-6 * scale + 1e-30)
    # against the float32 D: within the code's half unit (2^-p relative per entry)
    p, _ = quantize.FORMATS[fmt]
    d32 = model.dose(D, x.astype(np.float64))
    assert np.all(np.abs(d - d32) <= (2.0 ** -p + 1e-5) * np.abs(d32) + 1e-30)


@pytest.mark.parametrize("fmt", FORMATS)
def test_tiny_phantom_solve_against_dequantised_oracle(ctx, tiny_oracle, fmt):
    """200 iterations on the tiny phantom: the Armijo trajectory (backtracks,
    steps, G) of the oracle run on D~, and the stated error against the plan
    of the float32 D."""
    from paper_0908_4421_amd.imrt import Dose, Plan
    banner(f"tiny solve {fmt}")
    D, pen = tiny_oracle
    S = quantize.store(D.csr, fmt)
    lib = Dose.from_geometry(ctx, TINY, storage=fmt)
    plan = Plan(ctx, lib)
    plan.set_structures(None, 4)
    plan.set_penalties(penalty_table(TINY))
    st = TINY_SETTINGS
    lam0, sig = solver.lambda0_from_power_iteration(S.Dq, pen, power_start_vector(D.nb, TINY.seed))
    lam_g, sig_g = plan.lambda0(to_dev(power_start_vector(D.nb, TINY.seed).astype(np.float32)), st.power_iters)
    assert lam_g == lam0 and abs(sig_g - sig) <= 1e-5 * sig
    x1 = np.ones(D.nb)
    ref = solver.solve(S.Dq, pen, x1, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                       max_backtracks=st.max_backtracks, fixed_iters=True)
    x = to_dev(x1.astype(np.float32))
    res, tr = plan.solve(x, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks, fixed_iters=True, trace=True)
    assert res.status == 1 and res.iterations == 200
    for (k, m, lam, s, G), e in zip(tr, ref.trace):
        assert k == e.k and m == e.backtracks and lam == e.lam
        assert abs(G - e.G) <= 1e-6 * e.G
    assert abs(res.G_final - ref.G) <= 1e-6 * ref.G
    # dose of the GPU plan: against D~ (parity) and against the float32 D (stated)
    import torch
    xg = to_host(x).astype(np.float64)
    dose = torch.empty(D.nv, dtype=torch.float32, device="cuda")
    G_at = plan.objective(x, dose)
    assert G_at == res.G_final
    dg = to_host(dose)
    zq = model.dose(S.Dq, xg)
    assert np.max(np.abs(dg - zq)) <= 1e-5 * np.max(np.abs(zq))
    z32 = model.dose(D.csr, xg)
    err_abs = float(np.max(np.abs(dg - z32)))
    err_rel = err_abs / float(np.max(np.abs(z32)))
    ref32 = solver.solve(D.csr, pen, x1, eps=st.eps, alpha=st.alpha, lambda0=lam0, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks, fixed_iters=True)
    G_err = abs(res.G_final - ref32.G) / ref32.G
    banner(f"tiny {fmt}: dose vs float32 D max abs {err_abs:.3e} Gy, rel {err_rel:.3e}; "
           f"G after 200 iterations vs float32 oracle {G_err:.3e} relative")
    p, _ = quantize.FORMATS[fmt]
    assert err_rel <= 2.0 ** -p


def test_storage_rejections(ctx):
    from paper_0908_4421_amd import imrt
    A = random_csr(200, 30, 4.0, 9)
    with pytest.raises(imrt.ImrtError) as e:
        imrt.imrt_dose_from_csr(ctx.handle, A.nv, A.nb, int(A.row_ptr[-1]), A.row_ptr, A.col_idx, A.val, 7)
    assert e.value.code == imrt.IMRT_EINVAL
    lib = imrt.Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)
    with pytest.raises(imrt.ImrtError) as e:
        lib.export_codes()
    assert e.value.code == imrt.IMRT_EINVAL
    # the workgroup-granular forward pass takes float32 storage only
    from paper_0908_4421_amd.imrt import Context, Dose
    c2 = Context(0, fwd_wave=0)
    lib16 = Dose.from_csr(c2, A.nv, A.nb, A.row_ptr, A.col_idx, A.val, storage="bf16")
    with pytest.raises(imrt.ImrtError) as e:
        lib16.apply(to_dev(np.ones(A.nb, np.float32)))
    assert e.value.code == imrt.IMRT_EUNSUPPORTED
