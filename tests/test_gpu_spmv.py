"""GPU parity of the two sparse products (forward CSR, adjoint CSC) against the
FP64 oracle, on seeded ragged matrices that span many row blocks and column
chunks, with empty rows/columns, long rows and tiny edge shapes."""
import numpy as np
import pytest

from gpu_util import banner, csr_of, to_dev, to_host
from oracle import model
from workloads import random_csr

pytestmark = pytest.mark.gpu

CASES = {
    # name: (nv, nb, mean_row, seed, empty_frac, long_rows, long_len)
    "ragged": (5003, 211, 12.0, 1, 0.5, 0, 0),
    "long_rows": (700, 6000, 8.0, 2, 0.2, 4, 4500),   # rows beyond one LDS block
    "short_rows": (9000, 40, 1.0, 3, 0.4, 0, 0),      # blocks capped by the row limit
    "dense_cols": (3000, 7, 5.0, 4, 0.0, 0, 0),       # long columns, several chunks each
    "single": (1, 1, 1.0, 5, 0.0, 0, 0),
    "one_row": (1, 300, 200.0, 6, 0.0, 0, 0),
    "one_col": (4097, 1, 1.0, 7, 0.3, 0, 0),
    # thousands of mostly empty columns per adjoint workgroup: its column
    # bounds are reloaded 64 at a time many times over
    "many_cols": (2000, 20000, 3.0, 8, 0.3, 0, 0),
}


@pytest.fixture(scope="module", params=[(1024, 1, 1), (16, 0, 1), (1024, 1, 0)],
                ids=["default", "shared_cols_block_fwd", "col32_wave_fwd"])
def ctx(request):
    """Default launch settings, or many short adjoint workgroup ranges (most
    columns shared by several workgroups) with workgroup-wide forward blocks,
    or the wave forward over 32-bit column indices."""
    from paper_0908_4421_amd.imrt import Context
    min_nnz, wave, col16 = request.param
    return Context(0, adj_min_nnz=min_nnz, fwd_wave=wave, fwd_col16=col16)


def _dose(ctx, A):
    from paper_0908_4421_amd.imrt import Dose
    return Dose.from_csr(ctx, A.nv, A.nb, A.row_ptr, A.col_idx, A.val)


@pytest.mark.parametrize("name", list(CASES))
def test_forward_and_adjoint_match_oracle(ctx, name):
    nv, nb, mean, seed, empty, nlong, llen = CASES[name]
    banner(f"spmv {name} nv={nv} nb={nb}")
    A = random_csr(nv, nb, mean, seed, empty_frac=empty, long_rows=nlong, long_len=llen)
    D = csr_of(A)
    lib = _dose(ctx, A)
    assert (lib.nv, lib.nb, lib.nnz) == (nv, nb, D.nnz)
    rng = np.random.default_rng(seed + 100)
    x = rng.uniform(0.0, 2.0, nb).astype(np.float32)
    r = rng.standard_normal(nv).astype(np.float32)
    d = to_host(lib.apply(to_dev(x)))
    y = to_host(lib.apply_transpose(to_dev(r)))
    d_ref = model.dose(D, x.astype(np.float64))
    y_ref = model.adjoint(D, r.astype(np.float64))
    # forward: all terms are nonnegative, so an elementwise relative bound holds
    assert np.all(np.abs(d - d_ref) <= 1e-5 * np.abs(d_ref) + 1e-30)
    # adjoint: mixed signs; bound by the sum of absolute products
    Dabs = abs(D).astype(np.float64)
    scale = Dabs.T @ np.abs(r.astype(np.float64))
    assert np.all(np.abs(y - y_ref) <= 1e-6 * scale + 1e-30)
    # repeated products are bit-identical (fixed-order reductions)
    d2 = to_host(lib.apply(to_dev(x)))
    y2 = to_host(lib.apply_transpose(to_dev(r)))
    assert np.array_equal(d, d2) and np.array_equal(y, y2)


def test_export_round_trip_and_transpose(ctx):
    A = random_csr(2500, 97, 9.0, 11, empty_frac=0.3)
    lib = _dose(ctx, A)
    ex = lib.export()
    D = csr_of(A)
    assert np.array_equal(ex["row_ptr"], A.row_ptr)
    assert np.array_equal(ex["col_idx"], A.col_idx)
    assert np.array_equal(ex["val"], A.val)
    C = D.tocsc()
    C.sort_indices()
    assert np.array_equal(ex["col_ptr"], C.indptr)
    assert np.array_equal(ex["row_idx"], C.indices)
    assert np.array_equal(ex["cval"], C.data)


def test_empty_matrix(ctx):
    from paper_0908_4421_amd.imrt import Dose
    rp = np.zeros(6, np.int32)
    lib = Dose.from_csr(ctx, 5, 3, rp, np.zeros(0, np.int32), np.zeros(0, np.float32))
    d = to_host(lib.apply(to_dev(np.ones(3, np.float32))))
    y = to_host(lib.apply_transpose(to_dev(np.ones(5, np.float32))))
    assert np.all(d == 0) and np.all(y == 0)


def test_invalid_csr_rejected(ctx):
    from paper_0908_4421_amd import imrt
    rp = np.array([0, 2, 3], np.int32)
    bad_cols = [np.array([1, 1, 0], np.int32),     # not strictly increasing
                np.array([0, 5, 0], np.int32)]     # out of range
    for ci in bad_cols:
        with pytest.raises(imrt.ImrtError) as e:
            imrt.imrt_dose_from_csr(ctx.handle, 2, 3, 3, rp, ci, np.ones(3, np.float32))
        assert e.value.code == imrt.IMRT_EINVAL
    with pytest.raises(imrt.ImrtError) as e:
        imrt.imrt_dose_from_csr(ctx.handle, 2, 3, 3, rp, np.array([0, 1, 2], np.int32),
                                np.array([1, -1, 1], np.float32))
    assert e.value.code == imrt.IMRT_EINVAL


def test_context_options(ctx):
    from paper_0908_4421_amd import imrt
    assert ctx.get_option("adj_min_nnz") in (1024, 16)
    for bad in (("no_such_option", 1), ("fwd_wave", 2), ("adj_min_nnz", 3), ("fwd_wg_per_cu", 0)):
        with pytest.raises(imrt.ImrtError) as e:
            ctx.set_option(*bad)
        assert e.value.code == imrt.IMRT_EINVAL


def test_beamlets_beyond_the_staging_limit(ctx):
    """x is staged in LDS: a matrix with more beamlets than fit is built and
    exported, but its forward product reports IMRT_EUNSUPPORTED; its adjoint
    product needs no staging and still matches the oracle."""
    from paper_0908_4421_amd import imrt
    A = random_csr(3000, 70000, 10.0, 8, empty_frac=0.3)
    lib = _dose(ctx, A)
    assert np.array_equal(lib.export()["col_idx"], A.col_idx)
    with pytest.raises(imrt.ImrtError) as e:
        lib.apply(to_dev(np.ones(A.nb, np.float32)))
    assert e.value.code == imrt.IMRT_EUNSUPPORTED
    r = np.random.default_rng(3).standard_normal(A.nv).astype(np.float32)
    y = to_host(lib.apply_transpose(to_dev(r)))
    D = csr_of(A)
    y_ref = model.adjoint(D, r.astype(np.float64))
    assert np.all(np.abs(y - y_ref) <= 1e-6 * (abs(D).T @ np.abs(r.astype(np.float64))) + 1e-30)
