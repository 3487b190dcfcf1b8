"""GPU dose-matrix builder against the oracle's brute-force phantom:
bit-exact structure ids and sparsity (CSR and CSC), values within one
float32 ulp."""
import numpy as np
import pytest

from gpu_util import banner, f32_ulp_diff
from oracle import phantom
from workloads import SMALL, TINY, PhantomSpec, draw_batch_instance

pytestmark = pytest.mark.gpu

# radii that are not exact binary fractions make the decisions inexact
ODD = PhantomSpec(name="odd_29x23x17_4mm_7field", nx=29, ny=23, nz=17, h=4.0, r_ptv=17.3,
                  r_rectum=6.9, r_bladder=12.97, n_beams=7, beamlet=5.0, sigma=3.0, tau=0.005, seed=9)
# a batch-style draw on the coarse 5 mm box
BATCH5 = next(s for s in (draw_batch_instance(k) for k in range(100, 200)) if s.h == 5.0)


@pytest.fixture(scope="module", params=[1, 0], ids=["voxel_tiles", "grid_order"])
def ctx(request):
    """Rows of D held in 4x4x2 voxel tiles (default) or in grid order; the
    exported arrays are in grid order either way."""
    from paper_0908_4421_amd.imrt import Context
    return Context(0, voxel_tiles=request.param)


@pytest.mark.parametrize("spec", [TINY, SMALL, ODD, BATCH5], ids=lambda s: s.name)
def test_builder_matches_oracle(ctx, spec):
    from paper_0908_4421_amd.imrt import Dose
    banner(f"phantom {spec.name}")
    want = phantom.build_dose_matrix(spec)
    lib = Dose.from_geometry(ctx, spec)
    assert (lib.nv, lib.nb, lib.nnz) == (want.nv, want.nb, want.nnz)
    ex = lib.export(structures=True)
    assert np.array_equal(ex["struct_id"], want.struct_id)
    assert np.array_equal(ex["row_ptr"], want.csr.indptr)
    assert np.array_equal(ex["col_idx"], want.csr.indices)
    assert np.array_equal(ex["col_ptr"], want.csc.indptr)
    assert np.array_equal(ex["row_idx"], want.csc.indices)
    assert f32_ulp_diff(ex["val"], want.csr.data) <= 1
    assert f32_ulp_diff(ex["cval"], want.csc.data) <= 1
    # the library's two layouts hold identical values
    import scipy.sparse as sp
    C = sp.csr_matrix((ex["val"], ex["col_idx"], ex["row_ptr"]), shape=(lib.nv, lib.nb)).tocsc()
    C.sort_indices()
    assert np.array_equal(C.data, ex["cval"])


def test_products_in_grid_order(ctx):
    """D x and D^T r of a built phantom take and return voxel arrays in grid
    order, whatever the internal row order."""
    from gpu_util import to_dev, to_host
    from oracle import model
    from paper_0908_4421_amd.imrt import Dose
    want = phantom.build_dose_matrix(SMALL)
    lib = Dose.from_geometry(ctx, SMALL)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 2.0, want.nb).astype(np.float32)
    r = rng.standard_normal(want.nv).astype(np.float32)
    d = to_host(lib.apply(to_dev(x)))
    y = to_host(lib.apply_transpose(to_dev(r)))
    d_ref = model.dose(want.csr, x.astype(np.float64))
    y_ref = model.adjoint(want.csr, r.astype(np.float64))
    assert np.all(np.abs(d - d_ref) <= 1e-5 * np.abs(d_ref) + 1e-30)
    scale = abs(want.csr).T.astype(np.float64) @ np.abs(r.astype(np.float64))
    assert np.all(np.abs(y - y_ref) <= 1e-6 * scale + 1e-30)


def test_invalid_geometry_rejected(ctx):
    from paper_0908_4421_amd import imrt
    g = imrt.geometry_of(TINY)
    g.tau = 0.0
    with pytest.raises(imrt.ImrtError) as e:
        imrt.imrt_build_dose_matrix(ctx.handle, g)
    assert e.value.code == imrt.IMRT_EINVAL
    g = imrt.geometry_of(TINY)
    g.nx = 0
    with pytest.raises(imrt.ImrtError):
        imrt.imrt_build_dose_matrix(ctx.handle, g)
    with pytest.raises(imrt.ImrtError) as e:
        imrt.imrt_build_dose_matrix(ctx.handle, imrt.geometry_of(TINY), 3)   # no such storage
    assert e.value.code == imrt.IMRT_EINVAL
