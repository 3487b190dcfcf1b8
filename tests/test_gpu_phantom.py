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


@pytest.fixture(scope="module")
def ctx():
    from paper_0908_4421_amd.imrt import Context
    return Context(0)


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
        imrt.imrt_build_dose_matrix(ctx.handle, imrt.geometry_of(TINY), imrt.IMRT_BF16)
    assert e.value.code == imrt.IMRT_EUNSUPPORTED
