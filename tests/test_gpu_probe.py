"""The read-bandwidth probe (a measurement aid beside the roofline): a rate
below the HBM peak for a buffer beyond the last-level cache, the buffer left
unchanged, and its argument checks."""
import pytest

from gpu_util import banner

pytestmark = pytest.mark.gpu


def test_read_probe():
    import torch

    from paper_0908_4421_amd import imrt
    from paper_0908_4421_amd.imrt import Context, imrt_read_probe
    ctx = Context(0)
    buf = torch.ones((1 << 30) // 4, dtype=torch.float32, device="cuda")
    gbs = imrt_read_probe(ctx.handle, buf.data_ptr(), buf.numel() * 4, 3)
    banner(f"read probe over 1 GiB: {gbs:.0f} GB/s")
    assert 500.0 < gbs < 8000.0
    assert bool((buf == 1.0).all())
    for ptr, n, reps in ((buf.data_ptr() + 4, 1 << 20, 1), (buf.data_ptr(), 8, 1), (buf.data_ptr(), 1 << 20, 0)):
        with pytest.raises(imrt.ImrtError) as e:
            imrt_read_probe(ctx.handle, ptr, n, reps)
        assert e.value.code == imrt.IMRT_EINVAL
