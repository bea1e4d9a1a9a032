"""pic_inject_noalloc (the emission whose work memory is the library's static
device array) against pic_inject(ctx, NULL) (the same emission in the
context's scratch): two contexts of one configuration, stepped alike, must
hold the same electrons bit for bit and the same emission tallies. The first
configuration has 17 408 patches and the second 2 176, so the second call
works in a smaller part of the array the first call left filled."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_08404_amd import pic  # noqa: E402
from paper_2402_08404_amd import workloads as W  # noqa: E402


def _twins(az, field, precision):
    cfg = W.tiny()
    cfg.apex_field = field
    cfg.fn_az = az
    a = pic.Simulation(cfg, caps=(60000, 1024, 1024), precision=precision)
    b = pic.Simulation(cfg, caps=(60000, 1024, 1024), precision=precision)
    return a, b


@pytest.mark.parametrize("precision", [pic.PIC_F64, pic.PIC_F32])
def test_noalloc_emission_equals_pic_inject(precision):
    for az, field, steps in ((512, 20e9, 4), (64, 30e9, 4)):
        print("no-alloc emission: azimuths", az, "field", field, "precision", precision, flush=True)
        a, b = _twins(az, field, precision)
        tot = 0
        for _ in range(steps):
            na = pic.pic_inject(a.ctx, None)
            nb = pic.pic_inject_noalloc(b.ctx)
            assert na == nb
            tot += na
            a.step(1, pic.STEP_ADVANCE)
            b.step(1, pic.STEP_ADVANCE)
        assert tot > 10
        ma, mb = a.moments(), b.moments()
        for k in ("injected", "fn_clamped", "next_id", "n_alive"):
            assert np.array_equal(ma[k], mb[k]), k
        assert ma["fn_expected"] == mb["fn_expected"]
        sa, sb = a.state()[0], b.state()[0]
        for k in ("x", "y", "z", "vx", "vy", "vz", "id"):
            assert np.array_equal(sa[k], sb[k]), k
        a.close()
        b.close()


def test_noalloc_emission_rejects_too_many_patches():
    """320 000 patches need more than the 1 MiB array: INVALID_ARG with a
    message, and the context stays usable."""
    cfg = W.tiny()
    cfg.fn_az = 10000
    g = pic.Simulation(cfg, caps=(1024, 1024, 1024), precision=pic.PIC_F64)
    with pytest.raises(pic.PicError) as e:
        pic.pic_inject_noalloc(g.ctx)
    assert e.value.code == -1 and "static array" in str(e.value)
    assert pic.pic_inject(g.ctx, None) >= 0
    g.close()
