"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, sizes its work memory and rejects invalid arguments before
touching a device."""
import ctypes as C
import os
import re

import pytest

torch = pytest.importorskip("torch")

from paper_2402_08404_amd import pic, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b((?:pic|unet)_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol():
    names = _declared()
    assert {"pic_init", "pic_inject", "pic_step", "pic_solve_poisson", "pic_moments", "pic_destroy",
            "pic_rz_init", "pic_rz_step", "pic_rz_solve", "unet_forward"} <= set(names)
    L = pic.lib()
    for n in names:
        assert hasattr(L, n), n


def test_scratch_size_scales():
    c, keep = pic.make_config(W.tiny())
    a = pic.pic_scratch_size(c, (1000, 1000, 1000))
    b = pic.pic_scratch_size(c, (100000, 1000, 1000))
    assert 0 < a < b
    c2, keep2 = pic.make_config(W.tiny(), precision=pic.PIC_F32)
    assert pic.pic_scratch_size(c2, (100000, 1000, 1000)) < b


@pytest.mark.parametrize("field,value", [("nx", 3), ("dt", 0.0), ("h", -1.0), ("tip_r", 0.0), ("precision", 7),
                                         ("xs_n", 1), ("step_maxit", 0), ("tip_h", 1e-6)])
def test_invalid_config_rejected(field, value):
    c, keep = pic.make_config(W.tiny())
    setattr(c, field, value)
    n = C.c_size_t()
    assert pic.lib().pic_scratch_size(C.byref(c), (C.c_int64 * 3)(10, 10, 10), C.byref(n)) == -1
    b = pic.pic_buffers()
    ctx = C.c_void_p()
    assert pic.lib().pic_init(C.byref(c), C.byref(b), None, C.byref(ctx)) == -1
    assert not ctx.value
    assert pic.pic_last_error(None) != ""


def test_null_buffers_rejected():
    c, keep = pic.make_config(W.tiny())
    b = pic.pic_buffers()
    b.cap[0] = 10
    ctx = C.c_void_p()
    assert pic.lib().pic_init(C.byref(c), C.byref(b), None, C.byref(ctx)) == -1
    assert pic.lib().pic_step(None, 1, pic.STEP_PUSH) == -1
    assert pic.lib().pic_moments(None, None) == -1
