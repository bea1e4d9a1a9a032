"""Pins of the FP64 reference of the warm-start network (oracle/unet.py):
convolutions against loops written from their definitions, the wiring of the
skip connections and of the down / up path against networks whose output is
known in closed form, and the gradient against central differences."""
import numpy as np
import pytest
import torch

from oracle import unet as U

BASE = 16


def flat_weight(rng, taps, cin, cout):
    return rng.standard_normal(taps * cin * cout)


def test_param_count():
    # 3x3x3: 27 cin cout + cout; 2x2x2: 8 cin cout + cout; head 16 + 1
    assert U.n_params(BASE) == 1780129


def test_conv3_matches_loops():
    rng = np.random.default_rng(1)
    cin, cout, D, H, W = 3, 2, 4, 5, 3
    wf = flat_weight(rng, 27, cin, cout)
    b = rng.standard_normal(cout)
    x = rng.standard_normal((1, cin, D, H, W))
    got = U.conv3(torch.tensor(x), U.layer_weight(torch.tensor(wf), "conv3", cin, cout), torch.tensor(b)).numpy()
    Wt = wf.reshape(27, cin, cout)
    ref = np.zeros((1, cout, D, H, W))
    for co in range(cout):
        for z in range(D):
            for y in range(H):
                for xx in range(W):
                    s = b[co]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, x2 = z + dz, y + dy, xx + dx
                                if not (0 <= zz < D and 0 <= yy < H and 0 <= x2 < W):
                                    continue
                                t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                                s += sum(Wt[t, ci, co] * x[0, ci, zz, yy, x2] for ci in range(cin))
                    ref[0, co, z, y, xx] = s
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_down_matches_loops():
    rng = np.random.default_rng(2)
    cin, cout, D, H, W = 2, 3, 4, 6, 2
    wf = flat_weight(rng, 8, cin, cout)
    b = rng.standard_normal(cout)
    x = rng.standard_normal((1, cin, D, H, W))
    got = U.down(torch.tensor(x), U.layer_weight(torch.tensor(wf), "down", cin, cout), torch.tensor(b)).numpy()
    Wt = wf.reshape(8, cin, cout)
    ref = np.zeros((1, cout, D // 2, H // 2, W // 2))
    for co in range(cout):
        for z in range(D // 2):
            for y in range(H // 2):
                for xx in range(W // 2):
                    s = b[co]
                    for t in range(8):
                        pz, py, px = t >> 2, (t >> 1) & 1, t & 1
                        s += sum(Wt[t, ci, co] * x[0, ci, 2 * z + pz, 2 * y + py, 2 * xx + px] for ci in range(cin))
                    ref[0, co, z, y, xx] = s
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_up_matches_loops():
    rng = np.random.default_rng(3)
    cin, cout, D, H, W = 3, 2, 2, 3, 2
    wf = flat_weight(rng, 8, cin, cout)
    b = rng.standard_normal(cout)
    x = rng.standard_normal((1, cin, D, H, W))
    got = U.up(torch.tensor(x), U.layer_weight(torch.tensor(wf), "up", cin, cout), torch.tensor(b)).numpy()
    Wt = wf.reshape(8, cin, cout)
    ref = np.zeros((1, cout, 2 * D, 2 * H, 2 * W))
    for co in range(cout):
        for z in range(D):
            for y in range(H):
                for xx in range(W):
                    for t in range(8):
                        pz, py, px = t >> 2, (t >> 1) & 1, t & 1
                        ref[0, co, 2 * z + pz, 2 * y + py, 2 * xx + px] = b[co] + sum(
                            Wt[t, ci, co] * x[0, ci, z, y, xx] for ci in range(cin))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


class Builder:
    """Flat parameter vector with selected entries set."""

    def __init__(self):
        self.t = U.layer_table(BASE)
        self.off = []
        o = 0
        for kind, cin, cout in self.t:
            self.off.append(o)
            o += (27 if kind == "conv3" else 8) * cin * cout + cout
        self.head = o
        self.p = np.zeros(U.n_params(BASE))

    def w(self, layer, tap, ci, co, v):
        kind, cin, cout = self.t[layer]
        self.p[self.off[layer] + (tap * cin + ci) * cout + co] = v

    def centre(self, layer, ci=0, co=0):
        self.w(layer, 13, ci, co, 1.0)


def test_skip_connection_order():
    # only the level-0 skip carries the input: relu(x) through layers 0, 1,
    # the skip half (channels 16..31) of the concatenating layer 18, layer 19
    b = Builder()
    b.centre(0)
    b.centre(1)
    b.centre(18, ci=16)
    b.centre(19)
    b.p[b.head] = 1.0
    b.p[b.head + BASE] = 0.5
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 8, 8, 8))
    y = U.forward_np(b.p, x)
    np.testing.assert_allclose(y, np.maximum(x, 0) + 0.5, rtol=0, atol=1e-14)


def test_down_up_path():
    # level-1 path: mean of each 2x2x2 block of relu(x) (layer 2), identity
    # through 3, 4, the skip half of 15 and 16, copied to the 8 children by
    # the up layer 17 and taken from the upsampled half of 18
    b = Builder()
    b.centre(0)
    b.centre(1)
    for t in range(8):
        b.w(2, t, 0, 0, 1.0 / 8)
        b.w(17, t, 0, 0, 1.0)
    b.centre(3)
    b.centre(4)
    b.centre(15, ci=32)
    b.centre(16)
    b.centre(18, ci=0)
    b.centre(19)
    b.p[b.head] = 1.0
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 8, 16, 8))
    y = U.forward_np(b.p, x)
    r = np.maximum(x, 0)
    m = r.reshape(2, 4, 2, 8, 2, 4, 2).mean(axis=(2, 4, 6))
    ref = m.repeat(2, 1).repeat(2, 2).repeat(2, 3)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-14)


def test_gradient_central_differences():
    rng = np.random.default_rng(6)
    n = U.n_params(BASE)
    p = rng.standard_normal(n) * 0.05
    x = rng.standard_normal((1, 8, 8, 8))
    tg = rng.standard_normal((1, 8, 8, 8))
    loss, g, _ = U.loss_and_grad(p, x, tg)

    def L(q):
        with torch.no_grad():
            y = U.forward(torch.tensor(q), torch.tensor(x))
            return float(((y - torch.tensor(tg)) ** 2).mean())

    assert abs(L(p) - loss) < 1e-15 * max(1.0, loss)
    # unit directions (the gradient's own and two random ones); a step of
    # 1e-4 balances the truncation error against cancellation in the loss
    eps = 1e-4
    dirs = [g / np.linalg.norm(g)] + [rng.standard_normal(n) for _ in range(2)]
    for v in dirs:
        v = v / np.linalg.norm(v)
        fd = (L(p + eps * v) - L(p - eps * v)) / (2 * eps)
        assert fd == pytest.approx(float(g @ v), rel=1e-4, abs=1e-12)


def test_bf16_emulation_rounds_only_storage():
    # with weights and inputs exactly representable in bf16 and a linear
    # path of exact products, the emulated and the plain forward agree
    b = Builder()
    b.centre(0)
    b.centre(1)
    b.centre(18, ci=16)
    b.centre(19)
    b.p[b.head] = 1.0
    x = np.arange(-256, 256, dtype=np.float64).reshape(1, 8, 8, 8) / 64.0
    np.testing.assert_array_equal(U.forward_np(b.p, x, bf16=True), U.forward_np(b.p, x, bf16=False))
    # and an input off the bf16 grid is rounded to nearest even
    x2 = np.full((1, 8, 8, 8), 1.0 + 2.0 ** -8)  # halfway between 1 and 1 + 2^-7
    assert np.all(U.forward_np(b.p, x2, bf16=True) == 1.0)


def test_gradient_rounding_option():
    # rounding the back-propagated gradient changes the weight gradients by
    # about the bf16 resolution and leaves the bias gradients of the last
    # layer (which see the unrounded gradient) unchanged
    rng = np.random.default_rng(7)
    n = U.n_params(BASE)
    p = rng.standard_normal(n) * 0.05
    x = rng.standard_normal((1, 8, 8, 8))
    tg = rng.standard_normal((1, 8, 8, 8))
    l0, g0, _ = U.loss_and_grad(p, x, tg, bf16=True)
    l1, g1, _ = U.loss_and_grad(p, x, tg, bf16=True, bf16_grad=True)
    assert l0 == l1
    rel = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    assert 0 < rel < 2e-2
    t = U.layer_table(BASE)
    nlast = 27 * t[-1][1] * t[-1][2]
    last_b = slice(n - 17 - t[-1][2], n - 17)
    np.testing.assert_array_equal(g1[last_b], g0[last_b])
    assert nlast > 0
